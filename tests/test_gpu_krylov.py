"""The Krylov fallback of the stage solve (App. A eq. linsystem_primal and
App. B eq. linsystem_adjoint solved with restarted GMRES) on steps whose
splitting-iteration bound theta is >= 0.5, against the oracle (dense LU or
its own GMRES).  Tolerances as in the other parity tests: states and
objectives 1e-12 relative, gradients 1e-10 of the max-norm."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import random_alpha, random_pure_states, random_system  # noqa: E402

from _gpu import dev, rel_state_err, say  # noqa: E402

STATE_TOL = 1e-12
GRAD_TOL = 1e-10


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _strong(seed, nlev, NT, T, amp):
    rng = np.random.default_rng(seed)
    s = random_system(rng, nlev, NT=NT, T=T, Ns=5, Nf=2)
    return s, random_alpha(rng, s, amp=amp), rng


def _fallback_steps(lbx, plan, alpha):
    k = lbx.sweep_counts(plan, dev(alpha.reshape(-1)))[0, :, 1]
    return int((k < 1).sum()), int((k >= 1).sum())


@pytest.mark.parametrize("nlev,amp", [((2, 3), 0.35), ((3, 3, 3, 3), 0.12)])
def test_gradient_with_krylov_steps_matches_oracle(lbx, nlev, amp):
    # (2, 3) would run LDS-resident and (3, 3, 3, 3) streamed: the fallback
    # streams both; some steps keep the sweeps (bound below 0.5)
    s, alpha, rng = _strong(300 + len(nlev), nlev, NT=12, T=1.2, amp=amp)
    B = 2
    rho0 = random_pure_states(rng, s.N, B)
    tar = random_pure_states(rng, s.N, B)
    beta = rng.uniform(0.5, 2, B)
    plan = lbx.Plan([s])
    nk, ns = _fallback_steps(lbx, plan, alpha)
    say("krylov gradient", nlev, "krylov steps", nk, "sweep steps", ns)
    assert nk > 0 and ns > 0
    G, grad, rhoT = lbx.adjoint_gradient(plan, 0, dev(alpha.reshape(-1)), dev(rho0), dev(tar), dev(beta), [B],
                                         0.0, 0, want_rhoT=True)
    Gr, gr, rT = oracle.value_and_gradient(s, alpha, rho0, tar, beta, 0, return_final=True)
    assert rel_state_err([rhoT.cpu().numpy().reshape(B, s.N, s.N)], [rT]) < STATE_TOL
    assert abs(G.item() - Gr) <= 1e-12 * abs(Gr)
    assert np.max(np.abs(grad.cpu().numpy().reshape(gr.shape) - gr)) <= GRAD_TOL * np.max(np.abs(gr))


@pytest.mark.parametrize("adjoint", [False, True])
def test_imr_step_with_krylov_solve_matches_dense_solve(lbx, adjoint):
    s, alpha, rng = _strong(320, (3, 3), NT=10, T=1.0, amp=0.6)
    plan = lbx.Plan([s])
    k = lbx.sweep_counts(plan, dev(alpha.reshape(-1)))[0, :, 1]
    j = int(np.argmin(k))
    assert k[j] < 1
    q = rng.standard_normal((2, s.N, s.N)) + 1j * rng.standard_normal((2, s.N, s.N))
    say("krylov imr_step", adjoint, "step", j)
    out = lbx.imr_step(plan, 0, j, dev(alpha.reshape(-1)), dev(q), adjoint=adjoint).cpu().numpy()
    M = oracle.superoperator(s, alpha, (j + 0.5) * s.dt)
    if adjoint:
        M = M.conj().T
    A = np.eye(s.N * s.N) - 0.5 * s.dt * M
    ref = []
    for b in range(2):
        z = np.linalg.solve(A, oracle.vec(q[b]))
        ref.append(oracle.unvec(oracle.vec(q[b]) + s.dt * (M @ z), s.N))
    assert rel_state_err(out, np.stack(ref)) < STATE_TOL


def test_trajectory_of_a_krylov_forward_feeds_the_adjoint(lbx):
    """forward_solve (trajectory kept) and adjoint_backward, both in the
    fallback, give what adjoint_gradient gives."""
    s, alpha, rng = _strong(330, (2, 3), NT=12, T=1.2, amp=0.35)
    B = 2
    rho0 = dev(random_pure_states(rng, s.N, B))
    tar = dev(random_pure_states(rng, s.N, B))
    beta = dev(rng.uniform(0.5, 2, B))
    a = dev(alpha.reshape(-1))
    plan = lbx.Plan([s])
    say("krylov trajectory")
    G, grad, rT = lbx.adjoint_gradient(plan, 0, a, rho0, tar, beta, [B], 0.0, 0, want_rhoT=True)
    traj = torch.empty(plan.trajectory_bytes([B], 0), dtype=torch.uint8, device="cuda")
    rT2 = lbx.forward_solve(plan, a, rho0, [B], traj=traj, ckpt_every=0)
    g2 = lbx.adjoint_backward(plan, 0, a, traj, 0, tar, beta, [B])
    assert rel_state_err([rT2.cpu().numpy().reshape(B, s.N, s.N)], [rT.cpu().numpy().reshape(B, s.N, s.N)]) < 1e-14
    assert np.max(np.abs(g2.cpu().numpy() - grad.cpu().numpy())) <= 1e-13 * np.max(np.abs(grad.cpu().numpy()))


def test_asynchronous_call_reports_the_bound(lbx):
    s, alpha, rng = _strong(340, (2, 3), NT=12, T=1.2, amp=0.35)
    plan = lbx.Plan([s])
    plan.set_option(lbx._native.LB_OPT_SYNC, 0)
    B = 1
    rho0 = dev(random_pure_states(rng, s.N, B))
    ws_batch = [B]
    say("krylov async status")
    out = lbx.forward_solve(plan, dev(alpha.reshape(-1)), rho0, ws_batch)
    with pytest.raises(lbx._native.LbxError) as e:
        plan.status(plan.workspace(lbx._native.LB_OP_FORWARD, ws_batch, 1))
    assert e.value.code == lbx._native.LB_EUNSUPPORTED
    del out
