"""Jaynes-Cummings coupling (Sec. II, general form with unequal rotation
frequencies) on the GPU against the oracle: the apply against the dense
superoperator, one implicit-midpoint step against a dense solve, and
gradients on the LDS-resident and streamed paths, a mixed batch and the
GMRES fallback.  Tolerances as in the other parity tests."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import random_alpha, random_pure_states, random_system  # noqa: E402

from _gpu import dev, flat_alpha, flat_states, rel_state_err, say, split_states  # noqa: E402

STATE_TOL = 1e-12
GRAD_TOL = 1e-10


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _jc(seed, nlev, NT=12, T=1.2, jc=0.03, amp=0.02):
    rng = np.random.default_rng(seed)
    s = random_system(rng, nlev, NT=NT, T=T, Ns=5, Nf=2, jc=jc)
    return s, random_alpha(rng, s, amp=amp), rng


@pytest.mark.parametrize("nlev", [(2, 3), (3, 2, 2), (2, 2, 2, 2), (4, 3)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_coupled_apply_matches_dense_superoperator(lbx, nlev, adjoint):
    s, alpha, rng = _jc(600 + sum(nlev) + 13 * len(nlev), nlev)
    assert s.jc is not None and np.count_nonzero(s.jc) > 0
    N = s.N
    x = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    t = 0.83
    say("coupled apply", nlev, adjoint)
    y = lbx.lindblad_apply(lbx.Plan([s]), 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    M = oracle.superoperator(s, alpha, t)
    if adjoint:
        M = M.conj().T
    ref = np.stack([oracle.unvec(M @ oracle.vec(x[b]), N) for b in range(2)])
    assert rel_state_err(y, ref) < 1e-13


@pytest.mark.parametrize("adjoint", [False, True])
def test_coupled_imr_step_matches_dense_solve(lbx, adjoint):
    s, alpha, rng = _jc(620, (3, 3), NT=10, T=1.0)
    q = rng.standard_normal((2, s.N, s.N)) + 1j * rng.standard_normal((2, s.N, s.N))
    j = 7
    say("coupled imr_step", adjoint)
    out = lbx.imr_step(lbx.Plan([s]), 0, j, dev(alpha.reshape(-1)), dev(q), adjoint=adjoint).cpu().numpy()
    M = oracle.superoperator(s, alpha, (j + 0.5) * s.dt)
    if adjoint:
        M = M.conj().T
    A = np.eye(s.N * s.N) - 0.5 * s.dt * M
    ref = []
    for b in range(2):
        z = np.linalg.solve(A, oracle.vec(q[b]))
        ref.append(oracle.unvec(oracle.vec(q[b]) + s.dt * (M @ z), s.N))
    assert rel_state_err(out, np.stack(ref)) < STATE_TOL


def _gradient_case(lbx, systems, alphas, rng, path, B=2, kind=0, ckpt=0):
    batch = [B] * len(systems)
    rho0 = [random_pure_states(rng, s.N, B) for s in systems]
    tar = [random_pure_states(rng, s.N, B) for s in systems]
    beta = rng.uniform(0.5, 2, B * len(systems))
    plan = lbx.Plan(systems, path=path)
    G, grad, rhoT = lbx.adjoint_gradient(plan, kind, dev(flat_alpha(alphas)), dev(flat_states(rho0)),
                                         dev(flat_states(tar)), dev(beta), batch, 0.0, ckpt, want_rhoT=True)
    G, grad = G.cpu().numpy(), grad.cpu().numpy()
    got = split_states(rhoT.cpu().numpy(), systems, batch)
    off = 0
    for k, s in enumerate(systems):
        Gr, gr, rT = oracle.value_and_gradient(s, alphas[k], rho0[k], tar[k], beta[k * B:(k + 1) * B], kind,
                                               return_final=True)
        assert rel_state_err([got[k]], [rT]) < STATE_TOL
        assert abs(G[k] - Gr) <= 1e-12 * abs(Gr)
        gk = grad[off:off + alphas[k].size].reshape(gr.shape)
        assert np.max(np.abs(gk - gr)) <= GRAD_TOL * np.max(np.abs(gr))
        off += alphas[k].size


@pytest.mark.parametrize("nlev,path", [((2, 3), "lds"), ((2, 3), "stream"), ((3, 3, 3, 3), "auto"),
                                       ((2, 2, 2, 2), "lds")])
def test_coupled_gradient_matches_oracle(lbx, nlev, path):
    s, alpha, rng = _jc(640 + sum(nlev), nlev)
    say("coupled gradient", nlev, path)
    _gradient_case(lbx, [s], [alpha], rng, path)


def test_mixed_batch_with_and_without_coupling(lbx):
    # coupled systems on the generic kernels beside uncoupled ones on the
    # specialised LDS kernels and the block-tiled streamed kernels
    rng = np.random.default_rng(660)
    systems, alphas = [], []
    for nlev, jc in [((2, 3), 0.03), ((2, 3), 0.0), ((3, 3), 0.02), ((3,) * 5, 0.0)]:
        s = random_system(rng, nlev, NT=10, T=1.0, Ns=5, Nf=2, jc=jc)
        systems.append(s)
        alphas.append(random_alpha(rng, s, amp=0.02))
    say("mixed coupled batch")
    _gradient_case(lbx, systems, alphas, rng, "auto", B=1)


def test_coupled_steps_beyond_the_splitting_bound(lbx):
    # a strong coupling puts every step above theta = 0.5: GMRES fallback
    s, alpha, rng = _jc(680, (3, 3), NT=8, T=1.6, jc=0.6, amp=0.02)
    plan = lbx.Plan([s])
    k = lbx.sweep_counts(plan, dev(alpha.reshape(-1)))[0, :, 1]
    assert (k < 1).all()
    say("coupled krylov")
    _gradient_case(lbx, [s], [alpha], rng, "auto")


@pytest.mark.parametrize("kind", [0, 1])
def test_coupled_gradient_with_checkpoint_recomputation(lbx, kind):
    # checkpoints every 3 steps: the coupled streamed forward states are
    # recomputed between checkpoints in the adjoint
    s, alpha, rng = _jc(690 + kind, (3, 2, 2), NT=11, T=1.1)
    say("coupled gradient ckpt", kind)
    _gradient_case(lbx, [s], [alpha], rng, "auto", B=2, kind=kind, ckpt=3)
