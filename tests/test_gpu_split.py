"""The two-pass sweeps and apply (LB_OPT_TILE_KI = 100 + KA: pass A over the
KA least significant subsystems, pass B over the others) against the oracle
(App. A eq. mastereq_vectorized, eqs. IMR / linsystem_primal, App. B) and
against the block-tiled kernels at the eight-qutrit size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import make_config, random_alpha, random_pure_states, random_system  # noqa: E402

from _gpu import dev, rel_state_err, say  # noqa: E402

STATE_TOL = 1e-12
GRAD_TOL = 1e-10


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _plan(lbx, systems, ka, path=None):
    plan = lbx.Plan(systems, path=path) if path else lbx.Plan(systems)
    plan.set_option(lbx._native.LB_OPT_TILE, 1)
    plan.set_option(lbx._native.LB_OPT_TILE_KI, 100 + ka)
    return plan


@pytest.mark.parametrize("nlev,ka", [((3,) * 5, 2), ((3,) * 5, 3), ((2, 3, 4), 1), ((2, 3, 4), 2),
                                     ((4, 4, 4), 1), ((5, 2, 3, 2), 2)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_split_apply_matches_operator_form(lbx, nlev, ka, adjoint):
    rng = np.random.default_rng(400 + sum(nlev) + ka)
    s = random_system(rng, nlev, NT=8, T=0.8, Ns=5, Nf=2)
    alpha = random_alpha(rng, s, amp=0.03)
    N = s.N
    x = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    t = 0.37
    say("split apply", nlev, ka, adjoint)
    plan = _plan(lbx, [s], ka)
    y = lbx.lindblad_apply(plan, 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
    ref = np.stack([f(s, alpha, t, x[b]) for b in range(2)])
    assert rel_state_err(y, ref) < 1e-13


@pytest.mark.parametrize("nlev,ka", [((3, 3, 3), 1), ((3, 3, 3), 2), ((2, 3, 3), 1)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_split_imr_step_matches_dense_solve(lbx, nlev, ka, adjoint):
    rng = np.random.default_rng(420 + sum(nlev) + ka)
    s = random_system(rng, nlev, NT=10, T=1.0, Ns=5, Nf=2)
    alpha = random_alpha(rng, s, amp=0.02)
    q = rng.standard_normal((2, s.N, s.N)) + 1j * rng.standard_normal((2, s.N, s.N))
    j = 6
    say("split imr_step", nlev, ka, adjoint)
    plan = _plan(lbx, [s], ka)
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


@pytest.mark.parametrize("nlev,ka", [((3, 3, 3, 3), 2), ((2, 4, 3, 3), 1)])
def test_split_gradient_matches_oracle(lbx, nlev, ka):
    rng = np.random.default_rng(440 + sum(nlev) + ka)
    s = random_system(rng, nlev, NT=10, T=1.0, Ns=5, Nf=2)
    alpha = random_alpha(rng, s, amp=0.02)
    B = 2
    rho0 = random_pure_states(rng, s.N, B)
    tar = random_pure_states(rng, s.N, B)
    beta = rng.uniform(0.5, 2, B)
    say("split gradient", nlev, ka)
    plan = _plan(lbx, [s], ka, path="stream")
    G, grad, rhoT = lbx.adjoint_gradient(plan, 0, dev(alpha.reshape(-1)), dev(rho0), dev(tar), dev(beta), [B],
                                         0.0, 0, want_rhoT=True)
    Gr, gr, rT = oracle.value_and_gradient(s, alpha, rho0, tar, beta, 0, return_final=True)
    assert rel_state_err([rhoT.cpu().numpy().reshape(B, s.N, s.N)], [rT]) < STATE_TOL
    assert abs(G.item() - Gr) <= 1e-12 * abs(Gr)
    assert np.max(np.abs(grad.cpu().numpy().reshape(gr.shape) - gr)) <= GRAD_TOL * np.max(np.abs(gr))


@pytest.mark.parametrize("adjoint", [False, True])
def test_split_apply_eight_qutrits_matches_block_tiled(lbx, adjoint):
    p = make_config(5)
    s = p.systems[0]
    N = s.N
    g = torch.Generator(device="cuda")
    g.manual_seed(17)
    x = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    a = dev(p.alpha[0].reshape(-1))
    say("split apply eight qutrits", adjoint)
    y_split = lbx.lindblad_apply(_plan(lbx, [s], 4), 0, 41.0, a, x, adjoint=adjoint)
    y_tile = lbx.lindblad_apply(lbx.Plan([s]), 0, 41.0, a, x, adjoint=adjoint)
    err = (torch.linalg.vector_norm(y_split - y_tile) / torch.linalg.vector_norm(y_tile)).item()
    assert err < 1e-14
    # and a sample of entries against the oracle, entry by entry
    rng = np.random.default_rng(18)
    rows, cols = rng.integers(0, N, 32), rng.integers(0, N, 32)
    xs = x[0].cpu().numpy()
    ref = oracle.lindbladian_entries(s, p.alpha[0], 41.0, xs, rows, cols, adjoint=adjoint)
    got = y_split[0].cpu().numpy()[rows, cols]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("adjoint", [False, True])
def test_split_step_eight_qutrits_solves_its_stage_equation(lbx, adjoint):
    p = make_config(5)
    s = p.systems[0]
    N = s.N
    j = 777
    g = torch.Generator(device="cuda")
    g.manual_seed(19)
    q = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    say("split imr_step eight qutrits", adjoint)
    out = lbx.imr_step(_plan(lbx, [s], 4), 0, j, dev(p.alpha[0].reshape(-1)), q, adjoint=adjoint)
    z = ((q + out) * 0.5)[0].cpu().numpy()
    qn = q[0].cpu().numpy()
    del q, out
    rng = np.random.default_rng(20)
    rows, cols = rng.integers(0, N, 64), rng.integers(0, N, 64)
    Mz = oracle.lindbladian_entries(s, p.alpha[0], (j + 0.5) * s.dt, z, rows, cols, adjoint=adjoint)
    res = z[rows, cols] - 0.5 * s.dt * Mz - qn[rows, cols]
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(qn[rows, cols]))
