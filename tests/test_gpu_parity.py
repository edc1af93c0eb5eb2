"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP64 throughout): final states and single applications within
1e-12 relative (Frobenius norm per state), objectives within 1e-12
relative, gradients within 1e-10 relative to the max-norm of the oracle
gradient.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import (  # noqa: E402
    make_config, random_alpha, random_pure_states, random_system, truncate_steps,
)

from _gpu import dev, flat_alpha, flat_states, rel_state_err, say, split_states  # noqa: E402

STATE_TOL = 1e-12
GRAD_TOL = 1e-10

SHAPES = [(3,), (2, 3), (4, 4), (3, 2, 2), (2, 2, 2, 2), (5, 3), (3, 3, 3), (7,)]


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _sys(seed, nlev, NT=30, T=3.0, Ns=5, Nf=2, amp=0.02):
    rng = np.random.default_rng(seed)
    s = random_system(rng, nlev, NT=NT, T=T, Ns=Ns, Nf=Nf)
    return s, random_alpha(rng, s, amp=amp), rng


# --------------------------------------------------------------- control table

@pytest.mark.parametrize("cfg", [1, 2])
def test_control_table_matches_oracle(lbx, cfg):
    p = make_config(cfg)
    s = p.systems[0]
    say("control_table", cfg)
    plan = lbx.Plan([s])
    tab = lbx.control_table(plan, 0, dev(p.alpha[0].reshape(-1))).cpu().numpy()
    ref = np.stack([oracle.controls(s, p.alpha[0], (j + 0.5) * s.dt) for j in range(s.NT)])
    assert np.max(np.abs(tab - ref)) <= 1e-14 * np.max(np.abs(ref))


# --------------------------------------------------------------- apply

@pytest.mark.parametrize("nlev", SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_lindblad_apply_matches_dense_superoperator(lbx, nlev, adjoint):
    s, alpha, rng = _sys(hash(nlev) % 1000, nlev)
    N = s.N
    B = 3
    x = rng.standard_normal((B, N, N)) + 1j * rng.standard_normal((B, N, N))
    t = 1.234
    say("apply", nlev, adjoint)
    plan = lbx.Plan([s])
    y = lbx.lindblad_apply(plan, 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    if N * N <= 1024:
        M = oracle.superoperator(s, alpha, t)
        if adjoint:
            M = M.conj().T
        ref = np.stack([oracle.unvec(M @ oracle.vec(x[b]), N) for b in range(B)])
    else:
        f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
        ref = np.stack([f(s, alpha, t, x[b]) for b in range(B)])
    assert rel_state_err(y, ref) < 1e-13


def test_lindblad_apply_empty_batch_is_noop(lbx):
    s, alpha, _ = _sys(1, (2, 3))
    plan = lbx.Plan([s])
    x = torch.zeros((0, 6, 6), dtype=torch.complex128, device="cuda")
    y = lbx.lindblad_apply(plan, 0, 0.1, dev(alpha.reshape(-1)), x)
    assert y.shape == (0, 6, 6)


@pytest.mark.parametrize("tile,ki", [(1, 44), (1, 43), (1, 34), (1, 33), (1, 32), (1, 23), (2, 0)])
def test_lindblad_apply_eight_qutrits_sampled(lbx, tile, ki):
    # The 8-qutrit ring at full size (N = 6561, 43M entries per state): check
    # sampled entries, each formed by the oracle from single operator rows,
    # for the one-pass block-tiled and the two-pass split kernels.
    p = make_config(5)
    s = p.systems[0]
    rng = np.random.default_rng(55)
    N = s.N
    x = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))) / np.sqrt(2)
    t = 37.3
    say("apply c5 full size, tile", tile, ki)
    plan = lbx.Plan([s], tile=tile)
    plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
    al = dev(p.alpha[0].reshape(-1))
    xd = dev(x[None])
    for adjoint in (False, True):
        y = lbx.lindblad_apply(plan, 0, t, al, xd, adjoint=adjoint)
        rows = np.concatenate([rng.integers(0, N, 60), [0, N - 1, 0, N - 1]])
        cols = np.concatenate([rng.integers(0, N, 60), [0, N - 1, N - 1, 0]])
        got = y[0, torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().numpy()
        ref = oracle.lindbladian_entries(s, p.alpha[0], t, x, rows, cols, adjoint=adjoint)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale
        del y


# --------------------------------------------------------------- one IMR step

@pytest.mark.parametrize("nlev", [(3,), (2, 3), (4, 4), (3, 2, 2)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_imr_step_matches_dense_solve(lbx, nlev, adjoint):
    s, alpha, rng = _sys(7 + len(nlev), nlev, NT=10, T=1.0)
    N = s.N
    B = 2
    q = rng.standard_normal((B, N, N)) + 1j * rng.standard_normal((B, N, N))
    j = 4
    say("imr_step", nlev, adjoint)
    plan = lbx.Plan([s])
    out = lbx.imr_step(plan, 0, j, dev(alpha.reshape(-1)), dev(q), adjoint=adjoint).cpu().numpy()
    M = oracle.superoperator(s, alpha, (j + 0.5) * s.dt)
    if adjoint:
        M = M.conj().T
    A = np.eye(N * N) - 0.5 * s.dt * M
    ref = []
    for b in range(B):
        z = np.linalg.solve(A, oracle.vec(q[b]))
        ref.append(oracle.unvec(oracle.vec(q[b]) + s.dt * (M @ z), N))
    assert rel_state_err(out, np.stack(ref)) < STATE_TOL


# --------------------------------------------------------------- forward solve

def _multi(seeds_shapes, NT=30, B=(2, 1, 3, 2, 1, 2, 2, 1), T=3.0):
    systems, alphas, rho0, batch = [], [], [], []
    for k, (seed, nlev) in enumerate(seeds_shapes):
        s, a, rng = _sys(seed, nlev, NT=NT, T=T)
        systems.append(s)
        alphas.append(a)
        b = B[k % len(B)]
        batch.append(b)
        rho0.append(random_pure_states(rng, s.N, b))
    return systems, alphas, rho0, batch


@pytest.mark.parametrize("path", ["auto", "lds", "stream"])
def test_forward_solve_multi_system(lbx, path):
    shapes = [(3,), (2, 3), (4, 4), (3, 2, 2), (2, 2, 2), (5, 3)]
    if path == "stream":
        shapes.append((3, 3, 3))
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=20)))
    say("forward_solve", path, batch)
    plan = lbx.Plan(systems, path=path)
    rhoT = lbx.forward_solve(plan, dev(flat_alpha(alphas)), dev(flat_states(rho0)), batch)
    got = split_states(rhoT.cpu().numpy(), systems, batch)
    ref = [oracle.imr_forward(s, a, r) for s, a, r in zip(systems, alphas, rho0)]
    assert rel_state_err(got, ref) < STATE_TOL


def test_forward_solve_with_empty_system_and_trivial_subsystem(lbx):
    s1, a1, rng = _sys(31, (3, 1, 2))
    s2, a2, _ = _sys(32, (2, 2))
    rho1 = random_pure_states(rng, s1.N, 2)
    batch = [2, 0]
    say("forward_solve empty+trivial")
    plan = lbx.Plan([s1, s2])
    rhoT = lbx.forward_solve(plan, dev(flat_alpha([a1, a2])), dev(flat_states([rho1])), batch)
    got = split_states(rhoT.cpu().numpy(), [s1], [2])
    ref = [oracle.imr_forward(s1, a1, rho1)]
    assert rel_state_err(got, ref) < STATE_TOL


def test_config1_full_forward(lbx):
    p = make_config(1)
    s = p.systems[0]
    say("c1 full forward")
    plan = lbx.Plan([s])
    rhoT = lbx.forward_solve(plan, dev(p.alpha[0].reshape(-1)), dev(p.rho0[0]), [1]).cpu().numpy()
    ref = oracle.imr_forward(s, p.alpha[0], p.rho0[0])
    assert rel_state_err([rhoT], [ref]) < STATE_TOL


# --------------------------------------------------------------- objective

@pytest.mark.parametrize("kind", [0, 1])
def test_objective_matches_oracle(lbx, kind):
    systems, alphas, rho0, batch = _multi([(40, (2, 3)), (41, (3, 3)), (42, (4,))])
    rng = np.random.default_rng(43)
    tars = [random_pure_states(rng, s.N, b) for s, b in zip(systems, batch)]
    rhoT = [oracle.imr_forward(s, a, r) for s, a, r in zip(systems, alphas, rho0)]
    beta = rng.uniform(0.5, 2, sum(batch))
    say("objective", kind)
    plan = lbx.Plan(systems)
    G, J = lbx.objective(plan, kind, dev(flat_states(rhoT)), dev(flat_states(tars)), dev(beta),
                         batch, 0.7, dev(flat_alpha(alphas)))
    G = G.cpu().numpy()
    off = 0
    for k, s in enumerate(systems):
        ref = oracle.objective(kind, rhoT[k], tars[k], beta[off:off + batch[k]], 0.7, alphas[k])
        off += batch[k]
        assert abs(G[k] - ref) <= 1e-12 * abs(ref)


# --------------------------------------------------------------- adjoint gradient

def _grad_case(lbx, systems, alphas, rho0, batch, kind, gamma2, path, ckpt, seed=50):
    rng = np.random.default_rng(seed)
    tars = [random_pure_states(rng, s.N, b) for s, b in zip(systems, batch)]
    beta = rng.uniform(0.5, 2, sum(batch))
    plan = lbx.Plan(systems, path=path)
    G, grad, rhoT = lbx.adjoint_gradient(plan, kind, dev(flat_alpha(alphas)), dev(flat_states(rho0)),
                                         dev(flat_states(tars)), dev(beta), batch, gamma2, ckpt,
                                         want_rhoT=True)
    G, grad = G.cpu().numpy(), grad.cpu().numpy()
    got_rhoT = split_states(rhoT.cpu().numpy(), systems, batch)
    off_b, off_a = 0, 0
    for k, s in enumerate(systems):
        bk = batch[k]
        Gr, gr = oracle.value_and_gradient(s, alphas[k], rho0[k], tars[k], beta[off_b:off_b + bk], kind, gamma2)
        rT = oracle.imr_forward(s, alphas[k], rho0[k])
        assert rel_state_err([got_rhoT[k]], [rT]) < STATE_TOL
        assert abs(G[k] - Gr) <= 1e-12 * abs(Gr)
        ga = grad[off_a:off_a + alphas[k].size].reshape(alphas[k].shape)
        assert np.max(np.abs(ga - gr)) <= GRAD_TOL * np.max(np.abs(gr)), (k, np.max(np.abs(ga - gr)), np.max(np.abs(gr)))
        off_b += bk
        off_a += alphas[k].size


def test_streamed_systems_at_their_own_sweep_counts(lbx):
    # Streamed systems of one launch whose controls differ by two orders of
    # magnitude need different numbers of stage sweeps per step; each must
    # stop at its own count (last sweep, stage vector and integrands chosen
    # per segment) and still match the oracle.
    pairs = [(81, (3, 2), 0.1), (82, (2, 3), 0.001), (83, (3, 3), 0.03)]
    systems, alphas, rho0, batch = [], [], [], []
    for seed, nlev, amp in pairs:
        s, a, rng = _sys(seed, nlev, NT=20, T=2.0, amp=amp)
        systems.append(s)
        alphas.append(a)
        batch.append(2)
        rho0.append(random_pure_states(rng, s.N, 2))
    plan = lbx.Plan(systems, path="stream")
    k = lbx.sweep_counts(plan, dev(flat_alpha(alphas)))[:, :, 1]
    say("own sweep counts", k.min(axis=1), k.max(axis=1))
    assert k[0].min() > k[1].max()  # the launch runs the largest count, system 1 stops early
    _grad_case(lbx, systems, alphas, rho0, batch, 0, 0.0, "stream", 4)


@pytest.mark.parametrize("path,ckpt", [("lds", 1), ("stream", 1), ("stream", 4), ("stream", 0), ("auto", 7)])
@pytest.mark.parametrize("kind,gamma2", [(0, 0.0), (1, 0.25)])
def test_adjoint_gradient_matches_oracle(lbx, path, ckpt, kind, gamma2):
    shapes = [(3,), (2, 3), (3, 2, 2), (4, 4)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=60)), NT=18)
    say("adjoint_gradient", path, ckpt, kind, gamma2)
    _grad_case(lbx, systems, alphas, rho0, batch, kind, gamma2, path, ckpt)


def test_config1_full_gradient(lbx):
    p = make_config(1)
    s = p.systems[0]
    say("c1 full gradient")
    plan = lbx.Plan([s])
    G, grad, _ = lbx.adjoint_gradient(plan, p.kind, dev(p.alpha[0].reshape(-1)), dev(p.rho0[0]),
                                      dev(p.rhotar[0]), dev(p.beta[0]), [1])
    Gr, gr = oracle.value_and_gradient(s, p.alpha[0], p.rho0[0], p.rhotar[0], p.beta[0], p.kind)
    assert abs(G.item() - Gr) <= 1e-12 * abs(Gr)
    assert np.max(np.abs(grad.cpu().numpy().reshape(gr.shape) - gr)) <= GRAD_TOL * np.max(np.abs(gr))


def test_autograd_function_and_finite_differences(lbx):
    s, alpha, rng = _sys(77, (2, 3), NT=20, T=2.0)
    rho0 = random_pure_states(rng, s.N, 2)
    tar = random_pure_states(rng, s.N, 2)
    beta = np.array([1.0, 0.5])
    plan = lbx.Plan([s])
    a = dev(alpha.reshape(-1)).requires_grad_(True)
    say("autograd")
    G = lbx.lindblad_objective(a, plan, 0, dev(rho0), dev(tar), dev(beta), [2])
    (3.0 * G.sum()).backward()
    _, gr = oracle.value_and_gradient(s, alpha, rho0, tar, beta, 0)
    assert np.max(np.abs(a.grad.cpu().numpy() - 3.0 * gr.reshape(-1))) <= GRAD_TOL * 3 * np.max(np.abs(gr))
    # central differences of the GPU objective itself
    h = 1e-6
    base = alpha.reshape(-1)
    for k in [0, 5, 11, 17]:
        vals = []
        for sgn in (1, -1):
            ak = base.copy()
            ak[k] += sgn * h
            with torch.no_grad():
                vals.append(lbx.lindblad_objective(dev(ak), plan, 0, dev(rho0), dev(tar), dev(beta), [2]).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gr.reshape(-1)[k]) <= 1e-6 * np.max(np.abs(gr))


def _fd_check(lbx, p, idx, h=1e-6, rel=1e-6):
    """Central differences of the GPU objective (forward solve + objective) on
    coefficients idx against the autograd/adjoint gradient of the same call."""
    s = p.systems[0]
    batch = [p.rho0[0].shape[0]]
    plan = lbx.Plan([s])
    a0 = p.alpha[0].reshape(-1)
    args = (dev(p.rho0[0]), dev(p.rhotar[0]), dev(p.beta[0]), batch, p.gamma2, p.ckpt_every or 0)
    a = dev(a0).requires_grad_(True)
    lbx.lindblad_objective(a, plan, p.kind, *args).sum().backward()
    g = a.grad.cpu().numpy()
    gmax = np.max(np.abs(g))
    for k in idx:
        vals = []
        for sgn in (1, -1):
            ak = a0.copy()
            ak[k] += sgn * h
            with torch.no_grad():
                vals.append(lbx.lindblad_objective(dev(ak), plan, p.kind, *args).item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) <= rel * gmax, (k, fd, g[k], gmax)


def test_config2_full_length_finite_differences(lbx):
    # Two transmons, 16 basis states, 10000 steps: central differences with
    # h = 1e-6 on a seeded subset of 16 of the 160 coefficients.
    p = make_config(2)
    idx = np.random.default_rng(2).choice(p.alpha[0].size, 16, replace=False)
    say("c2 finite differences", list(idx))
    _fd_check(lbx, p, idx)


def test_config4_full_length_finite_differences(lbx):
    # Five-qutrit chain, 10 states, 20000 steps, checkpoints every 200 steps
    # recomputed in the adjoint: spot check on 8 coefficients.
    p = make_config(4)
    idx = np.random.default_rng(4).choice(p.alpha[0].size, 8, replace=False)
    say("c4 finite differences", list(idx))
    _fd_check(lbx, p, idx)


def test_gradient_is_bitwise_deterministic(lbx):
    shapes = [(2, 3), (3, 3, 3)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=90)), NT=12)
    rng = np.random.default_rng(3)
    tars = [random_pure_states(rng, s.N, b) for s, b in zip(systems, batch)]
    plan = lbx.Plan(systems)
    args = (dev(flat_alpha(alphas)), dev(flat_states(rho0)), dev(flat_states(tars)),
            dev(np.ones(sum(batch))), batch)
    say("determinism")
    g1 = lbx.adjoint_gradient(plan, 0, *args)[1].cpu().numpy()
    g2 = lbx.adjoint_gradient(plan, 0, *args)[1].cpu().numpy()
    assert np.array_equal(g1, g2)


@pytest.mark.parametrize("NT", [1, 2, 3, 4, 5, 6, 12])
def test_lds_extrapolated_start_on_short_horizons(lbx, NT):
    # The specialised LDS kernels start each stage iteration from the
    # polynomial extrapolation of the previous increments, of order 0 to 4
    # (second to sixth step onward); every start must converge.
    shapes = [(3, 3), (2, 2, 2)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=120)), NT=NT, T=0.2 * NT)
    say("lds extrapolated start", NT)
    _grad_case(lbx, systems, alphas, rho0, batch, 0, 0.0, "lds", 1)


def test_profile_work_counts_sweeps(lbx):
    p = truncate_steps(make_config(2), 200)
    s = p.systems[0]
    args = (dev(p.alpha[0].reshape(-1)), dev(p.rho0[0]), dev(p.rhotar[0]), dev(p.beta[0]), [16])
    entries = 16 * s.N * s.N
    say("profile work")
    nat = lbx._native
    plan = lbx.Plan([s], path="lds")
    plan.profile(True)
    lbx.adjoint_gradient(plan, p.kind, *args)
    apriori = int(lbx.sweep_counts(plan, args[0])[0, :, 0].sum()) * entries
    for k in (nat.LB_KERNEL_LDS_FORWARD, nat.LB_KERNEL_LDS_ADJOINT):
        w = plan.profile_work(k)
        assert w % (s.N * s.N) == 0 and s.NT * entries <= w <= 2 * apriori, (k, w, apriori)
        assert plan.profile_read(k, reset=True)[0] == 1
        assert plan.profile_work(k) == 0
    splan = lbx.Plan([s], path="stream")
    splan.profile(True)
    lbx.adjoint_gradient(splan, p.kind, *args)
    # one persistent launch per step of each pass (forward, recomputation,
    # adjoint), each with at least two sweeps
    n_steps, _ = splan.profile_read(nat.LB_KERNEL_SWEEP)
    w = splan.profile_work(nat.LB_KERNEL_SWEEP)
    assert n_steps >= 2 * s.NT and w % entries == 0 and w >= 2 * n_steps * entries
    n_grad, _ = splan.profile_read(nat.LB_KERNEL_STREAM_GRAD)
    assert n_grad == s.NT and splan.profile_work(nat.LB_KERNEL_STREAM_GRAD) == s.NT * entries


def test_lds_kernel_classes_with_several_entries_per_thread(lbx):
    # N^2 = 1296 (two entries per thread) and N^2 = 4096 (four per thread).
    shapes = [(6, 6), (4, 4, 4)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=95)), NT=6, B=(2, 1), T=0.6)
    say("lds classes ept 2/4", batch)
    _grad_case(lbx, systems, alphas, rho0, batch, 0, 0.0, "lds", 1)


def test_config3_subset_reduced_steps(lbx):
    p = truncate_steps(make_config(3), 12)
    # systems of the uneven batch on both kernel families: five small ones
    # (LDS-resident) and one with N^2 > 4096 (streamed)
    small = [k for k, s in enumerate(p.systems) if s.N <= 32][:5]
    big = [k for k, s in enumerate(p.systems) if 64 < s.N <= 81][:1]
    idx = small + big
    systems = [p.systems[k] for k in idx]
    alphas = [p.alpha[k] for k in idx]
    rho0 = [p.rho0[k] for k in idx]
    batch = [r.shape[0] for r in rho0]
    say("c3 subset", [s.nlev for s in systems], batch)
    _grad_case(lbx, systems, alphas, rho0, batch, 0, 0.0, "auto", 4)


def test_config2_full_length_against_stored_oracle(lbx):
    # Two transmons, 16 basis states, 10000 steps: expected values written by
    # tests/golden/make_golden.py from the oracle alone.
    import os
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_cnot_full.npz"))
    p = make_config(2)
    s = p.systems[0]
    say("c2 full gradient vs stored oracle")
    plan = lbx.Plan([s])
    G, grad, rhoT = lbx.adjoint_gradient(plan, p.kind, dev(p.alpha[0].reshape(-1)), dev(p.rho0[0]),
                                         dev(p.rhotar[0]), dev(p.beta[0]), [16], want_rhoT=True)
    assert rel_state_err([rhoT.cpu().numpy()], [gold["rhoT"]]) < STATE_TOL
    assert abs(G.item() - float(gold["G"])) <= 1e-12 * abs(float(gold["G"]))
    g = grad.cpu().numpy().reshape(gold["grad"].shape)
    assert np.max(np.abs(g - gold["grad"])) <= GRAD_TOL * np.max(np.abs(gold["grad"]))


# --------------------------------------------------------------- block-tiled kernels

TILE_SHAPES = [(2,) * 9, (3,) * 6, (4,) * 5]


@pytest.mark.parametrize("nlev", TILE_SHAPES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_row_tiled_apply_matches_operator_form(lbx, nlev, adjoint):
    s, alpha, rng = _sys(200 + len(nlev), nlev, Nf=1)
    N = s.N
    x = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    t = 0.77
    say("tile apply", nlev, adjoint)
    plan = lbx.Plan([s])
    y = lbx.lindblad_apply(plan, 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
    ref = np.stack([f(s, alpha, t, x[b]) for b in range(2)])
    assert rel_state_err(y, ref) < 1e-13
    plan_g = lbx.Plan([s], tile=False)
    yg = lbx.lindblad_apply(plan_g, 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    assert rel_state_err(y, yg) < 1e-14


@pytest.mark.parametrize("nlev,ki", [((3,) * 7, 43), ((3,) * 6, 43), ((3,) * 5, 33), ((3,) * 5, 32),
                                     ((3,) * 5, 23)])
def test_block_shapes_match_generic_kernel(lbx, nlev, ki):
    # Every instantiated block shape (some with 256-thread blocks) against
    # the generic streaming kernel and the operator form.
    s, alpha, rng = _sys(260 + ki, nlev, Nf=1)
    N = s.N
    x = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    t = 0.52
    say("block shape", nlev, ki)
    plan = lbx.Plan([s])
    plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
    al = dev(alpha.reshape(-1))
    for adjoint in (False, True):
        y = lbx.lindblad_apply(plan, 0, t, al, dev(x), adjoint=adjoint).cpu().numpy()
        yg = lbx.lindblad_apply(lbx.Plan([s], tile=0), 0, t, al, dev(x), adjoint=adjoint).cpu().numpy()
        assert rel_state_err(y, yg) < 1e-14
        if N <= 729:
            f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
            assert rel_state_err(y[:1], f(s, alpha, t, x[0])[None]) < 1e-13


@pytest.mark.parametrize("adjoint", [False, True])
def test_row_tiled_imr_step_matches_oracle(lbx, adjoint):
    s, alpha, rng = _sys(211, (3,) * 6, NT=8, T=0.4, Nf=1)
    N = s.N
    q = random_pure_states(rng, N, 1)
    j = 3
    say("tile imr_step", adjoint)
    plan = lbx.Plan([s])
    out = lbx.imr_step(plan, 0, j, dev(alpha.reshape(-1)), dev(q), adjoint=adjoint).cpu().numpy()
    t = (j + 0.5) * s.dt
    f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
    import scipy.sparse.linalg as spla
    v0 = oracle.vec(q[0])
    A = spla.LinearOperator((N * N, N * N), dtype=complex,
                            matvec=lambda v: v - 0.5 * s.dt * oracle.vec(f(s, alpha, t, oracle.unvec(v, N))))
    z, info = spla.gmres(A, v0, rtol=1e-14, atol=0.0, restart=60, maxiter=40)
    ref = oracle.unvec(v0 + s.dt * oracle.vec(f(s, alpha, t, oracle.unvec(z, N))), N)
    assert rel_state_err(out, ref[None]) < STATE_TOL


def test_row_tiled_gradient_matches_oracle(lbx):
    systems, alphas, rho0, batch = _multi([(220, (3,) * 6)], NT=3, B=(1,), T=0.15)
    say("tile gradient")
    _grad_case(lbx, systems, alphas, rho0, batch, 0, 0.0, "stream", 2)


@pytest.mark.parametrize("ki", [33, 23, 32])
def test_tiled_gradient_block_shapes_match_oracle(lbx, ki):
    # Five qutrits, two states: sweeps and gradient integrands in 256-thread
    # block shapes, against the oracle's discrete adjoint.
    systems, alphas, rho0, batch = _multi([(270 + ki, (3,) * 5)], NT=4, B=(2,), T=0.2)
    say("tile gradient shape", ki)
    rng = np.random.default_rng(ki)
    tars = [random_pure_states(rng, systems[0].N, 2)]
    beta = np.array([1.0, 0.7])
    plan = lbx.Plan(systems, path="stream")
    plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
    G, grad, rhoT = lbx.adjoint_gradient(plan, 1, dev(flat_alpha(alphas)), dev(flat_states(rho0)),
                                         dev(flat_states(tars)), dev(beta), batch, 0.0, 2, want_rhoT=True)
    Gr, gr = oracle.value_and_gradient(systems[0], alphas[0], rho0[0], tars[0], beta, 1)
    assert abs(G.item() - Gr) <= 1e-12 * abs(Gr)
    g = grad.cpu().numpy().reshape(gr.shape)
    assert np.max(np.abs(g - gr)) <= GRAD_TOL * np.max(np.abs(gr))


# --------------------------------------------------------------- two-pass split kernels

@pytest.mark.parametrize("nlev", [(3,) * 7, (2,) * 11])
@pytest.mark.parametrize("adjoint", [False, True])
def test_split_apply_matches_operator_form(lbx, nlev, adjoint):
    s, alpha, rng = _sys(230 + len(nlev), nlev, Nf=1)
    N = s.N
    x = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    t = 0.61
    say("split apply", nlev, adjoint)
    plan = lbx.Plan([s], tile=2)
    y = lbx.lindblad_apply(plan, 0, t, dev(alpha.reshape(-1)), dev(x), adjoint=adjoint).cpu().numpy()
    f = oracle.lindbladian_adjoint if adjoint else oracle.lindbladian
    assert rel_state_err(y, f(s, alpha, t, x[0])[None]) < 1e-13
    yg = lbx.lindblad_apply(lbx.Plan([s], tile=0), 0, t, dev(alpha.reshape(-1)), dev(x),
                            adjoint=adjoint).cpu().numpy()
    assert rel_state_err(y, yg) < 1e-14


def test_split_apply_four_level_sampled(lbx):
    # Six 4-level subsystems (N = 4096): sampled entries against the oracle,
    # every entry against the generic streaming kernel.
    s, alpha, rng = _sys(240, (4,) * 6, Nf=1)
    N = s.N
    x = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    t = 0.33
    say("split apply 4^6")
    al = dev(alpha.reshape(-1))
    for adjoint in (False, True):
        y = lbx.lindblad_apply(lbx.Plan([s], tile=2), 0, t, al, dev(x), adjoint=adjoint)
        rows = np.concatenate([rng.integers(0, N, 40), [0, N - 1]])
        cols = np.concatenate([rng.integers(0, N, 40), [N - 1, 0]])
        got = y[0, torch.as_tensor(rows, device="cuda"), torch.as_tensor(cols, device="cuda")].cpu().numpy()
        ref = oracle.lindbladian_entries(s, alpha, t, x[0], rows, cols, adjoint=adjoint)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
        yg = lbx.lindblad_apply(lbx.Plan([s], tile=0), 0, t, al, dev(x), adjoint=adjoint)
        assert rel_state_err(y.cpu().numpy(), yg.cpu().numpy()) < 1e-14


@pytest.mark.parametrize("adjoint", [False, True])
def test_split_imr_step_and_gradient_match_generic(lbx, adjoint):
    # The split and the generic kernels run the same sweeps (the generic ones
    # are checked against the oracle above): results agree to rounding.
    systems, alphas, rho0, batch = _multi([(250, (3,) * 7)], NT=3, B=(1,), T=0.15)
    s, alpha = systems[0], alphas[0]
    say("split imr_step/gradient", adjoint)
    al = dev(alpha.reshape(-1))
    q = dev(rho0[0])
    outs = [lbx.imr_step(lbx.Plan([s], tile=tile), 0, 1, al, q, adjoint=adjoint).cpu().numpy()
            for tile in (2, 0)]
    assert rel_state_err(outs[0], outs[1]) < 1e-14
    if adjoint:
        rng = np.random.default_rng(7)
        tar = dev(random_pure_states(rng, s.N, 1))
        res = [lbx.adjoint_gradient(lbx.Plan([s], tile=tile), 0, al, q, tar, dev(np.ones(1)), [1], 0.0, 2)
               for tile in (2, 0)]
        assert abs(res[0][0].item() - res[1][0].item()) <= 1e-13 * abs(res[1][0].item())
        g0, g1 = res[0][1].cpu().numpy(), res[1][1].cpu().numpy()
        assert np.max(np.abs(g0 - g1)) <= 1e-12 * np.max(np.abs(g1))


# --------------------------------------------------------------- graphs and autotuning

def test_graph_captured_time_loop_matches_direct_launches(lbx):
    from paper_2110_10310_amd import _native as nat
    systems, alphas, rho0, batch = _multi([(300, (3, 3, 3)), (301, (2, 3, 4))], NT=23, B=(3, 2))
    rng = np.random.default_rng(302)
    tars = [random_pure_states(rng, s.N, b) for s, b in zip(systems, batch)]
    args = (dev(flat_alpha(alphas)), dev(flat_states(rho0)), dev(flat_states(tars)),
            dev(np.ones(sum(batch))), batch)
    say("graph capture")
    direct = lbx.Plan(systems, path="stream")
    graph = lbx.Plan(systems, path="stream")
    graph.set_option(nat.LB_OPT_GRAPH, 5)  # chunks of 5 steps: several replays, ragged last chunk
    rd = lbx.forward_solve(direct, args[0], args[1], batch).cpu().numpy()
    for _ in range(3):  # replays interleaved with eager work and synchronisation
        rg = lbx.forward_solve(graph, args[0], args[1], batch).cpu().numpy()
        assert np.array_equal(rg, rd)
        torch.cuda.synchronize()
    Gd, gd, _ = lbx.adjoint_gradient(direct, 0, *args, ckpt_every=7)
    Gg, gg, _ = lbx.adjoint_gradient(graph, 0, *args, ckpt_every=7)
    assert np.array_equal(gd.cpu().numpy(), gg.cpu().numpy())
    assert np.array_equal(Gd.cpu().numpy(), Gg.cpu().numpy())
    ref = [oracle.imr_forward(s, a, r) for s, a, r in zip(systems, alphas, rho0)]
    assert rel_state_err(split_states(rg, systems, batch), ref) < STATE_TOL


def test_autotuner_choice_and_cache(lbx, tmp_path):
    systems, alphas, rho0, batch = _multi([(310, (3,) * 6)], NT=4, B=(1,), T=0.2)
    plan = lbx.Plan(systems)
    al = dev(flat_alpha(alphas))
    say("autotune")
    cache = str(tmp_path / "tune.json")
    ch = plan.autotune(al, batch, cache=cache)
    assert ch["tile"] in (0, 1) and ch["graph_steps"] >= 0
    plan2 = lbx.Plan(systems)
    assert plan2.autotune(al, batch, cache=cache) == ch  # served from the cache
    rT = lbx.forward_solve(plan, al, dev(flat_states(rho0)), batch).cpu().numpy()
    ref = [oracle.imr_forward(systems[0], alphas[0], rho0[0])]
    assert rel_state_err(split_states(rT, systems, batch), ref) < STATE_TOL


# --------------------------------------------------------------- stage-solve counts on the device

def test_streamed_steps_repeat_with_a_priori_counts(lbx):
    # Two sweeps launched per step are too few for these steps: every step
    # raises the retry bit, and the synchronous call repeats itself with the
    # a-priori counts read on the host; the result must still match the oracle.
    shapes = [(3, 3), (2, 3)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=140)), NT=10, B=(2, 1), T=1.0)
    say("retry with a-priori counts")
    nat = lbx._native
    plan = lbx.Plan(systems, path="stream")
    plan.set_option(nat.LB_OPT_SWEEPS, 2)
    rhoT = lbx.forward_solve(plan, dev(flat_alpha(alphas)), dev(flat_states(rho0)), batch)
    ref = [oracle.imr_forward(s, a, r) for s, a, r in zip(systems, alphas, rho0)]
    assert rel_state_err(split_states(rhoT.cpu().numpy(), systems, batch), ref) < STATE_TOL
    # asynchronous calls report the condition through lb_status instead
    plan.set_option(nat.LB_OPT_SYNC, 0)
    ws = plan.workspace(nat.LB_OP_FORWARD, batch)
    lbx.forward_solve(plan, dev(flat_alpha(alphas)), dev(flat_states(rho0)), batch)
    with pytest.raises(lbx._native.LbxError) as e:
        plan.status(ws)
    assert e.value.code == nat.LB_EUNSUPPORTED


@pytest.mark.parametrize("H", [0, 1, 2, 4, 6])
def test_streamed_history_lengths_match_oracle(lbx, H):
    # The first iterate of a streamed step extrapolated from 0 to 6 earlier
    # increments (in the diagonal Cayley frame): the converged steps agree
    # with the oracle whatever the start.
    shapes = [(3, 3), (2, 2, 2)]
    systems, alphas, rho0, batch = _multi(list(enumerate(shapes, start=150)), NT=14, B=(2, 1), T=1.4)
    say("history", H)
    rng = np.random.default_rng(151)
    tars = [random_pure_states(rng, s.N, b) for s, b in zip(systems, batch)]
    beta = np.ones(sum(batch))
    plan = lbx.Plan(systems, path="stream")
    plan.set_option(lbx._native.LB_OPT_HISTORY, H)
    G, grad, rhoT = lbx.adjoint_gradient(plan, 0, dev(flat_alpha(alphas)), dev(flat_states(rho0)),
                                         dev(flat_states(tars)), dev(beta), batch, 0.0, 5, want_rhoT=True)
    got = split_states(rhoT.cpu().numpy(), systems, batch)
    G, grad = G.cpu().numpy(), grad.cpu().numpy()
    off_b = off_a = 0
    for k, s in enumerate(systems):
        Gr, gr, rT = oracle.value_and_gradient(s, alphas[k], rho0[k], tars[k], beta[off_b:off_b + batch[k]], 0,
                                               return_final=True)
        assert rel_state_err([got[k]], [rT]) < STATE_TOL
        assert abs(G[k] - Gr) <= 1e-12 * abs(Gr)
        ga = grad[off_a:off_a + alphas[k].size].reshape(alphas[k].shape)
        assert np.max(np.abs(ga - gr)) <= GRAD_TOL * np.max(np.abs(gr))
        off_b += batch[k]
        off_a += alphas[k].size


# ------------------------------------------------- gradient integrands in the last sweep

@pytest.mark.parametrize("nlev,ki,fused", [((3,) * 5, 33, True), ((3,) * 5, 32, True), ((3,) * 5, 23, True),
                                           ((3,) * 6, 43, True), ((3,) * 7, 33, True), ((3,) * 6, 0, False),
                                           ((2,) * 9, 0, False)])
def test_fused_gradient_integrands_match_the_separate_kernel(lbx, nlev, ki, fused):
    # The last sweep of a block-tiled adjoint step forms the gradient
    # integrands with the stage vector one sweep before convergence; the
    # separate kernel uses the converged one.  Both agree with each other to
    # the stage solve's bound and with the oracle to the parity tolerance.
    # Block shapes whose fused kernel would not keep its values in registers
    # (the 81 x 81 qutrit and 64 x 64 qubit blocks) keep the separate kernel.
    systems, alphas, rho0, batch = _multi([(290 + len(nlev), nlev)], NT=5, B=(2,), T=0.25)
    rng = np.random.default_rng(291)
    tars = [random_pure_states(rng, systems[0].N, 2)]
    beta = np.array([0.8, 1.3])
    res = {}
    for fuse in (1, 0):
        plan = lbx.Plan(systems, path="stream")
        plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
        plan.set_option(lbx._native.LB_OPT_FUSE_GRAD, fuse)
        plan.profile(True)
        say("fused integrands", nlev, ki, fuse)
        G, grad, _ = lbx.adjoint_gradient(plan, 0, dev(flat_alpha(alphas)), dev(flat_states(rho0)),
                                          dev(flat_states(tars)), dev(beta), batch, 0.0, 2)
        n_grad = plan.profile_read(lbx._native.LB_KERNEL_STREAM_GRAD)[0]
        res[fuse] = (G.item(), grad.cpu().numpy(), n_grad)
    assert res[0][2] > 0 and (res[1][2] == 0) == fused  # a fused run launches no integrand kernel
    assert res[1][0] == res[0][0]
    g1, g0 = res[1][1], res[0][1]
    assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0))
    if systems[0].N <= 729:  # (seven qutrits: the oracle's gradient takes over a quarter of an hour)
        say("fused integrands oracle", nlev)
        Gr, gr = oracle.value_and_gradient(systems[0], alphas[0], rho0[0], tars[0], beta, 0)
        assert np.max(np.abs(g1.reshape(gr.shape) - gr)) <= GRAD_TOL * np.max(np.abs(gr))


def test_fused_gradient_integrands_eight_qutrits(lbx):
    # The eight-qutrit ring's block shape, three steps from a seeded random
    # state: fused and separate integrands against each other.
    from workloads import make_config, truncate_steps, with_random_states
    p = truncate_steps(with_random_states(make_config(5), 1, 77), 3)
    s = p.systems[0]
    alpha = dev(p.alpha[0].reshape(-1))
    r0, tar = dev(p.rho0[0][1:]), dev(p.rhotar[0][1:])
    out = {}
    for fuse in (1, 0):
        plan = lbx.Plan([s])
        plan.set_option(lbx._native.LB_OPT_TILE_KI, 34)
        plan.set_option(lbx._native.LB_OPT_FUSE_GRAD, fuse)
        say("fused integrands eight qutrits", fuse)
        G, grad, _ = lbx.adjoint_gradient(plan, 0, alpha, r0, tar, dev(np.ones(1)), [1], 0.0, 1)
        out[fuse] = (G.item(), grad.cpu().numpy())
        del plan
        torch.cuda.empty_cache()
    assert out[1][0] == out[0][0]
    assert np.max(np.abs(out[1][1] - out[0][1])) <= 1e-12 * np.max(np.abs(out[0][1]))


def test_one_sweep_steps_match_a_cold_start(lbx):
    # A three-qutrit cut of the eight-qutrit ring over its real horizon from
    # |0..0> (smooth controls, small contraction bound): with a history of 6
    # many forward steps meet the bound after their first sweep and are
    # finished by stage_finish_kernel; a cold start (no history) never is.
    # Both solve the same stage systems to the same bound.
    from dataclasses import replace
    p = make_config(5)
    s8 = p.systems[0]
    Q = 3
    s = replace(s8, nlev=s8.nlev[:Q], detuning=s8.detuning[:Q], selfkerr=s8.selfkerr[:Q],
                crosskerr=s8.crosskerr[:Q, :Q], T1=s8.T1[:Q], T2=s8.T2[:Q], carriers=s8.carriers[:Q])
    alpha = dev(np.ascontiguousarray(p.alpha[0].reshape(s8.Q, s8.Ns, s8.Nf, 2)[:Q]).reshape(-1))
    N = s.N
    r0 = np.zeros((1, N, N), complex)
    r0[0, 0, 0] = 1
    tar = np.zeros((1, N, N), complex)
    tar[0, N - 1, N - 1] = 1
    r0, tar, beta = dev(r0), dev(tar), dev(np.ones(1))
    out = {}
    for H in (6, 0):
        plan = lbx.Plan([s], path="stream")
        plan.set_option(lbx._native.LB_OPT_HISTORY, H)
        plan.profile(True)
        plan.profile_read(lbx._native.LB_KERNEL_SWEEP, reset=True)
        say("one-sweep steps", H)
        lbx.forward_solve(plan, alpha, r0, [1])
        n, _ = plan.profile_read(lbx._native.LB_KERNEL_SWEEP)
        sweeps = plan.profile_work(lbx._native.LB_KERNEL_SWEEP) / (N * N) / n
        G, grad, rhoT = lbx.adjoint_gradient(plan, 0, alpha, r0, tar, beta, [1], 0.0, 0, want_rhoT=True)
        out[H] = (G.item(), grad.cpu().numpy(), rhoT.cpu().numpy(), sweeps)
    # forward sweeps per step: many steps took one sweep with the history
    assert out[6][3] < 1.95 and out[0][3] > 2.5, (out[6][3], out[0][3])
    assert rel_state_err([out[6][2]], [out[0][2]]) < STATE_TOL
    assert abs(out[6][0] - out[0][0]) <= 1e-12 * abs(out[0][0])
    assert np.max(np.abs(out[6][1] - out[0][1])) <= GRAD_TOL * np.max(np.abs(out[0][1]))
