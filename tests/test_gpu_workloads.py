"""GPU parity at the named workloads' own inputs (eqs. IMR, linsystem_primal,
linsystem_adjoint and the reduced gradient of App. A/B).

* Stored oracle values (tests/golden/make_golden.py, oracle only): the whole
  uneven batch of 96 systems over its first 20 steps, the five-qutrit chain
  over 400 steps with checkpoints every 200, and the eight-qutrit ring over
  2 steps from |0..0> and from a seeded random pure state.  G within 1e-12 relative, the gradient within 1e-10 of its
  max-norm, sampled entries of rho(T) within 1e-12 of each state's
  Frobenius norm, traces and norms within 1e-12 relative.
* The eight-qutrit ring's implicit-midpoint step (forward and adjoint) at
  its full size, checked through the stage equation
  z - dt/2 M z = q at sampled entries, with M z formed entry by entry by the
  oracle.
* The LDS-resident kernels specialised for four subsystems.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from workloads import (  # noqa: E402
    make_config, random_alpha, random_pure_states, random_system, truncate_steps, with_random_states,
)

from _gpu import dev, flat_alpha, flat_states, rel_state_err, say, split_states  # noqa: E402

STATE_TOL = 1e-12
GRAD_TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _check_against_golden(lbx, name, ckpt):
    gold = np.load(os.path.join(GOLDEN, name + ".npz"))
    cfg, nt = int(gold["config"]), int(gold["NT"])
    p = make_config(cfg)
    if "extra" in gold.files and int(gold["extra"]) > 0:
        p = with_random_states(p, int(gold["extra"]), int(gold["extra_seed"]))
    p = truncate_steps(p, nt)
    plan = lbx.Plan(p.systems)
    alpha = dev(flat_alpha(p.alpha))
    say(name, "systems", len(p.systems), "steps", nt, "ckpt", ckpt)
    G, grad, rhoT = lbx.adjoint_gradient(plan, p.kind, alpha, dev(flat_states(p.rho0)), dev(flat_states(p.rhotar)),
                                         dev(np.concatenate(p.beta)), p.batch, p.gamma2, ckpt, want_rhoT=True)
    G = G.cpu().numpy()
    grad = grad.cpu().numpy()
    Gr = gold["G"]
    assert np.max(np.abs(G - Gr) / np.abs(Gr)) <= 1e-12, np.max(np.abs(G - Gr) / np.abs(Gr))
    off = 0
    for k, a in enumerate(p.alpha):
        gk, rk = grad[off:off + a.size], gold["grad"][off:off + a.size]
        assert np.max(np.abs(gk - rk)) <= GRAD_TOL * np.max(np.abs(rk)), (k, np.max(np.abs(gk - rk)))
        off += a.size
    states = split_states(rhoT.cpu().numpy(), p.systems, p.batch)
    del rhoT
    tr, fro = [], []
    for st in states:
        for b in range(st.shape[0]):
            tr.append(np.trace(st[b]))
            fro.append(np.linalg.norm(st[b]))
    tr, fro = np.array(tr), np.array(fro)
    assert np.max(np.abs(fro - gold["fro"]) / gold["fro"]) <= STATE_TOL
    assert np.max(np.abs(tr - gold["trace"]) / gold["fro"]) <= STATE_TOL
    # sampled entries, each against its state's Frobenius norm
    first = np.cumsum([0] + [st.shape[0] for st in states])
    got = np.array([states[k][b, i, j] for k, b, i, j in
                    zip(gold["samp_sys"], gold["samp_state"], gold["samp_row"], gold["samp_col"])])
    scale = gold["fro"][first[gold["samp_sys"]] + gold["samp_state"]]
    assert np.max(np.abs(got - gold["samp_val"]) / scale) <= STATE_TOL


def test_uneven_batch_all_96_systems_20_steps(lbx):
    _check_against_golden(lbx, "c3_uneven_nt20", 0)


def test_five_qutrit_chain_400_steps_checkpoints_every_200(lbx):
    _check_against_golden(lbx, "c4_chain_nt400", 200)


def test_eight_qutrit_ring_two_steps(lbx):
    if not os.path.exists(os.path.join(GOLDEN, "c5_ring_nt2.npz")):
        pytest.skip("c5_ring_nt2.npz not written yet (tests/golden/make_golden.py c5)")
    _check_against_golden(lbx, "c5_ring_nt2", 0)


@pytest.mark.parametrize("adjoint", [False, True])
def test_eight_qutrit_ring_step_solves_its_stage_equation(lbx, adjoint):
    """imr_step at N = 6561 with the block-tiled sweep kernels (Q = 8): with
    out = q + dt M z (eq. IMR), z = (q + out) / 2 must satisfy
    z - dt/2 M z = q (eq. linsystem_primal; M^+ for the adjoint step,
    eq. linsystem_adjoint) at 96 sampled entries."""
    p = make_config(5)
    s = p.systems[0]
    N = s.N
    j = 1234
    g = torch.Generator(device="cuda")
    g.manual_seed(61)
    q = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    plan = lbx.Plan([s])
    say("eight-qutrit imr_step", adjoint)
    out = lbx.imr_step(plan, 0, j, dev(p.alpha[0].reshape(-1)), q, adjoint=adjoint)
    z = ((q + out) * 0.5)[0].cpu().numpy()
    qn = q[0].cpu().numpy()
    del q, out
    rng = np.random.default_rng(62)
    rows = rng.integers(0, N, 96)
    cols = rng.integers(0, N, 96)
    t = (j + 0.5) * s.dt
    Mz = oracle.lindbladian_entries(s, p.alpha[0], t, z, rows, cols, adjoint=adjoint)
    res = z[rows, cols] - 0.5 * s.dt * Mz - qn[rows, cols]
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(qn[rows, cols]))
    # the step moved the state: the check is not vacuous
    assert np.max(np.abs(z[rows, cols] - qn[rows, cols])) > 1e-4


def test_lds_kernels_for_four_subsystems(lbx):
    """Four two-level subsystems (N^2 = 256): the LDS-resident kernels
    specialised for Q = 4, forward and adjoint, against the oracle."""
    rng = np.random.default_rng(140)
    s = random_system(rng, (2, 2, 2, 2), NT=16, T=1.6, Ns=5, Nf=2)
    alpha = random_alpha(rng, s, amp=0.02)
    B = 3
    rho0 = random_pure_states(rng, s.N, B)
    tar = random_pure_states(rng, s.N, B)
    beta = rng.uniform(0.5, 2, B)
    plan = lbx.Plan([s], path="lds")
    say("lds four subsystems")
    G, grad, rhoT = lbx.adjoint_gradient(plan, 0, dev(alpha.reshape(-1)), dev(rho0), dev(tar), dev(beta), [B],
                                         0.0, 1, want_rhoT=True)
    Gr, gr = oracle.value_and_gradient(s, alpha, rho0, tar, beta, 0)
    rT = oracle.imr_forward(s, alpha, rho0)
    assert rel_state_err([rhoT.cpu().numpy().reshape(B, s.N, s.N)], [rT]) < STATE_TOL
    assert abs(G.item() - Gr) <= 1e-12 * abs(Gr)
    assert np.max(np.abs(grad.cpu().numpy().reshape(gr.shape) - gr)) <= GRAD_TOL * np.max(np.abs(gr))
