"""imr_step_noalloc (the step on the library's static device scratch)
against imr_step with a workspace, on two calls in a row, the second with a
smaller batch: the same step to the state tolerance of the parity tests
(1e-12 relative per state)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workloads import random_alpha, random_system  # noqa: E402

from _gpu import dev, rel_state_err, say  # noqa: E402

STATE_TOL = 1e-12


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _states(rng, B, N):
    return rng.standard_normal((B, N, N)) + 1j * rng.standard_normal((B, N, N))


# (levels of the systems in the plan, system stepped): the block-tiled sweep
# kernel (five qutrits) and the generic one on the second system of a plan
CASES = [([(3,) * 5], 0), ([(4, 4), (2, 3)], 1)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("adjoint", [False, True])
def test_noalloc_step_matches_workspace_step_twice(lbx, case, adjoint):
    shapes, sys = case
    rng = np.random.default_rng(4242 + sys)
    systems = [random_system(rng, nl, NT=12, T=1.2, Ns=5, Nf=2) for nl in shapes]
    s = systems[sys]
    alpha = dev(random_alpha(rng, s, amp=0.02).reshape(-1))
    plan = lbx.Plan(systems)
    for call, (B, j) in enumerate([(6, 5), (2, 9)]):
        q = dev(_states(rng, B, s.N))
        say("imr_step_noalloc", shapes, sys, adjoint, "call", call, "B", B)
        out = torch.empty_like(q)
        lbx.imr_step_noalloc(plan, sys, j, alpha, q, out, adjoint=adjoint)
        ref = lbx.imr_step(plan, sys, j, alpha, q, adjoint=adjoint)
        assert rel_state_err(out.cpu().numpy(), ref.cpu().numpy()) < STATE_TOL


@pytest.mark.parametrize("adjoint", [False, True])
def test_noalloc_step_with_coupling(lbx, adjoint):
    # a Jaynes-Cummings coupled system (generic sweep kernel with the coupling
    # terms and its contraction bound), two calls, the second smaller
    rng = np.random.default_rng(4300)
    s = random_system(rng, (3, 2, 2), NT=12, T=1.2, Ns=5, Nf=2, jc=0.04)
    alpha = dev(random_alpha(rng, s, amp=0.02).reshape(-1))
    plan = lbx.Plan([s])
    for call, (B, j) in enumerate([(5, 3), (2, 8)]):
        q = dev(_states(rng, B, s.N))
        say("imr_step_noalloc coupled", adjoint, "call", call, "B", B)
        out = torch.empty_like(q)
        lbx.imr_step_noalloc(plan, 0, j, alpha, q, out, adjoint=adjoint)
        ref = lbx.imr_step(plan, 0, j, alpha, q, adjoint=adjoint)
        assert rel_state_err([out.cpu().numpy()], [ref.cpu().numpy()]) < STATE_TOL


def test_noalloc_step_async_status(lbx):
    """With LB_OPT_SYNC off the call only enqueues; lb_status(plan, NULL)
    then reads the status of the last call on the device: clean with enough
    launched sweeps, LB_EUNSUPPORTED (a step needed more) with two."""
    rng = np.random.default_rng(77)
    s = random_system(rng, (2, 3), NT=12, T=1.2, Ns=5, Nf=2)
    alpha = dev(random_alpha(rng, s, amp=0.02).reshape(-1))
    plan = lbx.Plan([s])
    nat = lbx._native
    q = dev(_states(rng, 3, s.N))
    out = torch.empty_like(q)
    plan.set_option(nat.LB_OPT_SYNC, 0)
    plan.set_option(nat.LB_OPT_SWEEPS, 40)
    say("imr_step_noalloc async, 40 sweeps")
    lbx.imr_step_noalloc(plan, 0, 3, alpha, q, out)
    plan.status(None)
    plan.set_option(nat.LB_OPT_SYNC, 1)
    ref = lbx.imr_step(plan, 0, 3, alpha, q)
    assert rel_state_err(out.cpu().numpy(), ref.cpu().numpy()) < STATE_TOL
    plan.set_option(nat.LB_OPT_SYNC, 0)
    plan.set_option(nat.LB_OPT_SWEEPS, 2)
    say("imr_step_noalloc async, 2 sweeps")
    lbx.imr_step_noalloc(plan, 0, 3, alpha, q, out)
    with pytest.raises(nat.LbxError) as e:
        plan.status(None)
    assert e.value.code == nat.LB_EUNSUPPORTED
    plan.set_option(nat.LB_OPT_SYNC, 1)
    say("imr_step_noalloc sync retry, 2 sweeps")
    lbx.imr_step_noalloc(plan, 0, 3, alpha, q, out)
    assert rel_state_err(out.cpu().numpy(), ref.cpu().numpy()) < STATE_TOL


def test_noalloc_step_rejects_batches_beyond_the_scratch(lbx):
    rng = np.random.default_rng(5)
    s = random_system(rng, (3,) * 5, NT=4, T=0.4, Ns=5, Nf=1)
    alpha = dev(random_alpha(rng, s, amp=0.02).reshape(-1))
    plan = lbx.Plan([s])
    B = lbx._native.LB_NOALLOC_MAX_ENTRIES // (s.N * s.N) + 1
    q = torch.zeros((B, s.N, s.N), dtype=torch.complex128, device="cuda")
    out = torch.empty_like(q)
    say("imr_step_noalloc over the limit", B)
    with pytest.raises(lbx._native.LbxError) as e:
        lbx.imr_step_noalloc(plan, 0, 1, alpha, q, out)
    assert e.value.code == lbx._native.LB_EINVAL
    assert "scratch" in str(e.value)
