"""Behaviour of the C ABI that the parity tests do not reach: the adjoint runs
in the autograd backward only, non-finite objectives are reported as
LB_ENONFINITE, and concurrent calls on one plan (separate streams and
workspaces, profiling on) give the results of the same calls made one after
another."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workloads import random_alpha, random_pure_states, random_system  # noqa: E402

from _gpu import dev, say  # noqa: E402


@pytest.fixture(scope="module")
def lbx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_10310_amd as lbx
    return lbx


def _case(seed, nlev, B=2, NT=16):
    rng = np.random.default_rng(seed)
    s = random_system(rng, nlev, NT=NT, T=0.1 * NT, Ns=5, Nf=2)
    alpha = random_alpha(rng, s, amp=0.02)
    return s, alpha, random_pure_states(rng, s.N, B), random_pure_states(rng, s.N, B), rng.uniform(0.5, 2, B)


@pytest.mark.parametrize("nlev", [(2, 3), (3, 3, 3, 3)])
def test_forward_with_grad_runs_no_adjoint_until_backward(lbx, nlev):
    # (2, 3) runs LDS-resident, (3, 3, 3, 3) streamed
    s, alpha, rho0, tar, beta = _case(500 + len(nlev), nlev)
    nat = lbx._native
    plan = lbx.Plan([s])
    plan.profile(True)
    for k in range(nat.LB_KERNEL_COUNT):
        plan.profile_read(k, reset=True)
    a = dev(alpha.reshape(-1)).requires_grad_(True)
    say("autograd forward only", nlev)
    G = lbx.lindblad_objective(a, plan, 0, dev(rho0), dev(tar), dev(beta), [2])
    torch.cuda.synchronize()
    assert plan.profile_read(nat.LB_KERNEL_LDS_ADJOINT)[0] == 0
    assert plan.profile_read(nat.LB_KERNEL_STREAM_GRAD)[0] == 0
    fwd = plan.profile_read(nat.LB_KERNEL_LDS_FORWARD)[0] + plan.profile_read(nat.LB_KERNEL_SWEEP)[0]
    assert fwd > 0
    G.sum().backward()
    torch.cuda.synchronize()
    adj = plan.profile_read(nat.LB_KERNEL_LDS_ADJOINT)[0] + plan.profile_read(nat.LB_KERNEL_STREAM_GRAD)[0]
    assert adj > 0 and a.grad is not None
    plan.profile(False)


def test_nonfinite_objective_is_reported(lbx):
    s, alpha, rho0, tar, beta = _case(510, (2, 3))
    nat = lbx._native
    plan = lbx.Plan([s])
    rhoT = rho0.copy()
    rhoT[1, 2, 3] = np.nan
    say("nonfinite objective")
    with pytest.raises(nat.LbxError) as e:
        lbx.objective(plan, 0, dev(rhoT), dev(tar), dev(beta), [2], 0.0, dev(alpha.reshape(-1)))
    assert e.value.code == nat.LB_ENONFINITE
    bad = rho0.copy()
    bad[0, 1, 1] = np.inf
    say("nonfinite gradient")
    with pytest.raises(nat.LbxError) as e:
        lbx.adjoint_gradient(plan, 0, dev(alpha.reshape(-1)), dev(bad), dev(tar), dev(beta), [2])
    assert e.value.code == nat.LB_ENONFINITE
    # the plan still works afterwards
    G, grad, _ = lbx.adjoint_gradient(plan, 0, dev(alpha.reshape(-1)), dev(rho0), dev(tar), dev(beta), [2])
    assert np.isfinite(G.cpu().numpy()).all() and torch.isfinite(grad).all()


def test_concurrent_calls_on_one_plan(lbx):
    """Two threads, each on its own stream with its own workspace, run
    gradients on one plan (an LDS-resident and a streamed system, profiling
    on) at the same time; each result equals the sequential one."""
    s1, a1, r1, t1, b1 = _case(520, (2, 3), NT=40)
    s2, a2, r2, t2, b2 = _case(521, (3, 3, 3, 3), NT=40)
    plan = lbx.Plan([s1, s2])
    plan.profile(True)
    batch = [2, 2]
    nat = lbx._native
    inputs = []
    for k in range(2):
        rng = np.random.default_rng(530 + k)
        al = np.concatenate([random_alpha(rng, s1, amp=0.02).reshape(-1), random_alpha(rng, s2, amp=0.02).reshape(-1)])
        rho = np.concatenate([random_pure_states(rng, s1.N, 2).reshape(-1), random_pure_states(rng, s2.N, 2).reshape(-1)])
        tar = np.concatenate([t1.reshape(-1), t2.reshape(-1)])
        inputs.append((dev(al), dev(rho), dev(tar), dev(np.concatenate([b1, b2]))))
    nbytes = plan.workspace_bytes(nat.LB_OP_GRADIENT, batch, 1)
    wss = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
    say("concurrent calls: sequential reference")
    ref = [lbx.adjoint_gradient(plan, 0, *inputs[k], batch, workspace=wss[k])[:2] for k in range(2)]
    ref = [(G.cpu().numpy(), g.cpu().numpy()) for G, g in ref]
    torch.cuda.synchronize()
    out = [None, None]
    err = []

    def run(k):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for _ in range(3):
                    G, g, _ = lbx.adjoint_gradient(plan, 0, *inputs[k], batch, workspace=wss[k])
                st.synchronize()
                out[k] = (G.cpu().numpy(), g.cpu().numpy())
        except Exception as ex:  # reported below
            err.append(ex)

    say("concurrent calls: two threads")
    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not err, err
    for k in range(2):
        assert np.array_equal(out[k][0], ref[k][0])
        assert np.array_equal(out[k][1], ref[k][1])
    plan.profile(False)
