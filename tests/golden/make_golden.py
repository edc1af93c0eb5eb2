"""Write the expected values of the workloads' parity fixtures.

Calls only the CPU oracle (and the seeded input generator); nothing here
touches the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py [c2|c3|c4|c5|all] [processes]

Each target writes tests/golden/<name>.npz:

* c2_cnot_full      the two-transmon CNOT at its full 10000 steps: rho(T) of
                    the 16 basis states, G and dG/dalpha.  A few minutes.
* c3_uneven_nt20    all 96 systems of the uneven batch over their first 20
                    steps: G and dG/dalpha per system, and sampled entries,
                    trace and Frobenius norm of every rho(T).  About two
                    CPU-hours.
* c4_chain_nt400    the five-qutrit chain (10 states) over its first 400
                    steps: G, dG/dalpha, sampled entries, traces and norms of
                    rho(T).  About two CPU-hours.
* c5_ring_nt2       the eight-qutrit ring shortened to 2 steps (T = 2 dt, the
                    controls' splines over that horizon), from |0..0> and from
                    one seeded random pure state (random target):
                    G, dG/dalpha, sampled entries, traces and norms of rho(T).
                    About an hour and 20 GB of memory per state.  (From
                    |0..0> alone the 2-step gradient is 2.6e-11, eleven orders
                    below G, a sum of cancelling terms whose rounding floor in
                    FP64 is about 1e-19; the random state makes it large.)

The states of a workload are evaluated one per task over a process pool
(default: the CPU count less two).

Sampled entries are taken at seeded positions (the positions are stored).
A truncated workload keeps the step size and the inputs of the full one
(workloads.truncate_steps): the horizon is shortened, so the control
B-splines span the shorter horizon.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import make_config, truncate_steps, with_random_states  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (workload, steps kept, sampled entries per state, name, extra random states)
TARGETS = {
    "c3": (3, 20, 8, "c3_uneven_nt20", 0),
    "c4": (4, 400, 64, "c4_chain_nt400", 0),
    "c5": (5, 2, 512, "c5_ring_nt2", 1),
}
EXTRA_SEED = 5150  # seed of the extra random states


def problem(cfg, nt, extra):
    """The truncated workload, with `extra` random states per system."""
    p = make_config(cfg)
    if extra:
        p = with_random_states(p, extra, EXTRA_SEED)
    return truncate_steps(p, nt)


def make_c2():
    p = make_config(2)
    s = p.systems[0]
    t0 = time.time()
    G, grad, rhoT = oracle.value_and_gradient(s, p.alpha[0], p.rho0[0], p.rhotar[0], p.beta[0],
                                              p.kind, p.gamma2, return_final=True)
    out = os.path.join(HERE, "c2_cnot_full.npz")
    np.savez_compressed(out, rhoT=rhoT, G=np.array(G), grad=grad,
                        seed=np.array(20211020 + 2), NT=np.array(s.NT))
    print(f"wrote {out}: G={G:.16e} |grad|max={np.abs(grad).max():.6e} in {time.time() - t0:.1f}s")


def _one_state(args):
    """The oracle's G and gradient of one state of one system (weight beta_b,
    no regularisation) and its rho(T)."""
    cfg, nt, extra, k, b = args
    p = problem(cfg, nt, extra)
    s = p.systems[k]
    g, gr, rhoT = oracle.value_and_gradient(s, p.alpha[k], p.rho0[k][b:b + 1], p.rhotar[k][b:b + 1],
                                            p.beta[k][b:b + 1], p.kind, 0.0, return_final=True)
    return k, b, g, np.asarray(gr), rhoT[0]


def make_truncated(key, procs):
    """G of a system is the mean over its states of beta_b J_b plus the
    Tikhonov term (eq. optimproblem), and its gradient the mean of the
    states' gradients plus gamma2 alpha: the states are evaluated one per
    task, over `procs` processes."""
    import multiprocessing as mp
    cfg, nt, nsamp, name, extra = TARGETS[key]
    p = problem(cfg, nt, extra)
    tasks = [(cfg, nt, extra, k, b) for k in range(len(p.systems)) for b in range(p.rho0[k].shape[0])]
    # largest systems first, so the pool ends together
    tasks.sort(key=lambda a: -p.systems[a[3]].N)
    t0 = time.time()
    res = {}
    with mp.get_context("spawn").Pool(procs) as pool:
        for n, (k, b, g, gr, rT) in enumerate(pool.imap_unordered(_one_state, tasks)):
            res[(k, b)] = (g, gr, rT)
            if n % 10 == 0 or n == len(tasks) - 1:
                print(f"  {n + 1}/{len(tasks)} states ({time.time() - t0:.0f}s)", flush=True)
    rng = np.random.default_rng(777 + cfg)
    G, grads = [], []
    si, sb, sr, sc, sv = [], [], [], [], []
    tr, fro = [], []
    for k, s in enumerate(p.systems):
        B = p.rho0[k].shape[0]
        a = np.asarray(p.alpha[k])
        G.append(sum(res[(k, b)][0] for b in range(B)) / B + 0.5 * p.gamma2 * float(np.sum(a ** 2)))
        grads.append((sum(res[(k, b)][1] for b in range(B)) / B + p.gamma2 * a).reshape(-1))
        for b in range(B):
            rT = res[(k, b)][2]
            r = rng.integers(0, s.N, nsamp)
            c = rng.integers(0, s.N, nsamp)
            si += [k] * nsamp
            sb += [b] * nsamp
            sr.append(r)
            sc.append(c)
            sv.append(rT[r, c])
            tr.append(np.trace(rT))
            fro.append(np.linalg.norm(rT))
    out = os.path.join(HERE, name + ".npz")
    np.savez_compressed(out, G=np.array(G), grad=np.concatenate(grads), NT=np.array(nt),
                        config=np.array(cfg), extra=np.array(extra), extra_seed=np.array(EXTRA_SEED),
                        samp_sys=np.array(si), samp_state=np.array(sb),
                        samp_row=np.concatenate(sr), samp_col=np.concatenate(sc),
                        samp_val=np.concatenate(sv), trace=np.array(tr), fro=np.array(fro))
    print(f"wrote {out}: {len(p.systems)} systems, |grad|max={np.abs(np.concatenate(grads)).max():.6e} "
          f"in {time.time() - t0:.1f}s")


def main():
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else max(1, (os.cpu_count() or 2) - 2)
    keys = ["c2", "c3", "c4", "c5"] if which == "all" else [which]
    for k in keys:
        if k == "c2":
            make_c2()
        else:
            make_truncated(k, procs)


if __name__ == "__main__":
    main()
