#!/usr/bin/env python3
"""Throughput of the Lindblad optimal-control hot path on one MI355X.

Workload (one "step" = one forward + adjoint gradient evaluation): two
coupled transmons with 4 levels each (N = 16), all 16 basis density matrices
of the 2x2 essential subspace batched, CNOT target, Frobenius merit,
20 B-splines x 2 carriers per control (160 real coefficients), T = 200 ns,
10000 implicit-midpoint steps.  Inputs are seeded and synthetic and already
resident in GPU memory when the timed region starts.

Printed as one JSON line:
  value          gradient evaluations per second,
  roofline       the dominant kernel of the step (the LDS-resident adjoint
                 time loop), algorithmic FP64 flops per launch over its
                 HIP-event duration, against the FP64 vector peak,
  apply_roofline lindblad_apply on the eight-qutrit ring (N = 6561,
                 43,046,721 entries per state), algorithmic bytes (read x,
                 write y: 32 B per entry) over its HIP-event duration,
                 against the HBM peak,
  per_state_loop the same gradient with one state at a time through the
                 streaming kernels (one launch per sweep), for the speedup of
                 batching and persistence,
  cpu_baseline   the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector, dense
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
APPLY_SOURCES = ["paper_2110_10310_amd/csrc/kernels_stream.hip",
                 "paper_2110_10310_amd/csrc/lbx_device.hpp"]
LDS_SOURCES = ["paper_2110_10310_amd/csrc/kernels_lds.hip",
               "paper_2110_10310_amd/csrc/lbx_device.hpp"]


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key, files, launches_per_unit=1):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_sha(files):
        return None
    return rec.get("bytes_per_launch")


def neighbour_counts(nlev):
    """Mean number of existing control neighbours (row and column ladder
    shifts) and decay-jump neighbours per entry, summed over subsystems."""
    ctl = jump = 0.0
    for n in nlev:
        ex_p = (n - 1) / n   # digit can move up
        ex_m = (n - 1) / n   # digit can move down
        ctl += 2 * (ex_p + ex_m)
        jump += ex_p * ex_p
    return ctl, jump


def flops_per_entry(nlev):
    """Algorithmic FP64 flops per entry: one stage sweep, and the per-step
    adjoint extras (gradient integrands, stage start, state update)."""
    ctl, jump = neighbour_counts(nlev)
    sweep = 8 * ctl + 4 * jump + 10          # complex MACs + (q + h acc) * w
    grad = 4 * ctl + 12 * len(nlev) + 14     # U, V, S, D, gp, gq; z, qh, w*qh
    return sweep, grad


def run_gradient_bench(lbx, torch, steps, warmup):
    from workloads import make_config
    p = make_config(2)
    s = p.systems[0]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda")
    alpha = dev(p.alpha[0].reshape(-1))
    rho0, tar, beta = dev(p.rho0[0]), dev(p.rhotar[0]), dev(p.beta[0])
    plan = lbx.Plan([s])
    B = rho0.shape[0]
    batch = [B]
    for _ in range(warmup):
        lbx.adjoint_gradient(plan, p.kind, alpha, rho0, tar, beta, batch)
    plan.profile(True)
    for k in range(4):
        plan.profile_read(k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        G, grad, _ = lbx.adjoint_gradient(plan, p.kind, alpha, rho0, tar, beta, batch)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nat = lbx._native
    n_f, ms_f = plan.profile_read(nat.LB_KERNEL_LDS_FORWARD)
    n_a, ms_a = plan.profile_read(nat.LB_KERNEL_LDS_ADJOINT)
    plan.profile(False)
    counts = lbx.sweep_counts(plan, alpha)[0, :, 0].astype(np.int64)
    entries = B * s.N * s.N
    f_sweep, f_grad = flops_per_entry(s.nlev)
    fl_fwd = float(counts.sum()) * entries * f_sweep
    fl_adj = fl_fwd + s.NT * entries * f_grad
    if ms_a >= ms_f:
        name, n, ms, fl = "lds_adjoint_kernel", n_a, ms_a, fl_adj
    else:
        name, n, ms, fl = "lds_forward_kernel", n_f, ms_f, fl_fwd
    avg_s = ms / max(n, 1) / 1e3
    achieved = fl / avg_s / 1e12
    traffic = measured_traffic(name, LDS_SOURCES)
    return {
        "value": steps / elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "G": float(G.item()),
        "grad_norm": float(grad.abs().max().item()),
        "sweeps_per_step_mean": float(counts.mean()),
        "roofline": {
            "kernel": name, "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
            "avg_launch_ms": 1e3 * avg_s, "launches": n, "flops_per_launch": fl,
            "workgroups": B, "note": "one workgroup per state: 16 of 256 CUs busy",
        },
        "kernel_ms": {"lds_forward_kernel": ms_f / max(n_f, 1), "lds_adjoint_kernel": ms_a / max(n_a, 1)},
    }


def run_apply_bench(lbx, torch, reps):
    from workloads import make_config
    p = make_config(5)
    s = p.systems[0]
    plan = lbx.Plan([s])
    N = s.N
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    y = torch.empty_like(x)
    alpha = torch.as_tensor(p.alpha[0].reshape(-1)).to("cuda")
    out = {}
    for adj in (False, True):
        for _ in range(3):
            lbx.lindblad_apply(plan, 0, 41.0, alpha, x, adjoint=adj, out=y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for k in range(reps):
            ev[k][0].record()
            lbx.lindblad_apply(plan, 0, 41.0 + 0.01 * k, alpha, x, adjoint=adj, out=y)
            ev[k][1].record()
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        out["adjoint" if adj else "forward"] = ms
    algo = 32.0 * N * N
    ms = out["forward"]
    achieved = algo / (ms / 1e3) / 1e9
    traffic = measured_traffic("apply_kernel_forward", APPLY_SOURCES)
    return {
        "kernel": "apply_kernel<forward>", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
        "avg_launch_ms": ms, "adjoint_avg_launch_ms": out["adjoint"],
        "adjoint_achieved": algo / (out["adjoint"] / 1e3) / 1e9,
        "bytes_per_launch": algo, "workload": "8 qutrits ring, N=6561, 1 state",
    }


def run_loop_baseline(lbx, torch, nsteps):
    """Per-state streaming loop: one state at a time, one launch per sweep."""
    from workloads import make_config, truncate_steps
    p = truncate_steps(make_config(2), nsteps)
    s = p.systems[0]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda")
    plan = lbx.Plan([s], path="stream")
    alpha = dev(p.alpha[0].reshape(-1))
    states = [(dev(p.rho0[0][b:b + 1]), dev(p.rhotar[0][b:b + 1]), dev(p.beta[0][b:b + 1]))
              for b in range(p.rho0[0].shape[0])]
    lbx.adjoint_gradient(plan, p.kind, alpha, *states[0], [1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r0, t, b in states:
        lbx.adjoint_gradient(plan, p.kind, alpha, r0, t, b, [1])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    scale = make_config(2).systems[0].NT / nsteps
    return {"evals_per_s": 1.0 / (el * scale),
            "sample": f"16 states one by one, streaming path, {nsteps} of 10000 steps, time x{scale:g}"}


def run_cpu_baseline(nsteps):
    import oracle
    from workloads import make_config, truncate_steps
    p = truncate_steps(make_config(2), nsteps)
    s = p.systems[0]
    t0 = time.perf_counter()
    oracle.value_and_gradient(s, p.alpha[0], p.rho0[0], p.rhotar[0], p.beta[0], p.kind)
    el = time.perf_counter() - t0
    scale = make_config(2).systems[0].NT / nsteps
    return {"value": 1.0 / (el * scale), "unit": "evals/s", "cores": oracle.lindblad.ORACLE_BLAS_THREADS,
            "kind": "oracle",
            "sample": f"two-transmon CNOT, 16 states, {nsteps} of 10000 steps ({el:.1f} s), scaled x{scale:g}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--loop-steps", type=int, default=250)
    ap.add_argument("--cpu-steps", type=int, default=800)
    ap.add_argument("--no-apply", action="store_true")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the batch of states would shard over GPUs with one all-reduce of G and dG/dalpha).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2110_10310_amd as lbx
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    print("[bench] gradient evaluations", file=sys.stderr, flush=True)
    res = run_gradient_bench(lbx, torch, args.steps, args.warmup)
    line = {
        "metric": "forward+adjoint gradient evals/sec; lindblad_apply HBM GB/s vs peak",
        "value": res["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "c2_cnot_2x4: 2 transmons x 4 levels (N=16), 16 basis states, "
                               "10000 IMR steps, 160 controls, J_Frob, forward+adjoint gradient",
                   "global_batch": 16, "parallelism": "single GPU"},
        "roofline": res["roofline"],
        "detail": {"G": res["G"], "grad_max": res["grad_norm"],
                   "sweeps_per_step_mean": res["sweeps_per_step_mean"],
                   "kernel_avg_ms": res["kernel_ms"]},
    }
    if not args.no_apply:
        print("[bench] lindblad_apply 8 qutrits", file=sys.stderr, flush=True)
        line["apply_roofline"] = run_apply_bench(lbx, torch, args.apply_reps)
    if not args.no_loop:
        print("[bench] per-state loop baseline", file=sys.stderr, flush=True)
        lb = run_loop_baseline(lbx, torch, args.loop_steps)
        lb["speedup"] = res["value"] / lb["evals_per_s"]
        line["per_state_loop"] = lb
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = run_cpu_baseline(args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
