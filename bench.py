#!/usr/bin/env python3
"""Throughput of the Lindblad optimal-control hot path on one MI355X.

Headline workload: the eight-qutrit ring (N = 6561, 43,046,721 complex FP64
entries per state, 689 MB), one state |0..0>, J_Frob to |1..1>, 20
B-splines per control, T = 100 ns, 5000 implicit-midpoint steps, forward
pass plus discrete-adjoint gradient with checkpoints every ceil(sqrt(5000))
= 71 steps recomputed in the adjoint.  One bench step is one gradient
evaluation of that system over its whole horizon: control table, forward
pass with checkpoints, objective, adjoint with recomputation and gradient
contraction (about 90 s).  Inputs are seeded and synthetic and already
resident in GPU memory when the timed region starts.  `--window W` times W
steps instead, with the horizon shortened to W dt: the B-spline controls
then vary faster per step than in the workload (more stage sweeps per step),
so such a line is a quick look, not the workload's rate.

Printed as one JSON line:
  value          c5 gradient evaluations per second,
  roofline       the dominant kernel: the block-tiled stage sweep, 48
                 algorithmic bytes per entry and executed sweep (read the
                 iterate and q, write the next iterate) over the HIP-event
                 time of the streamed steps, against the HBM peak,
  apply_roofline lindblad_apply on the same state, 32 B per entry (read x,
                 write y), against the HBM peak,
  c2_cnot        the two-transmon CNOT gradient (N = 16, 16 states, 10000
                 steps) with its LDS-resident roofline, the per-state loop
                 speedup and its own CPU baseline,
  cpu_baseline   the CPU oracle on a bounded sample of the headline workload,
                 one process per core of the box's share.
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
                 "paper_2110_10310_amd/csrc/kernels_tile.hip",
                 "paper_2110_10310_amd/csrc/lbx_device.hpp"]
STEP_SOURCES = ["paper_2110_10310_amd/csrc/kernels_step.hip",
                "paper_2110_10310_amd/csrc/tile_unit.hpp"]
LDS_SOURCES = ["paper_2110_10310_amd/csrc/kernels_lds.hip",
               "paper_2110_10310_amd/csrc/kernels_lds_fast.hip",
               "paper_2110_10310_amd/csrc/lbx_device.hpp"]
# traffic keys: (substrings of the kernel name in the counter CSV, sources it is built from)
TILE_KIS = {44: 512, 43: 256, 34: 256, 33: 256, 32: 256, 23: 256}  # eight-qutrit block shapes, threads
TRAFFIC_KEYS = {
    "lds_forward_kernel": (["lds_forward_fast_kernel"], LDS_SOURCES),
    "lds_adjoint_kernel": (["lds_adjoint_fast_kernel"], LDS_SOURCES),
    "lds_adjoint_integrands": (["lds_grad_fast_kernel"], LDS_SOURCES),
}
for _ki, _thr in TILE_KIS.items():
    _tail = f"<3, 8, {_ki // 10}, {_ki % 10}"
    TRAFFIC_KEYS[f"apply_kernel_forward_ki{_ki}"] = ([f"lbx::tile_kernel{_tail}, false, {_thr}>"], APPLY_SOURCES)
    TRAFFIC_KEYS[f"apply_kernel_adjoint_ki{_ki}"] = ([f"lbx::tile_kernel{_tail}, true, {_thr}>"], APPLY_SOURCES)
    # executed launches only (a launch after the step's solve has converged
    # returns at once and moves nothing)
    TRAFFIC_KEYS[f"stage_sweep_c5_ki{_ki}"] = ([f"lbx::sweep_tile_kernel{_tail}, "], APPLY_SOURCES + STEP_SOURCES,
                                               "executed")


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key, files, traffic_file=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(traffic_file or TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_sha(files):
        return None
    return rec.get("bytes_per_launch")


def with_traffic_rate(roof):
    """Add the counter-measured HBM rate to a roofline object that holds a
    `traffic` figure (bytes per launch from the rocprofv3 counters) and an
    average launch duration: traffic_GBps and its fraction of the peak,
    beside the algorithmic `achieved` (whose gap to it is the extra traffic
    of the tiling)."""
    if roof and roof.get("traffic") and roof.get("avg_launch_ms") and roof.get("unit") == "GB/s":
        rate = roof["traffic"] / (roof["avg_launch_ms"] / 1e3) / 1e9
        roof["traffic_GBps"] = rate
        roof["traffic_frac"] = rate / roof["peak"]
    return roof


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


WORKLOADS = {
    1: "c1_qutrit: 1 qutrit (N=3), 1 state, 2000 IMR steps, 20 controls, J_Frob",
    2: "c2_cnot_2x4: 2 transmons x 4 levels (N=16), 16 basis states, 10000 IMR steps, "
       "160 controls, J_Frob, forward+adjoint gradient",
    3: "c3_uneven_96: 96 systems of 2-4 qudits with 3-5 levels (N 9..500), 1-8 states each, "
       "5000 IMR steps, J_Frob",
    4: "c4_5qutrit_chain: 5 qutrits (N=243), 10 states, 20000 IMR steps, 300 controls, J_Tr, "
       "checkpoints every 200 steps",
    5: "c5_8qutrit_ring: 8 qutrits (N=6561, 43M entries), 1 state, 5000 IMR steps, 320 controls, "
       "J_Frob, checkpoints every ceil(sqrt(5000)) = 71 steps",
}


HEADLINE = 5
WORKLOADS_NT = {1: 2000, 2: 10000, 3: 5000, 4: 20000, 5: 5000}
DEFAULT_STEPS = {1: 20, 2: 20, 3: 1, 4: 3, 5: 1}   # timed evaluations (about a minute or less)


LDS_MAX_N2 = 4096   # systems up to this N^2 run LDS-resident (every state kept, no recomputation)


def window_ckpt(p):
    """Checkpoint interval that gives a window of the horizon the segments of
    the full evaluation: the workload's own, or, where every system streams,
    the library's automatic ceil(sqrt(NT)) of the full horizon made explicit.
    (An explicit interval above 1 would move LDS-resident systems to the
    streamed path, so mixed workloads keep the automatic choice.)"""
    import math
    if p.ckpt_every > 0:
        return p.ckpt_every
    if all(s.N * s.N > LDS_MAX_N2 for s in p.systems):
        return max(1, math.ceil(math.sqrt(p.systems[0].NT)))
    return 0


def run_gradient_bench(lbx, torch, steps, warmup, workload=HEADLINE, window=0):
    from workloads import make_config, truncate_steps
    p = make_config(workload)
    nt_full = p.systems[0].NT
    ckpt = p.ckpt_every
    if window and window < nt_full:
        ckpt = window_ckpt(p)
        p = truncate_steps(p, window)
        ckpt = min(ckpt, window)
    nat = lbx._native
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda")
    alpha = dev(np.concatenate([a.reshape(-1) for a in p.alpha]))
    rho0 = dev(np.concatenate([r.reshape(-1) for r in p.rho0]))
    tar = dev(np.concatenate([r.reshape(-1) for r in p.rhotar]))
    beta = dev(np.concatenate(p.beta))
    batch = p.batch
    plan = lbx.Plan(p.systems)
    tuned = plan.autotune(alpha, batch)
    for k in range(warmup):
        lbx.adjoint_gradient(plan, p.kind, alpha, rho0, tar, beta, batch, p.gamma2, ckpt)
        print(f"[bench] warm-up evaluation {k + 1} of {warmup} done", file=sys.stderr, flush=True)
    plan.profile(True)
    for k in range(4):
        plan.profile_read(k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        G, grad, _ = lbx.adjoint_gradient(plan, p.kind, alpha, rho0, tar, beta, batch, p.gamma2, ckpt)
        if steps <= 5:  # evaluations of a minute or more: name each one
            print(f"[bench] evaluation {k + 1} of {steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {k: plan.profile_read(k) for k in range(4)}
    work = {k: plan.profile_work(k) for k in range(4)}
    plan.profile(False)
    counts = lbx.sweep_counts(plan, alpha)  # [nsys, NT, 2], a-priori
    # Algorithmic flops of the LDS-resident kernels: entry-sweeps done (read
    # back from the kernels) times flops per entry and sweep, averaged over
    # the systems with their a-priori sweep counts as weights.
    wsum = fsum = grad_fl = 0.0
    lds_entries = st_entries = 0
    for k, s in enumerate(p.systems):
        entries = batch[k] * s.N * s.N
        if s.N * s.N <= LDS_MAX_N2 and ckpt <= 1:
            f_sweep, f_grad = flops_per_entry(s.nlev)
            wk = float(counts[k, :, 0].sum()) * entries
            wsum += wk
            fsum += wk * f_sweep
            grad_fl += s.NT * entries * f_grad
            lds_entries += entries
        else:
            st_entries += entries
    f_avg = fsum / wsum if wsum else 0.0
    lds_fwd = work[nat.LB_KERNEL_LDS_FORWARD] * f_avg / steps
    lds_adj = work[nat.LB_KERNEL_LDS_ADJOINT] * f_avg / steps + grad_fl
    n = {k: max(v[0], 1) for k, v in prof.items()}
    ms = {k: v[1] for k, v in prof.items()}
    name_of = {nat.LB_KERNEL_LDS_FORWARD: "lds_forward_kernel", nat.LB_KERNEL_LDS_ADJOINT: "lds_adjoint_kernel",
               nat.LB_KERNEL_SWEEP: "stage_sweep_kernel", nat.LB_KERNEL_STREAM_GRAD: "stream_grad_kernel"}
    dom = max(ms, key=lambda k: ms[k])
    avg_s = ms[dom] / n[dom] / 1e3
    if dom in (nat.LB_KERNEL_LDS_FORWARD, nat.LB_KERNEL_LDS_ADJOINT):
        fl = (lds_fwd if dom == nat.LB_KERNEL_LDS_FORWARD else lds_adj) / (n[dom] / steps)
        achieved = fl / avg_s / 1e12
        # The counters were taken on the two-transmon gradient; an adjoint
        # launch of the family is the adjoint kernel plus its integrand kernel.
        traffic = measured_traffic(name_of[dom], LDS_SOURCES) if workload == 2 else None
        if traffic is not None and dom == nat.LB_KERNEL_LDS_ADJOINT:
            extra = measured_traffic("lds_adjoint_integrands", LDS_SOURCES)
            traffic = traffic + extra if extra is not None else None
        roof = {"kernel": name_of[dom], "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": traffic,
                "avg_launch_ms": 1e3 * avg_s, "launches": prof[dom][0], "flops_per_launch": fl,
                "workgroups": sum(b for k, b in enumerate(batch) if p.systems[k].N ** 2 <= 4096)}
    elif dom == nat.LB_KERNEL_SWEEP:
        # A profiled unit is the sweep launches of one streamed step: the
        # sweeps that run, the launches that return at once because the step's
        # solve has converged, and the count kernel.  The work read back from
        # the device is entries x executed sweeps, so work / entries executed
        # launches share the unit time; each moves 48 B per entry by the
        # algorithm (read the iterate and q, write the next iterate).
        launches = work[dom] / st_entries
        by = 48.0 * st_entries
        avg_s = ms[dom] / 1e3 / launches
        achieved = by / avg_s / 1e9
        ki = tuned.get("tile_ki", 0)
        tiled = tuned.get("tile", 0) == 1 and ki > 0 and len(p.systems) == 1
        s0 = p.systems[0]
        if tiled and ki >= 100:
            kname = "split_a_kernel + split_b_sweep_kernel<forward|adjoint>"
        elif tiled:
            kname = (f"sweep_tile_kernel<{s0.nlev[0]}, {s0.Q}, {ki // 10}, {ki % 10}, forward|adjoint, "
                     f"{TILE_KIS.get(ki, 256) if s0.Q == 8 else 256}>")
        else:
            kname = "sweep_generic_kernel<forward|adjoint>"
        roof = {"kernel": kname,
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"stage_sweep_c{workload}_ki{ki}", APPLY_SOURCES + STEP_SOURCES)
                if tiled else None,
                "avg_launch_ms": 1e3 * avg_s, "launches": launches, "bytes_per_launch": by,
                "step_units": prof[dom][0], "unit_ms": ms[dom] / n[dom]}
    else:
        by = 64.0 * work[dom] / n[dom]
        achieved = by / avg_s / 1e9
        roof = {"kernel": name_of[dom], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "avg_launch_ms": 1e3 * avg_s, "launches": prof[dom][0], "bytes_per_launch": by}
    nt = p.systems[0].NT
    sweeps = {}
    if lds_entries:
        sweeps["lds_forward"] = work[nat.LB_KERNEL_LDS_FORWARD] / (steps * nt * lds_entries)
        sweeps["lds_adjoint"] = work[nat.LB_KERNEL_LDS_ADJOINT] / (steps * nt * lds_entries)
        sweeps["lds_a_priori"] = wsum / (nt * lds_entries)
    if st_entries:
        sweeps["stream_all_passes"] = work[nat.LB_KERNEL_SWEEP] / (steps * st_entries) / nt
    scale = nt_full / p.systems[0].NT
    return {
        "scale": scale,
        "value": steps / (elapsed * scale),
        "ms_per_step": 1e3 * elapsed * scale / steps,
        "sample": None if scale == 1 else (f"{p.systems[0].NT} of {nt_full} time steps of the full-size "
                                           f"evaluation timed, checkpoint interval {ckpt or 'automatic'}, "
                                           f"time scaled x{scale:g}"),
        "window_ms": 1e3 * elapsed / steps,
        "ckpt_every": ckpt,
        "G": [float(v) for v in G.cpu().numpy()[:4]],
        "grad_norm": float(grad.abs().max().item()),
        "sweeps_per_step_mean": sweeps,
        "roofline": roof,
        "kernel_ms": {name_of[k]: ms[k] / n[k] for k in ms if prof[k][0] > 0},
        "kernel_total_ms": {name_of[k]: ms[k] / steps for k in ms if prof[k][0] > 0},
        "autotune": tuned,
        "states": sum(batch),
        # applications of M per evaluation on the streamed path: every sweep of
        # every pass, plus the gradient integrands of every step
        "apply_equivalents": (work[nat.LB_KERNEL_SWEEP] / steps / st_entries + nt) if st_entries else None,
        # stage-sweep bytes (48 B per entry and executed sweep) over the whole
        # timed region, host clock
        "sweep_GBps_timed_region": 48.0 * work[nat.LB_KERNEL_SWEEP] / elapsed / 1e9 if st_entries else None,
    }


def run_apply_bench(lbx, torch, reps):
    """lindblad_apply on the eight-qutrit ring with the one-pass block-tiled
    kernel (LB_OPT_TILE 1) and the two-pass split kernels (2); the faster
    forward apply is the reported roofline."""
    from workloads import make_config
    p = make_config(5)
    s = p.systems[0]
    N = s.N
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    y = torch.empty_like(x)
    alpha = torch.as_tensor(p.alpha[0].reshape(-1)).to("cuda")
    times = {}
    for tile, ki in tuple((1, k) for k in TILE_KIS) + ((2, 0),):
        plan = lbx.Plan([s], tile=tile)
        plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
        for adj in (False, True):
            for _ in range(3):
                lbx.lindblad_apply(plan, 0, 41.0, alpha, x, adjoint=adj, out=y)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for k in range(reps):
                ev[k][0].record()
                lbx.lindblad_apply(plan, 0, 41.0 + 0.01 * k, alpha, x, adjoint=adj, out=y)
                ev[k][1].record()
            torch.cuda.synchronize()
            times[(tile, ki, adj)] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    tile, ki = min({(t, k) for t, k, _ in times}, key=lambda c: times[(c[0], c[1], False)])
    algo = 32.0 * N * N
    ms = times[(tile, ki, False)]
    achieved = algo / (ms / 1e3) / 1e9
    key = f"apply_kernel_forward_ki{ki}" if tile == 1 else "multipass_apply_forward"
    return {
        "kernel": f"tile_kernel<3, 8, {ki // 10}, {ki % 10}, forward>" if tile == 1
                  else "pass_kernel<forward> (three passes)",
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(key, APPLY_SOURCES),
        "avg_launch_ms": ms, "adjoint_avg_launch_ms": times[(tile, ki, True)],
        "adjoint_achieved": algo / (times[(tile, ki, True)] / 1e3) / 1e9,
        "bytes_per_launch": algo, "workload": "8 qutrits ring, N=6561, 1 state",
        "ms_by_kernel": {f"tile{t}_ki{k}_{'adjoint' if a else 'forward'}": v for (t, k, a), v in times.items()},
    }


def run_traffic_probe(lbx, torch):
    """Launches whose HBM counters are read by rocprofv3 --pmc: a plain device
    copy of one eight-qutrit state (the calibration of the counters); for each
    block shape two forward and two adjoint applies of that state and one
    gradient evaluation of the eight-qutrit ring over 24 steps with
    checkpoints every 12 (forward, recomputation and adjoint sweeps in the mix
    of the timed window); and one two-transmon gradient evaluation."""
    from workloads import make_config, truncate_steps
    p = make_config(5)
    s = p.systems[0]
    N = s.N
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = torch.randn((1, N, N), dtype=torch.complex128, device="cuda", generator=g)
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    alpha = torch.as_tensor(p.alpha[0].reshape(-1)).to("cuda")
    for ki in TILE_KIS:
        plan = lbx.Plan([s])
        plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
        for adj in (False, True):
            for _ in range(2):
                lbx.lindblad_apply(plan, 0, 41.0, alpha, x, adjoint=adj, out=y)
    del x, y
    torch.cuda.synchronize()
    print("[probe] eight-qutrit applies done", file=sys.stderr, flush=True)
    pw = truncate_steps(p, 24)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda")
    args = (dev(pw.rho0[0]), dev(pw.rhotar[0]), dev(pw.beta[0]), pw.batch, pw.gamma2, 12)
    for ki in TILE_KIS:
        plan = lbx.Plan(pw.systems)
        plan.set_option(lbx._native.LB_OPT_TILE_KI, ki)
        lbx.adjoint_gradient(plan, pw.kind, alpha, *args)
        torch.cuda.synchronize()
        print(f"[probe] eight-qutrit gradient window, block shape {ki} done", file=sys.stderr, flush=True)
        del plan
    p = make_config(2)
    plan = lbx.Plan(p.systems)
    lbx.adjoint_gradient(plan, p.kind, dev(p.alpha[0].reshape(-1)), dev(p.rho0[0]), dev(p.rhotar[0]),
                         dev(p.beta[0]), p.batch, p.gamma2, p.ckpt_every)
    torch.cuda.synchronize()
    print("[probe] two-transmon gradient done", file=sys.stderr, flush=True)
    return {"copy_bytes": 16 * N * N}


def traffic_summary(fetch_csv, write_csv, copy_bytes, out_path=None):
    """Per-launch HBM bytes from two rocprofv3 --pmc runs (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
    for the plain device copy of copy_bytes bytes.  Writes profiles/traffic.json
    and prints a markdown table."""
    import csv

    def per_kernel(path):
        out = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch, write = per_kernel(fetch_csv), per_kernel(write_csv)
    cal_f = copy_bytes / 1024 / max(fetch.get("__amd_rocclr_copyBuffer", [0]))
    cal_w = copy_bytes / 1024 / max(write.get("__amd_rocclr_copyBuffer", [0]))
    table = {"calibration": {"copy_bytes": copy_bytes, "fetch_factor": cal_f, "write_factor": cal_w}}
    rows = []
    for key, (pats, files, *mode) in TRAFFIC_KEYS.items():
        fv = [v for k, vs in fetch.items() if any(pt in k for pt in pats) for v in vs]
        wv = [v for k, vs in write.items() if any(pt in k for pt in pats) for v in vs]
        if not fv or not wv:
            continue
        if mode and mode[0] == "executed":
            # launches that returned at once read and write almost nothing
            fv = [v for v in fv if v >= 0.01 * max(fv)]
            wv = [v for v in wv if v >= 0.01 * max(wv)]
        fb = 1024 * cal_f * float(np.mean(fv))
        wb = 1024 * cal_w * float(np.mean(wv))
        table[key] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                      "fetch_kib_raw": float(np.mean(fv)), "write_kib_raw": float(np.mean(wv)),
                      "dispatches": [len(fv), len(wv)], "source_sha": source_sha(files)}
        rows.append(f"| {key} | {len(fv)} | {np.mean(fv):.1f} | {np.mean(wv):.1f} | {fb / 1e9:.4f} | "
                    f"{wb / 1e9:.4f} |")
    with open(out_path or TRAFFIC_FILE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print(f"calibration: copy of {copy_bytes} B; FETCH_SIZE x{cal_f:.3f}, WRITE_SIZE x{cal_w:.3f}")
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | fetch GB (scaled) | write GB (scaled) |")
    print("|---|---|---|---|---|---|")
    print("\n".join(rows))


def kernel_records(path):
    """(kernel name, duration in ms) of every dispatch in a rocprofv3 kernel
    trace: a results database, or the kernel_trace.csv of --output-format csv."""
    if path.endswith(".csv"):
        import csv
        with open(path, newline="") as fh:
            return [(r["Kernel_Name"], (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
                    for r in csv.DictReader(fh)]
    import sqlite3
    con = sqlite3.connect(path)
    return [(n, (t1 - t0) / 1e6) for n, t0, t1 in con.execute("select name, start, end from kernels")]


def kernel_stats(path):
    """Markdown table of the per-kernel times in a rocprofv3 kernel trace; for
    the stage sweep kernels also the average over executed launches (a launch
    after its step's solve has converged returns at once)."""
    recs = kernel_records(path)
    tot = {}
    for name, d in recs:
        short = name.split("(")[0].replace("void ", "")
        c, t = tot.get(short, (0, 0.0))
        tot[short] = (c + 1, t + d)
    grand = sum(t for _, t in tot.values()) or 1.0
    print("| kernel | calls | total ms | average ms | % |")
    print("|---|---|---|---|---|")
    for short, (c, t) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:16]:
        print(f"| `{short}` | {c} | {t:.3f} | {t / c:.4f} | {100 * t / grand:.1f} |")
    by = {}
    for name, d in recs:
        if "sweep_tile_kernel" in name or "sweep_generic_kernel" in name:
            by.setdefault(name.split("(")[0].replace("void ", ""), []).append(d)
    if not by:
        return
    print()
    print("| stage sweep kernel | launches | executed (>= 5 % of the longest) | executed average ms | "
          "others average ms |")
    print("|---|---|---|---|---|")
    for name, d in sorted(by.items()):
        cut = 0.05 * max(d)
        ex = [v for v in d if v >= cut]
        rest = [v for v in d if v < cut]
        print(f"| `{name}` | {len(d)} | {len(ex)} | {np.mean(ex):.4f} | "
              f"{np.mean(rest) if rest else 0.0:.4f} |")
    allex = []
    for d in by.values():
        cut = 0.05 * max(d)
        allex += [v for v in d if v >= cut]
    print(f"\nall executed stage sweep launches: {len(allex)}, average {np.mean(allex):.4f} ms")


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


CPU_PROCS_MAX = 16        # the host-core share of one GPU on the box
CPU_PROC_BYTES = {5: 6 << 30, 2: 1 << 30}   # host memory one oracle worker of a workload may hold


def host_info():
    """CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count()
    mem = None
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemAvailable"):
                    mem = int(line.split()[1]) * 1024
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": aff, "mem_available": mem}


def cpu_procs(workload, info):
    n = min(CPU_PROCS_MAX, info["affinity"] or 1)
    if info["mem_available"]:
        n = min(n, max(1, int(0.5 * info["mem_available"] // CPU_PROC_BYTES[workload])))
    return n


def _oracle_worker(kind, tasks, barrier, out):
    """One CPU process: prepares its tasks, waits for the others, then times
    the oracle on them (one BLAS thread, the oracle's own setting)."""
    import oracle
    from workloads import make_config, truncate_steps
    if kind == "apply5":
        p = make_config(5)
        s = p.systems[0]
        xs = []
        for seed in tasks:
            rng = np.random.default_rng(seed)
            xs.append(rng.standard_normal((s.N, s.N)) + 1j * rng.standard_normal((s.N, s.N)))
        barrier.wait()
        t0 = time.perf_counter()
        for x in xs:
            oracle.lindbladian(s, p.alpha[0], 41.0, x)
    else:
        # the whole 16-state evaluation per task (the oracle solves all states
        # of a system together)
        nsteps = kind[1]
        p = truncate_steps(make_config(2), nsteps)
        s = p.systems[0]
        barrier.wait()
        t0 = time.perf_counter()
        for _ in tasks:
            oracle.value_and_gradient(s, p.alpha[0], p.rho0[0], p.rhotar[0], p.beta[0], p.kind)
    out.put(time.perf_counter() - t0)


def run_oracle_pool(kind, tasks, nproc):
    """Runs the tasks over nproc fresh processes (round robin) that start
    together; returns the wall time of the slowest."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(nproc)
    out = ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(kind, tasks[k::nproc], barrier, out)) for k in range(nproc)]
    for pr in procs:
        pr.start()
    times = [out.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
        if pr.exitcode != 0:
            raise RuntimeError(f"oracle worker ended with {pr.exitcode}")
    return max(times)


def run_cpu_apply_baseline(apply_equivalents, scale):
    """The oracle's operator-form apply of M(t) on the eight-qutrit state, one
    apply per process on its own state, all processes at once, extrapolated to
    whole gradient evaluations by the applications of M per evaluation that
    the GPU path makes (one per stage sweep and one per gradient integrand)."""
    info = host_info()
    n = cpu_procs(5, info)
    wall = run_oracle_pool("apply5", list(range(1, n + 1)), n)
    applies = apply_equivalents * scale
    return {"value": n / (wall * applies), "unit": "evals/s", "cores": n, "kind": "oracle",
            "sample": f"{n} processes, each one operator-form apply of M(t) on its own eight-qutrit state, "
                      f"all at once ({wall:.1f} s wall); each process extrapolated x{applies:.0f} applies per "
                      f"gradient evaluation (value = {n} evaluations in parallel)",
            **info}


def run_cpu_baseline(nsteps):
    """The oracle's two-transmon gradient (all 16 states), one evaluation per
    process on every process of the share at once, over nsteps of the 10000
    steps, scaled to the horizon."""
    from workloads import make_config
    info = host_info()
    n = cpu_procs(2, info)
    wall = run_oracle_pool(("grad2", nsteps), list(range(n)), n)
    scale = make_config(2).systems[0].NT / nsteps
    return {"value": n / (wall * scale), "unit": "evals/s", "cores": n, "kind": "oracle",
            "sample": f"two-transmon CNOT (16 states), {n} processes each one evaluation over {nsteps} of 10000 "
                      f"steps, all at once ({wall:.1f} s wall), scaled x{scale:g} (value = {n} evaluations in "
                      f"parallel)", **info}


def c2_summary(lbx, torch, args):
    """The two-transmon CNOT gradient (LDS-resident path) with its per-state
    loop speedup and CPU baseline, reported beside the headline."""
    res = run_gradient_bench(lbx, torch, args.c2_steps, 3, 2, 0)
    out = {"workload": WORKLOADS[2], "value": res["value"], "unit": "evals/s", "ms_per_eval": res["ms_per_step"],
           "steps": args.c2_steps, "roofline": res["roofline"], "sweeps_per_step_mean": res["sweeps_per_step_mean"],
           "G": res["G"]}
    if not args.no_loop:
        print("[bench] two-transmon per-state loop", file=sys.stderr, flush=True)
        lb = run_loop_baseline(lbx, torch, args.loop_steps)
        lb["speedup"] = res["value"] / lb["evals_per_s"]
        out["per_state_loop"] = lb
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed evaluations of the headline workload (default 1 for workloads 3 and 5, 3 for 4, "
                         "20 otherwise)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=HEADLINE, choices=[1, 2, 3, 4, 5],
                    help="headline workload (default 5, the eight-qutrit ring)")
    ap.add_argument("--window", "--sample-steps", type=int, default=0, dest="window",
                    help="time W steps with the horizon shortened to W dt (0, the default: the whole "
                         "horizon); the rate is scaled to the full horizon, but the controls vary faster "
                         "per step than in the workload")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--c2-steps", type=int, default=20)
    ap.add_argument("--loop-steps", type=int, default=250)
    ap.add_argument("--cpu-steps", type=int, default=2000)
    ap.add_argument("--no-apply", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-loop", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only the launches whose HBM counters profiles/traffic.json records")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter CSVs")
    ap.add_argument("--kernel-stats", metavar="TRACE",
                    help="print the per-kernel table of a rocprofv3 kernel trace (results database or "
                         "kernel_trace.csv)")
    args = ap.parse_args()
    if args.kernel_stats:
        kernel_stats(args.kernel_stats)
        return
    if args.traffic_summary:
        from workloads import make_config
        n = make_config(5).systems[0].N
        traffic_summary(*args.traffic_summary, 16 * n * n)
        return
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
    if args.traffic_probe:
        print(json.dumps(run_traffic_probe(lbx, torch)), flush=True)
        return
    w = args.workload
    if args.steps is None:
        args.steps = DEFAULT_STEPS[w]
    window = args.window
    print(f"[bench] workload {w} gradient evaluations (window {window or 'all'})", file=sys.stderr, flush=True)
    res = run_gradient_bench(lbx, torch, args.steps, args.warmup, w, window)
    print(f"[bench] {res['value']:.4g} evals/s, {res['window_ms']:.1f} ms per bench step", file=sys.stderr,
          flush=True)
    line = {
        "metric": "forward+adjoint gradient evals/sec; lindblad_apply HBM GB/s vs peak",
        "value": res["value"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["window_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[w], "global_batch": res["states"], "parallelism": "single GPU",
                   "step": ("one gradient evaluation of the full-size system over a shortened horizon "
                            "(controls compressed into it); value scaled to the whole horizon")
                   if res["scale"] != 1 else "one gradient evaluation of the whole horizon",
                   "window_steps": round(WORKLOADS_NT[w] / res["scale"]), "horizon_steps": WORKLOADS_NT[w],
                   "ckpt_every": res["ckpt_every"]},
        "sample": res["sample"],
        "ms_per_eval": res["ms_per_step"],
        "roofline": with_traffic_rate(res["roofline"]),
        "detail": {"G": res["G"], "grad_max": res["grad_norm"],
                   "sweeps_per_step_mean": res["sweeps_per_step_mean"],
                   "kernel_avg_ms": res["kernel_ms"], "kernel_ms_per_step": res["kernel_total_ms"],
                   "sweep_GBps_timed_region": res["sweep_GBps_timed_region"],
                   "autotune": res["autotune"]},
    }
    if w == 5 and not args.no_apply:
        print("[bench] lindblad_apply 8 qutrits", file=sys.stderr, flush=True)
        line["apply_roofline"] = with_traffic_rate(run_apply_bench(lbx, torch, args.apply_reps))
    if w != 2 and not args.no_c2:
        print("[bench] two-transmon gradient", file=sys.stderr, flush=True)
        line["c2_cnot"] = c2_summary(lbx, torch, args)
    elif w == 2 and not args.no_loop:
        print("[bench] per-state loop baseline", file=sys.stderr, flush=True)
        lb = run_loop_baseline(lbx, torch, args.loop_steps)
        lb["speedup"] = res["value"] / lb["evals_per_s"]
        line["per_state_loop"] = lb
    if not args.no_cpu:
        if w == 5 and res["apply_equivalents"]:
            print("[bench] cpu baseline (oracle applies, all processes at once)", file=sys.stderr, flush=True)
            line["cpu_baseline"] = run_cpu_apply_baseline(res["apply_equivalents"], res["scale"])
        if w == 2 or "c2_cnot" in line:
            print("[bench] cpu baseline (two-transmon oracle, one process per state)", file=sys.stderr, flush=True)
            cb = run_cpu_baseline(args.cpu_steps)
            if w == 2:
                line["cpu_baseline"] = cb
            else:
                line["c2_cnot"]["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
