"""Python binding of liblbx with the same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the HIP
kernels of liblbx.so.  PyTorch supplies device memory (tensors) and the
stream (``torch.cuda.current_stream()``).  States are complex128 tensors of
shape [B, N, N] (row-major rho[i][j]); control coefficients are float64
tensors laid out [Q][Ns][Nf][2] per system and concatenated over systems.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np
import torch

from . import _native as nat
from ._native import check, lib

KIND = {"frob": nat.LB_J_FROB, "tr": nat.LB_J_TR, "nm": nat.LB_J_NM, 0: nat.LB_J_FROB, 1: nat.LB_J_TR,
        2: nat.LB_J_NM}
PATHS = {"auto": 0, "lds": 1, "stream": 2}


def _vp(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, numel: int | None = None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t


class Plan:
    """Owns an lb_plan built from System-like objects (see workloads.System)."""

    def __init__(self, systems: Sequence, path: str = "auto", solve_tol: float | None = None,
                 tile: int = 1):
        self.systems = list(systems)
        n = len(self.systems)
        descs = (nat.SystemDesc * n)()
        self._keep = []
        for k, s in enumerate(self.systems):
            Q = len(s.nlev)
            arrs = {
                "nlev": np.ascontiguousarray(s.nlev, dtype=np.int32),
                "detuning": np.ascontiguousarray(s.detuning, dtype=np.float64),
                "selfkerr": np.ascontiguousarray(s.selfkerr, dtype=np.float64),
                "crosskerr": np.ascontiguousarray(np.asarray(s.crosskerr, dtype=np.float64).reshape(Q * Q)),
                "T1": np.ascontiguousarray(s.T1, dtype=np.float64),
                "T2": np.ascontiguousarray(s.T2, dtype=np.float64),
                "carrier": np.ascontiguousarray(np.asarray(s.carriers, dtype=np.float64).reshape(-1)),
            }
            self._keep.append(arrs)
            d = descs[k]
            d.Q = Q
            d.nlev = arrs["nlev"].ctypes.data_as(nat._ip)
            for f in ("detuning", "selfkerr", "crosskerr", "T1", "T2", "carrier"):
                setattr(d, f, arrs[f].ctypes.data_as(nat._dp))
            d.Ns = int(s.Ns)
            d.Nf = int(np.asarray(s.carriers).shape[1])
            d.T = float(s.T)
            d.NT = int(s.NT)
            jc, rot = getattr(s, "jc", None), getattr(s, "rotfreq", None)
            if jc is not None:
                arrs["jc"] = np.ascontiguousarray(np.asarray(jc, dtype=np.float64).reshape(Q * Q))
                d.jc = arrs["jc"].ctypes.data_as(nat._dp)
            if rot is not None:
                arrs["rotfreq"] = np.ascontiguousarray(rot, dtype=np.float64)
                d.rotfreq = arrs["rotfreq"].ctypes.data_as(nat._dp)
        handle = C.c_void_p()
        check(lib.lb_plan_create(descs, n, C.byref(handle)), "lb_plan_create")
        self.handle = handle
        self.N, self.nalpha = [], []
        for k in range(n):
            N, na, NT = C.c_int32(), C.c_int32(), C.c_int32()
            check(lib.lb_plan_info(self.handle, k, C.byref(N), C.byref(na), C.byref(NT)), "lb_plan_info")
            self.N.append(N.value)
            self.nalpha.append(na.value)
        self.NT = NT.value
        self.alpha_off = np.concatenate([[0], np.cumsum(self.nalpha)]).astype(np.int64)
        self._ws = {}
        self._alpha_sys = None
        if path != "auto":
            self.set_option(nat.LB_OPT_PATH, PATHS[path])
        if solve_tol is not None:
            self.set_option(nat.LB_OPT_SOLVE_TOL, solve_tol)
        if int(tile) != 1:  # 0: generic streaming kernels, 2: two-pass split kernels
            self.set_option(nat.LB_OPT_TILE, int(tile))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib.lb_plan_destroy(h)
            self.handle = None

    def set_option(self, option: int, value: float) -> None:
        check(lib.lb_plan_set_option(self.handle, option, float(value)), "lb_plan_set_option")
        self._ws.clear()

    def profile(self, on: bool = True) -> None:
        """Time kernel launches of forward_solve/adjoint_gradient with HIP events."""
        self.set_option(nat.LB_OPT_PROFILE, 1.0 if on else 0.0)

    def profile_read(self, kernel: int, reset: bool = False):
        """(launches, total milliseconds) of one LB_KERNEL_* family."""
        n, ms = C.c_int64(), C.c_double()
        check(lib.lb_profile_read(self.handle, kernel, C.byref(n), C.byref(ms), int(reset)),
              "lb_profile_read")
        return n.value, ms.value

    def profile_work(self, kernel: int) -> int:
        """Entries x stage sweeps (entries x steps for the gradient kernel) done
        by one LB_KERNEL_* family while profiling; reset by profile_read."""
        w = C.c_int64()
        check(lib.lb_profile_work(self.handle, kernel, C.byref(w)), "lb_profile_work")
        return w.value

    def autotune(self, alpha: torch.Tensor, batch: Sequence[int], cache: str | None = None) -> dict:
        """Pick the fastest kernel configuration of the streamed systems.

        Runs lb_autotune, or reuses the choice stored in the JSON file `cache`
        under a key made of the system shapes and the batch.
        """
        import json
        import os
        key = json.dumps([[list(s.nlev) for s in self.systems], [int(b) for b in batch], self.NT])
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                table = json.load(fh)
        if key in table:
            ch = table[key]
            self.set_option(nat.LB_OPT_TILE, ch["tile"])
            self.set_option(nat.LB_OPT_TILE_KI, ch["tile_ki"])
            self.set_option(nat.LB_OPT_GRAPH, ch["graph_steps"])
            return ch
        b = self.batch_array(batch)
        _need(alpha, "alpha", torch.float64, int(self.alpha_off[-1]))
        ws = self.workspace(nat.LB_OP_FORWARD, batch)
        res = np.zeros(3, dtype=np.int32)
        check(lib.lb_autotune(self.handle, _vp(alpha), b.ctypes.data_as(nat._ip), _vp(ws), ws.numel(),
                              _stream(), res.ctypes.data_as(nat._ip)), "lb_autotune")
        self._ws.clear()
        ch = {"tile": int(res[0]), "tile_ki": int(res[1]), "graph_steps": int(res[2])}
        if cache:
            table[key] = ch
            with open(cache, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
        return ch

    def set_path(self, path: str) -> None:
        self.set_option(nat.LB_OPT_PATH, PATHS[path])

    def batch_array(self, batch: Sequence[int]):
        b = np.ascontiguousarray(batch, dtype=np.int32)
        if b.shape != (len(self.systems),):
            raise ValueError("batch_per_sys must have one entry per system")
        return b

    def workspace_bytes(self, op: int, batch: Sequence[int], ckpt_every: int = 1) -> int:
        b = self.batch_array(batch)
        out = C.c_size_t()
        check(lib.lb_workspace_bytes(self.handle, op, b.ctypes.data_as(nat._ip), int(ckpt_every),
                                     C.byref(out)), "lb_workspace_bytes")
        return out.value

    def workspace(self, op: int, batch: Sequence[int], ckpt_every: int = 1) -> torch.Tensor:
        key = (op, tuple(int(x) for x in batch), int(ckpt_every))
        ws = self._ws.get(key)
        if ws is None:
            nbytes = self.workspace_bytes(op, batch, ckpt_every)
            ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
            self._ws[key] = ws
        return ws

    def trajectory_bytes(self, batch: Sequence[int], ckpt_every: int = 0) -> int:
        b = self.batch_array(batch)
        out = C.c_size_t()
        check(lib.lb_trajectory_bytes(self.handle, b.ctypes.data_as(nat._ip), int(ckpt_every), C.byref(out)),
              "lb_trajectory_bytes")
        return out.value

    def trajectory(self, batch: Sequence[int], ckpt_every: int = 0) -> torch.Tensor:
        """A new buffer for the forward trajectory of forward_solve."""
        return torch.empty(max(self.trajectory_bytes(batch, ckpt_every), 1), dtype=torch.uint8, device="cuda")

    def status(self, ws: torch.Tensor | None) -> None:
        """Raises LbxError for the device status of the last call on ws (with
        ws None: of the last imr_step_noalloc call on the current device)."""
        check(lib.lb_status(self.handle, _vp(ws) if ws is not None else None, _stream()), "lb_status")

    def entries(self, batch: Sequence[int]) -> int:
        return int(sum(int(b) * n * n for b, n in zip(batch, self.N)))

    def alpha_system_index(self) -> torch.Tensor:
        if self._alpha_sys is None:
            idx = np.repeat(np.arange(len(self.systems)), self.nalpha)
            self._alpha_sys = torch.as_tensor(idx, device="cuda")
        return self._alpha_sys


def sweep_counts(plan: Plan, alpha: torch.Tensor) -> np.ndarray:
    """Stage-solve sweeps per step, [nsys, NT, 2] (LDS-resident, streaming)."""
    _need(alpha, "alpha", torch.float64, int(plan.alpha_off[-1]))
    out = np.zeros((len(plan.systems), plan.NT, 2), dtype=np.int32)
    check(lib.sweep_counts(plan.handle, _vp(alpha), out.ctypes.data_as(nat._ip), _stream()),
          "sweep_counts")
    return out


def control_table(plan: Plan, sys: int, alpha: torch.Tensor) -> torch.Tensor:
    """d_q(t_{j+1/2}) for every step, [NT, Q] complex128 (rad/ns)."""
    _need(alpha, "alpha", torch.float64, plan.nalpha[sys])
    out = torch.empty((plan.NT, len(plan.systems[sys].nlev)), dtype=torch.complex128, device="cuda")
    check(lib.control_table(plan.handle, sys, _vp(alpha), _vp(out), _stream()), "control_table")
    return out


def lindblad_apply(plan: Plan, sys: int, t: float, alpha: torch.Tensor, x: torch.Tensor,
                   adjoint: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """y = M(t) x (or M(t)^+ x) for x of shape [B, N, N]."""
    N = plan.N[sys]
    _need(alpha, "alpha", torch.float64, plan.nalpha[sys])
    _need(x, "x", torch.complex128)
    if x.dim() != 3 or x.shape[1:] != (N, N):
        raise ValueError(f"x must be [B, {N}, {N}]")
    y = torch.empty_like(x) if out is None else _need(out, "out", torch.complex128, x.numel())
    check(lib.lindblad_apply(plan.handle, sys, float(t), _vp(alpha), _vp(x), _vp(y), x.shape[0],
                             int(bool(adjoint)), _stream()), "lindblad_apply")
    return y


def imr_step(plan: Plan, sys: int, j: int, alpha: torch.Tensor, q_in: torch.Tensor,
             adjoint: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """One implicit-midpoint step (or adjoint step) for q_in of shape [B, N, N]."""
    N = plan.N[sys]
    _need(alpha, "alpha", torch.float64, plan.nalpha[sys])
    _need(q_in, "q_in", torch.complex128)
    if q_in.dim() != 3 or q_in.shape[1:] != (N, N):
        raise ValueError(f"q_in must be [B, {N}, {N}]")
    B = q_in.shape[0]
    batch = [0] * len(plan.systems)
    batch[sys] = B
    ws = plan.workspace(nat.LB_OP_IMR_STEP, batch)
    q_out = torch.empty_like(q_in) if out is None else _need(out, "out", torch.complex128, q_in.numel())
    check(lib.imr_step(plan.handle, sys, int(j), _vp(alpha), _vp(q_in), _vp(q_out), B,
                       int(bool(adjoint)), _vp(ws), ws.numel(), _stream()), "imr_step")
    return q_out


def imr_step_noalloc(plan: Plan, sys: int, j: int, alpha: torch.Tensor, q_in: torch.Tensor,
                     out: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
    """imr_step without a workspace: the library's static device scratch
    serves it, so the call allocates nothing (out is the caller's)."""
    N = plan.N[sys]
    _need(alpha, "alpha", torch.float64, plan.nalpha[sys])
    _need(q_in, "q_in", torch.complex128)
    if q_in.dim() != 3 or q_in.shape[1:] != (N, N):
        raise ValueError(f"q_in must be [B, {N}, {N}]")
    _need(out, "out", torch.complex128, q_in.numel())
    check(lib.imr_step_noalloc(plan.handle, sys, int(j), _vp(alpha), _vp(q_in), _vp(out), q_in.shape[0],
                               int(bool(adjoint)), _stream()), "imr_step_noalloc")
    return out


def _states(plan: Plan, t: torch.Tensor, name: str, batch) -> torch.Tensor:
    return _need(t, name, torch.complex128, plan.entries(batch))


def forward_solve(plan: Plan, alpha: torch.Tensor, rho0: torch.Tensor, batch: Sequence[int],
                  out: torch.Tensor | None = None, traj: torch.Tensor | None = None,
                  ckpt_every: int = 0) -> torch.Tensor:
    """rho(T) for every state of every system (batched layout).  With `traj`
    (a uint8 tensor of Plan.trajectory_bytes(batch, ckpt_every) bytes) the
    forward states that adjoint_backward needs are kept in it."""
    b = plan.batch_array(batch)
    _need(alpha, "alpha", torch.float64, int(plan.alpha_off[-1]))
    _states(plan, rho0, "rho0", batch)
    rhoT = torch.empty_like(rho0) if out is None else _states(plan, out, "out", batch)
    if traj is not None:
        _need(traj, "traj", torch.uint8)
        if traj.numel() < plan.trajectory_bytes(batch, ckpt_every):
            raise ValueError("traj is smaller than Plan.trajectory_bytes")
    ck = int(ckpt_every) if traj is not None else 1
    ws = plan.workspace(nat.LB_OP_FORWARD, batch, ck)
    check(lib.forward_solve(plan.handle, _vp(alpha), _vp(rho0), _vp(rhoT), b.ctypes.data_as(nat._ip),
                            _vp(traj) if traj is not None else None, ck, _vp(ws), ws.numel(), _stream()),
          "forward_solve")
    return rhoT


def objective(plan: Plan, kind, rhoT: torch.Tensor, rhotar: torch.Tensor, beta: torch.Tensor,
              batch: Sequence[int], gamma2: float, alpha: torch.Tensor):
    """(G per system, J per state)."""
    b = plan.batch_array(batch)
    _states(plan, rhoT, "rhoT", batch)
    _states(plan, rhotar, "rhotar", batch)
    _need(beta, "beta", torch.float64, int(b.sum()))
    _need(alpha, "alpha", torch.float64, int(plan.alpha_off[-1]))
    G = torch.empty(len(plan.systems), dtype=torch.float64, device="cuda")
    J = torch.empty(max(int(b.sum()), 1), dtype=torch.float64, device="cuda")
    ws = plan.workspace(nat.LB_OP_FORWARD, batch)
    check(lib.objective(plan.handle, KIND[kind], _vp(rhoT), _vp(rhotar), _vp(beta),
                        b.ctypes.data_as(nat._ip), float(gamma2), _vp(alpha), _vp(G), _vp(J),
                        _vp(ws), ws.numel(), _stream()), "objective")
    return G, J[: int(b.sum())]


def adjoint_gradient(plan: Plan, kind, alpha: torch.Tensor, rho0: torch.Tensor,
                     rhotar: torch.Tensor, beta: torch.Tensor, batch: Sequence[int],
                     gamma2: float = 0.0, ckpt_every: int = 1, want_rhoT: bool = False,
                     workspace: torch.Tensor | None = None, gamma1: float = 0.0, penalty_a: float = 1.0):
    """(G per system, dG/dalpha, rho(T) or None).  `workspace` (uint8, at
    least Plan.workspace_bytes(LB_OP_GRADIENT, batch, ckpt_every)) replaces
    the plan's cached one: calls that may overlap need their own.  `gamma1`
    and `penalty_a` add the running penalty (weight gamma1, width a in ns)."""
    b = plan.batch_array(batch)
    _need(alpha, "alpha", torch.float64, int(plan.alpha_off[-1]))
    _states(plan, rho0, "rho0", batch)
    _states(plan, rhotar, "rhotar", batch)
    _need(beta, "beta", torch.float64, int(b.sum()))
    G = torch.empty(len(plan.systems), dtype=torch.float64, device="cuda")
    grad = torch.empty_like(alpha)
    rhoT = torch.empty_like(rho0) if want_rhoT else None
    if workspace is None:
        ws = plan.workspace(nat.LB_OP_GRADIENT, batch, ckpt_every)
    else:
        ws = _need(workspace, "workspace", torch.uint8)
        if ws.numel() < plan.workspace_bytes(nat.LB_OP_GRADIENT, batch, ckpt_every):
            raise ValueError("workspace is smaller than Plan.workspace_bytes")
    check(lib.adjoint_gradient(plan.handle, KIND[kind], _vp(alpha), _vp(rho0), _vp(rhotar),
                               _vp(beta), b.ctypes.data_as(nat._ip), float(gamma2), float(gamma1),
                               float(penalty_a), int(ckpt_every), _vp(G), _vp(grad),
                               _vp(rhoT) if rhoT is not None else None,
                               _vp(ws), ws.numel(), _stream()), "adjoint_gradient")
    return G, grad, rhoT


def adjoint_backward(plan: Plan, kind, alpha: torch.Tensor, traj: torch.Tensor, ckpt_every: int,
                     rhotar: torch.Tensor, beta: torch.Tensor, batch: Sequence[int], gamma2: float = 0.0,
                     gscale: torch.Tensor | None = None) -> torch.Tensor:
    """sum_s gscale[s] dG_s/dalpha from a trajectory kept by forward_solve."""
    b = plan.batch_array(batch)
    _need(alpha, "alpha", torch.float64, int(plan.alpha_off[-1]))
    _need(traj, "traj", torch.uint8)
    _states(plan, rhotar, "rhotar", batch)
    _need(beta, "beta", torch.float64, int(b.sum()))
    if gscale is not None:
        _need(gscale, "gscale", torch.float64, len(plan.systems))
    grad = torch.empty_like(alpha)
    ws = plan.workspace(nat.LB_OP_BACKWARD, batch, ckpt_every)
    check(lib.adjoint_backward(plan.handle, KIND[kind], _vp(alpha), _vp(traj), int(ckpt_every), _vp(rhotar),
                               _vp(beta), b.ctypes.data_as(nat._ip), float(gamma2),
                               _vp(gscale) if gscale is not None else None, _vp(grad), _vp(ws), ws.numel(),
                               _stream()), "adjoint_backward")
    return grad


class LindbladObjective(torch.autograd.Function):
    """G(alpha) per system; backward runs the discrete adjoint (App. B).

    forward(alpha, plan, kind, rho0, rhotar, beta, batch, gamma2, ckpt_every,
    gamma1, penalty_a).  The forward pass integrates every state
    (forward_solve) and forms G (objective); when alpha requires a gradient it
    keeps the forward trajectory (checkpoints every ckpt_every steps, see
    lb_workspace_bytes) for the backward pass.  The backward pass runs the
    adjoint sweep from that trajectory with the incoming gradient of G as the
    weights of the terminal conditions (adjoint_backward).  With a running
    penalty (gamma1 != 0) G needs every state of the trajectory: the forward
    pass then runs adjoint_gradient, and the backward pass scales its
    gradient by the incoming one.
    """

    @staticmethod
    def forward(ctx, alpha, plan, kind, rho0, rhotar, beta, batch, gamma2=0.0, ckpt_every=0, gamma1=0.0,
                penalty_a=1.0):
        alpha = alpha.detach().contiguous()
        if gamma1 != 0.0:
            G, grad, _ = adjoint_gradient(plan, kind, alpha, rho0, rhotar, beta, batch, gamma2, ckpt_every,
                                          gamma1=gamma1, penalty_a=penalty_a)
            ctx.grads, ctx.alpha_off = grad, plan.alpha_off
            return G
        ctx.grads = None
        traj = plan.trajectory(batch, ckpt_every) if ctx.needs_input_grad[0] else None
        rhoT = forward_solve(plan, alpha, rho0, batch, traj=traj, ckpt_every=ckpt_every)
        G, _ = objective(plan, kind, rhoT, rhotar, beta, batch, gamma2, alpha)
        if traj is not None:
            ctx.save_for_backward(alpha, traj, rhotar, beta)
            ctx.plan, ctx.kind, ctx.batch, ctx.gamma2, ctx.ckpt_every = plan, kind, batch, gamma2, ckpt_every
        return G

    @staticmethod
    def backward(ctx, gG):
        gscale = gG.detach().to(torch.float64).contiguous()
        nones = (None,) * 10
        if ctx.grads is not None:
            # one gradient per system, each over that system's own coefficients
            g = ctx.grads.clone()
            off = ctx.alpha_off
            for s in range(len(off) - 1):
                g[int(off[s]):int(off[s + 1])] *= gscale[s]
            return (g,) + nones
        alpha, traj, rhotar, beta = ctx.saved_tensors
        grad = adjoint_backward(ctx.plan, ctx.kind, alpha, traj, ctx.ckpt_every, rhotar, beta, ctx.batch,
                                ctx.gamma2, gscale)
        return (grad,) + nones


def lindblad_objective(alpha, plan, kind, rho0, rhotar, beta, batch, gamma2=0.0, ckpt_every=0, gamma1=0.0,
                       penalty_a=1.0):
    return LindbladObjective.apply(alpha, plan, kind, rho0, rhotar, beta, batch, gamma2, ckpt_every, gamma1,
                                   penalty_a)
