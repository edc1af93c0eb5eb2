"""Helpers shared by the GPU parity tests (marshalling only, no arithmetic
of the method)."""
import sys

import numpy as np
import torch


def say(*a):
    """Name the case before each GPU step, flushed, so a crash log shows it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def flat_states(states):
    """Concatenate per-system [B, N, N] arrays into the batched layout."""
    return np.concatenate([np.asarray(s, dtype=np.complex128).reshape(-1) for s in states])


def split_states(flat, systems, batch):
    out, off = [], 0
    for s, b in zip(systems, batch):
        n = b * s.N * s.N
        out.append(np.asarray(flat[off:off + n]).reshape(b, s.N, s.N))
        off += n
    return out


def flat_alpha(alphas):
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in alphas])


def rel_state_err(got, ref):
    """max over states of ||got - ref||_F / ||ref||_F."""
    errs = []
    for g, r in zip(got, ref):
        for b in range(r.shape[0]):
            errs.append(np.linalg.norm(g[b] - r[b]) / max(np.linalg.norm(r[b]), 1e-300))
    return max(errs) if errs else 0.0
