"""L-BFGS on the control coefficients (Sec. III: the optimisation problem is
solved with L-BFGS updates; App. B gives the exact discrete gradient).

The objective is the sum over the plan's systems of G_s(alpha) from
``lindblad_objective``; every evaluation runs the forward pass on the GPU and
every gradient the discrete adjoint (the autograd backward of
``LindbladObjective``).  The quasi-Newton update itself is torch's L-BFGS
with a strong-Wolfe line search on the device.
"""
from __future__ import annotations

from typing import Callable, Sequence

import torch

from .api import Plan, lindblad_objective


def optimize(plan: Plan, kind, alpha0: torch.Tensor, rho0: torch.Tensor, rhotar: torch.Tensor,
             beta: torch.Tensor, batch: Sequence[int], gamma2: float = 0.0, ckpt_every: int = 0,
             max_iter: int = 100, tolerance_grad: float = 1e-9, tolerance_change: float = 1e-14,
             history_size: int = 20, callback: Callable[[int, float], None] | None = None,
             gamma1: float = 0.0, penalty_a: float = 1.0):
    """Minimise sum_s G_s(alpha) from alpha0 (with the running penalty when
    gamma1 != 0).

    Returns (alpha, history) where history lists the objective of every
    evaluation (line-search trials included).  `callback(k, G)` is called
    after each evaluation.
    """
    alpha = alpha0.detach().clone().contiguous().requires_grad_(True)
    opt = torch.optim.LBFGS([alpha], lr=1.0, max_iter=max_iter, max_eval=2 * max_iter,
                            tolerance_grad=tolerance_grad, tolerance_change=tolerance_change,
                            history_size=history_size, line_search_fn="strong_wolfe")
    history: list[float] = []

    def closure():
        opt.zero_grad()
        G = lindblad_objective(alpha, plan, kind, rho0, rhotar, beta, batch, gamma2, ckpt_every, gamma1,
                               penalty_a).sum()
        G.backward()
        history.append(float(G.detach()))
        if callback is not None:
            callback(len(history), history[-1])
        return G

    opt.step(closure)
    return alpha.detach(), history
