"""Gradient-based thin-film design with the adjoint gradients (the use the
paper gives for TMM-Torch: an MSE against a target reflectance, minimised with
L-BFGS-B; section "TMM-Torch" and App. A.3).

Orchestration only: R comes from tmm_rt and dl/dd from tmm_rt_grad; SciPy's
L-BFGS-B drives the iterations on the host.
"""
from __future__ import annotations

import numpy as np

from . import tmm


def reflectance_objective(n_layers, n_amb, n_sub, wl, theta, target, pol="both", device="cuda"):
    """Returns f(d) -> (loss, grad) for loss = mean over (pol, theta, wl) of
    (R - target)^2, for one stack with constant layer indices n_layers [L]
    between ambient n_amb and substrate n_sub; d in the unit of wl."""
    import torch
    L = len(n_layers)
    nk = np.concatenate([[n_amb], np.asarray(n_layers, dtype=np.complex128), [n_sub]]).astype(np.complex128)
    nk_t = torch.as_tensor(nk, device=device)
    wl_t = torch.as_tensor(np.asarray(wl, dtype=np.float64), device=device)
    th = np.asarray(theta, dtype=np.float64)
    s_t = torch.as_tensor(np.sin(th), device=device)
    c_t = torch.as_tensor(np.cos(th), device=device)
    P = 2 if pol == "both" else 1
    shape = (1, P, th.size, wl_t.numel())
    tgt = torch.as_tensor(np.broadcast_to(np.asarray(target, dtype=np.float64), shape).copy(), device=device)
    R = torch.empty(shape, dtype=torch.float64, device=device)
    gd = torch.empty((1, L), dtype=torch.float64, device=device)
    N = float(np.prod(shape))

    def f(d):
        d_t = torch.as_tensor(np.asarray(d, dtype=np.float64).reshape(1, L), device=device)
        tmm.tmm_rt(d_t, nk_t, wl_t, s_t, c_t, pol_mask=tmm.POL[pol], R=R)
        diff = R - tgt
        loss = float((diff * diff).sum().item() / N)
        tmm.tmm_rt_grad(d_t, nk_t, wl_t, s_t, c_t, pol_mask=tmm.POL[pol], dl_dR=(2.0 / N) * diff, grad_d=gd)
        return loss, gd.cpu().numpy()[0].copy()

    return f


def design(n_layers, n_amb, n_sub, wl, theta, target, d0, bounds=(0.0, 500.0), max_iter=100, pol="both"):
    """Minimise the reflectance MSE over the thicknesses with L-BFGS-B.
    Returns (d_opt, history of losses, scipy result)."""
    from scipy.optimize import minimize
    f = reflectance_objective(n_layers, n_amb, n_sub, wl, theta, target, pol)
    hist = []

    def fun(d):
        loss, g = f(d)
        hist.append(loss)
        return loss, g

    res = minimize(fun, np.asarray(d0, dtype=np.float64), jac=True, method="L-BFGS-B",
                   bounds=[bounds] * len(d0), options={"maxiter": max_iter})
    return res.x, hist, res


def reward(R, R_target):
    """Reward of the paper's thin-film environment: -sum |R_target - R| (section "Environment")."""
    return -float(np.abs(np.asarray(R_target) - np.asarray(R)).sum())
