"""Thin ctypes binding of libtmm_rt (include/tmm_rt.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmm_rt.so")

TMM_OK = 0
TMM_ERR_INVALID_ARG = 1
TMM_ERR_UNSUPPORTED = 2
TMM_ERR_NONFINITE = 3
TMM_ERR_HIP = 4
TMM_ERR_WORKSPACE = 5
TMM_F64 = 0
TMM_F32 = 1
POL = {"s": 1, "p": 2, "both": 3}
TMM_CHECK_FINITE = 1


class TmmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class TmmRtArgs(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int32), ("L", ctypes.c_int32),
        ("n_wl", ctypes.c_int32), ("n_theta", ctypes.c_int32),
        ("d", ctypes.c_void_p), ("nk", ctypes.c_void_p),
        ("n_mat", ctypes.c_int32), ("dispersive", ctypes.c_int32),
        ("mat", ctypes.c_void_p), ("wl", ctypes.c_void_p),
        ("sin_theta", ctypes.c_void_p), ("cos_theta", ctypes.c_void_p),
        ("pol_mask", ctypes.c_uint32),
        ("R", ctypes.c_void_p), ("T", ctypes.c_void_p),
        ("r", ctypes.c_void_p), ("t", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


_lib = None


def library() -> ctypes.CDLL:
    """Open libtmm_rt.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.tmm_rt.restype = ctypes.c_int
        lib.tmm_rt.argtypes = [ctypes.POINTER(TmmRtArgs), ctypes.c_int, ctypes.c_void_p]
        lib.tmm_status_string.restype = ctypes.c_char_p
        lib.tmm_status_string.argtypes = [ctypes.c_int]
        lib.tmm_last_error.restype = ctypes.c_char_p
        lib.tmm_version.restype = ctypes.c_char_p
        lib.tmm_rt_grad_workspace_size.restype = ctypes.c_size_t
        lib.tmm_rt_grad_workspace_size.argtypes = [ctypes.POINTER(TmmRtArgs)]
        lib.tmm_rt_grad_workspace_min_size.restype = ctypes.c_size_t
        lib.tmm_rt_grad_workspace_min_size.argtypes = [ctypes.POINTER(TmmRtArgs)]
        lib.tmm_rt_grad.restype = ctypes.c_int
        lib.tmm_rt_grad.argtypes = [ctypes.POINTER(TmmRtArgs)] + [ctypes.c_void_p] * 5 + \
            [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
        lib.tmm_rt_points.restype = ctypes.c_int
        lib.tmm_rt_points.argtypes = [ctypes.POINTER(TmmRtArgs), ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                      ctypes.c_void_p]
        lib.tmm_rt_grad_noalloc.restype = ctypes.c_int
        lib.tmm_rt_grad_noalloc.argtypes = [ctypes.POINTER(TmmRtArgs)] + [ctypes.c_void_p] * 4 + \
            [ctypes.c_int, ctypes.c_void_p]
        lib.tmm_rt_grad_noalloc_scratch_bytes.restype = ctypes.c_size_t
        lib.tmm_rt_grad_noalloc_scratch_bytes.argtypes = []
        _lib = lib
    return _lib


def _check(status: int):
    if status != TMM_OK:
        lib = library()
        raise TmmError(status, lib.tmm_last_error().decode() or lib.tmm_status_string(status).decode())


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(x) -> Optional[int]:
    return None if x is None else x.data_ptr()


def tmm_rt(d, nk, wl, sin_theta, cos_theta, *, mat=None, n_mat=None, dispersive=None,
           pol_mask: int = 3, R=None, T=None, r=None, t=None, flags: int = 0, stream=None) -> None:
    """Launch tmm_rt on device tensors (see include/tmm_rt.h for the layout).

    d [B, L] real; nk complex [n_mat, n_wl] or [n_mat]; mat [B, L+2] int32 or None;
    wl [n_wl], sin_theta / cos_theta [n_theta]; R, T real and r, t complex
    [B, P, n_theta, n_wl] outputs (any may be None).  All real tensors share one
    dtype (float64 or float32); complex ones are the matching complex dtype.
    flags: 0 or TMM_CHECK_FINITE (validate the device inputs first).
    """
    import torch
    real = d.dtype
    if real == torch.float64:
        dt, cdt = TMM_F64, torch.complex128
    elif real == torch.float32:
        dt, cdt = TMM_F32, torch.complex64
    else:
        raise TypeError("d must be float64 or float32")
    for name, x in (("wl", wl), ("sin_theta", sin_theta), ("cos_theta", cos_theta), ("R", R), ("T", T)):
        if x is not None and x.dtype != real:
            raise TypeError(f"{name} must be {real}")
    for name, x in (("nk", nk), ("r", r), ("t", t)):
        if x is not None and x.dtype != cdt:
            raise TypeError(f"{name} must be {cdt}")
    tensors = [d, nk, wl, sin_theta, cos_theta, mat, R, T, r, t]
    for x in tensors:
        if x is not None and (not x.is_cuda or not x.is_contiguous()):
            raise ValueError("every tensor must be a contiguous device tensor")
    if mat is not None and mat.dtype != torch.int32:
        raise TypeError("mat must be int32")
    B, L = d.shape
    n_mat = _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive)
    if dispersive is None:
        dispersive = nk.dim() == 2
    P = 2 if pol_mask == 3 else 1
    shape = (B, P, sin_theta.numel(), wl.numel())
    for name, x in (("R", R), ("T", T), ("r", r), ("t", t)):
        if x is not None and tuple(x.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    a = TmmRtArgs(B, L, wl.numel(), sin_theta.numel(), _ptr(d), _ptr(nk), n_mat, int(dispersive),
                  _ptr(mat), _ptr(wl), _ptr(sin_theta), _ptr(cos_theta), pol_mask,
                  _ptr(R), _ptr(T), _ptr(r), _ptr(t), flags)
    _check(library().tmm_rt(ctypes.byref(a), dt, _stream_handle(stream)))


def tmm_rt_points(d, nk, wl, sin_theta, cos_theta, points, *, mat=None, n_mat=None, dispersive=None,
                  pol_mask: int = 3, R=None, T=None, r=None, t=None, flags: int = 0, stream=None) -> None:
    """Launch tmm_rt_points: R, T (real) and / or r, t (complex) at the listed
    points (int64 device tensor of flat indices (b * n_theta + k) * n_wl + i),
    written into outputs laid out as tmm_rt's [B, P, n_theta, n_wl]; other
    elements are left as they are."""
    import torch
    real = d.dtype
    if real == torch.float64:
        dt, cdt = TMM_F64, torch.complex128
    elif real == torch.float32:
        dt, cdt = TMM_F32, torch.complex64
    else:
        raise TypeError("d must be float64 or float32")
    for name, x in (("wl", wl), ("sin_theta", sin_theta), ("cos_theta", cos_theta), ("R", R), ("T", T)):
        if x is not None and x.dtype != real:
            raise TypeError(f"{name} must be {real}")
    if nk.dtype != cdt:
        raise TypeError(f"nk must be {cdt}")
    for name, x in (("r", r), ("t", t)):
        if x is not None and x.dtype != cdt:
            raise TypeError(f"{name} must be {cdt}")
    if points.dtype != torch.int64 or points.dim() != 1:
        raise TypeError("points must be a 1-D int64 tensor")
    for x in (d, nk, wl, sin_theta, cos_theta, mat, R, T, r, t, points):
        if x is not None and (not x.is_cuda or not x.is_contiguous()):
            raise ValueError("every tensor must be a contiguous device tensor")
    if mat is not None and mat.dtype != torch.int32:
        raise TypeError("mat must be int32")
    B, L = d.shape
    n_mat = _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive)
    P = 2 if pol_mask == 3 else 1
    shape = (B, P, sin_theta.numel(), wl.numel())
    for name, x in (("R", R), ("T", T), ("r", r), ("t", t)):
        if x is not None and tuple(x.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    a = _rt_args(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive, pol_mask, R, T, r, t, flags=flags)
    _check(library().tmm_rt_points(ctypes.byref(a), _ptr(points), points.numel(), dt, _stream_handle(stream)))


def _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive) -> int:
    """Host-side size checks of the device tensors (the C library cannot see
    tensor sizes): every array must hold what the kernels will read.  Returns
    the number of index-table rows."""
    if d.dim() != 2:
        raise ValueError("d must be [B, L]")
    B, L = d.shape
    if sin_theta.dim() != 1 or cos_theta.dim() != 1 or sin_theta.numel() != cos_theta.numel():
        raise ValueError("sin_theta and cos_theta must be 1-D of equal length")
    if wl.dim() != 1:
        raise ValueError("wl must be 1-D")
    if dispersive is None:
        dispersive = nk.dim() == 2
    if dispersive and (nk.dim() != 2 or nk.shape[1] != wl.numel()):
        raise ValueError("a dispersive nk must be [n_mat, n_wl]")
    if not dispersive and nk.dim() != 1:
        raise ValueError("a constant nk must be [n_mat]")
    rows = nk.shape[0]
    if n_mat is None:
        n_mat = rows
    if n_mat > rows:
        raise ValueError(f"n_mat={n_mat} exceeds the {rows} rows of nk")
    if mat is not None:
        if tuple(mat.shape) != (B, L + 2):
            raise ValueError(f"mat must be [B, L+2] = {(B, L + 2)}, got {tuple(mat.shape)}")
    elif n_mat < B * (L + 2):
        raise ValueError(f"without mat, nk needs B*(L+2) = {B * (L + 2)} rows")
    return n_mat


def _rt_args(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive, pol_mask, R=None, T=None,
             r=None, t=None, flags=0):
    B, L = d.shape
    if dispersive is None:
        dispersive = nk.dim() == 2
    if n_mat is None:
        n_mat = nk.shape[0]
    return TmmRtArgs(B, L, wl.numel(), sin_theta.numel(), _ptr(d), _ptr(nk), n_mat, int(dispersive),
                     _ptr(mat), _ptr(wl), _ptr(sin_theta), _ptr(cos_theta), pol_mask,
                     _ptr(R), _ptr(T), _ptr(r), _ptr(t), flags)


def grad_workspace_size(d, nk, wl, sin_theta, cos_theta, *, mat=None, pol_mask=3, minimum=False) -> int:
    """Preferred (or, with minimum=True, smallest accepted) tmm_rt_grad workspace bytes."""
    _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, None, None)
    a = _rt_args(d, nk, wl, sin_theta, cos_theta, mat, None, None, pol_mask)
    lib = library()
    f = lib.tmm_rt_grad_workspace_min_size if minimum else lib.tmm_rt_grad_workspace_size
    return int(f(ctypes.byref(a)))


def tmm_rt_grad(d, nk, wl, sin_theta, cos_theta, *, mat=None, n_mat=None, dispersive=None,
                pol_mask: int = 3, dl_dR=None, dl_dT=None, grad_d=None, grad_n=None,
                workspace=None, R=None, T=None, flags: int = 0, stream=None) -> None:
    """Launch tmm_rt_grad (float64): gradients of sum(dl_dR * R + dl_dT * T) w.r.t.
    d [B, L] into grad_d [B, L] and w.r.t. the finite layers' indices into
    grad_n [B, L] complex128.  workspace: a uint8 device tensor of at least
    grad_workspace_size(..., minimum=True) bytes (the preferred size is
    allocated here if None)."""
    import torch
    if d.dtype != torch.float64:
        raise TypeError("tmm_rt_grad is float64 only")
    for x in (d, nk, wl, sin_theta, cos_theta, mat, dl_dR, dl_dT, grad_d, grad_n, R, T):
        if x is not None and (not x.is_cuda or not x.is_contiguous()):
            raise ValueError("every tensor must be a contiguous device tensor")
    B, L = d.shape
    P = 2 if pol_mask == 3 else 1
    shape = (B, P, sin_theta.numel(), wl.numel())
    for name, x in (("dl_dR", dl_dR), ("dl_dT", dl_dT), ("R", R), ("T", T)):
        if x is not None and (tuple(x.shape) != shape or x.dtype != torch.float64):
            raise ValueError(f"{name} must be float64 {shape}")
    if grad_d is not None and (tuple(grad_d.shape) != (B, L) or grad_d.dtype != torch.float64):
        raise ValueError("grad_d must be float64 [B, L]")
    if grad_n is not None and (tuple(grad_n.shape) != (B, L) or grad_n.dtype != torch.complex128):
        raise ValueError("grad_n must be complex128 [B, L]")
    if mat is not None and mat.dtype != torch.int32:
        raise TypeError("mat must be int32")
    if nk.dtype != torch.complex128:
        raise TypeError("nk must be complex128")
    n_mat = _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive)
    a = _rt_args(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive, pol_mask, R, T, flags=flags)
    lib = library()
    need = int(lib.tmm_rt_grad_workspace_size(ctypes.byref(a)))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=d.device)
    _check(lib.tmm_rt_grad(ctypes.byref(a), _ptr(dl_dR), _ptr(dl_dT), _ptr(grad_d), _ptr(grad_n),
                           _ptr(workspace), workspace.numel() * workspace.element_size(), TMM_F64,
                           _stream_handle(stream)))


def tmm_rt_grad_noalloc(d, nk, wl, sin_theta, cos_theta, *, mat=None, n_mat=None, dispersive=None,
                        pol_mask: int = 3, dl_dR=None, dl_dT=None, grad_d=None, grad_n=None, R=None, T=None,
                        flags: int = 0, stream=None) -> None:
    """tmm_rt_grad on the library's static scratch: no workspace argument and no
    device allocation anywhere in the call (same arguments and results)."""
    import torch
    if d.dtype != torch.float64:
        raise TypeError("tmm_rt_grad_noalloc is float64 only")
    for x in (d, nk, wl, sin_theta, cos_theta, mat, dl_dR, dl_dT, grad_d, grad_n, R, T):
        if x is not None and (not x.is_cuda or not x.is_contiguous()):
            raise ValueError("every tensor must be a contiguous device tensor")
    B, L = d.shape
    P = 2 if pol_mask == 3 else 1
    shape = (B, P, sin_theta.numel(), wl.numel())
    for name, x in (("dl_dR", dl_dR), ("dl_dT", dl_dT), ("R", R), ("T", T)):
        if x is not None and (tuple(x.shape) != shape or x.dtype != torch.float64):
            raise ValueError(f"{name} must be float64 {shape}")
    if grad_d is not None and (tuple(grad_d.shape) != (B, L) or grad_d.dtype != torch.float64):
        raise ValueError("grad_d must be float64 [B, L]")
    if grad_n is not None and (tuple(grad_n.shape) != (B, L) or grad_n.dtype != torch.complex128):
        raise ValueError("grad_n must be complex128 [B, L]")
    if mat is not None and mat.dtype != torch.int32:
        raise TypeError("mat must be int32")
    if nk.dtype != torch.complex128:
        raise TypeError("nk must be complex128")
    n_mat = _check_shapes(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive)
    a = _rt_args(d, nk, wl, sin_theta, cos_theta, mat, n_mat, dispersive, pol_mask, R, T, flags=flags)
    _check(library().tmm_rt_grad_noalloc(ctypes.byref(a), _ptr(dl_dR), _ptr(dl_dT), _ptr(grad_d), _ptr(grad_n),
                                         TMM_F64, _stream_handle(stream)))


# ---------------------------------------------------------------------------
# Convenience layer in the style of the paper's API.

def _dev(x, dtype, device):
    import torch
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)


def evaluate(d, nk, wl, sin_theta, cos_theta, *, mat=None, pol: str = "both", dtype="f64",
             amplitudes: bool = False, device="cuda"):
    """Allocate outputs on the device and run tmm_rt; returns a dict of tensors
    'R', 'T' (and 'r', 't') shaped [B, P, n_theta, n_wl]."""
    import torch
    real = torch.float64 if dtype in ("f64", torch.float64) else torch.float32
    cplx = torch.complex128 if real == torch.float64 else torch.complex64
    d_t = _dev(np.asarray(d) if not isinstance(d, torch.Tensor) else d, real, device)
    if d_t.dim() == 1:
        d_t = d_t.reshape(1, -1)
    nk_t = _dev(nk, cplx, device)
    wl_t = _dev(wl, real, device)
    s_t = _dev(sin_theta, real, device)
    c_t = _dev(cos_theta, real, device)
    mat_t = None if mat is None else _dev(mat, torch.int32, device)
    B = d_t.shape[0]
    P = 2 if pol == "both" else 1
    shape = (B, P, s_t.numel(), wl_t.numel())
    out = {"R": torch.empty(shape, dtype=real, device=device),
           "T": torch.empty(shape, dtype=real, device=device)}
    if amplitudes:
        out["r"] = torch.empty(shape, dtype=cplx, device=device)
        out["t"] = torch.empty(shape, dtype=cplx, device=device)
    tmm_rt(d_t, nk_t, wl_t, s_t, c_t, mat=mat_t, pol_mask=POL[pol], R=out["R"], T=out["T"],
           r=out.get("r"), t=out.get("t"))
    return out


def evaluate_workload(w, *, dtype="f64", amplitudes=False, pol="both", device="cuda"):
    """Run a workloads.Workload through tmm_rt."""
    return evaluate(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, pol=pol, dtype=dtype,
                    amplitudes=amplitudes, device=device)


def coh_tmm(pol: str, n, d, theta, wl, *, dtype="f64", amplitudes=True, device="cuda"):
    """Paper-style call: ``coh_tmm(pol, n, d, theta, wl)``.

    n  [L+2] or [N, L+2] indices (constant) or [N, L+2, n_wl] (dispersive), media
       0 and L+1 semi-infinite; d [L+2] or [N, L+2] thicknesses with +-inf (or any
       value) in the two semi-infinite slots, same length unit as wl; theta in
       rad; pol 's', 'p' or 'both'.  Returns a dict like the paper's
       ('R', 'T', 'r', 't' as [N, P, n_theta, n_wl]; P is squeezed out for a
       single polarisation).  sin/cos of theta are taken in float64 here.
    """
    import torch
    n = np.asarray(n.cpu() if isinstance(n, torch.Tensor) else n)
    d = np.asarray(d.detach().cpu() if isinstance(d, torch.Tensor) else d, dtype=np.float64)
    if d.ndim == 1:
        d = d[None]
    if n.ndim == 1 or (n.ndim == 2 and n.shape[0] != d.shape[0]):
        n = n[None]
    N, M = d.shape
    d_fin = np.ascontiguousarray(d[:, 1:M - 1])
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    wl = np.atleast_1d(np.asarray(wl, dtype=np.float64))
    if n.ndim == 3:
        nk = n.reshape(N * M, wl.size).astype(np.complex128)
    else:
        nk = n.reshape(N * M).astype(np.complex128)
    out = evaluate(d_fin, nk, wl, np.sin(theta), np.cos(theta), pol=pol, dtype=dtype,
                   amplitudes=amplitudes, device=device)
    if pol != "both":
        out = {k: v[:, 0] for k, v in out.items()}
    return out


def unpolarised(out):
    """(X_s + X_p) / 2 over the polarisation axis of a pol='both' result."""
    return {k: 0.5 * (v[:, 0] + v[:, 1]) for k, v in out.items() if k in ("R", "T")}


# ---------------------------------------------------------------------------
# Differentiable evaluation: forward through tmm_rt, backward through tmm_rt_grad.

def _autograd_function():
    import torch

    class TMMFunction(torch.autograd.Function):
        """R, T of B stacks with per-layer constant indices; differentiable w.r.t.
        the thicknesses d [B, L] and the layer indices n [B, L] (complex).  The
        ambient and substrate indices are constants."""

        @staticmethod
        def forward(ctx, d, n_layers, n_amb, n_sub, wl, sin_t, cos_t, pol_mask):
            B, L = d.shape
            nk = torch.cat([n_amb.reshape(1, 1).expand(B, 1), n_layers,
                            n_sub.reshape(1, 1).expand(B, 1)], dim=1).reshape(-1).contiguous()
            P = 2 if pol_mask == 3 else 1
            shape = (B, P, sin_t.numel(), wl.numel())
            R = torch.empty(shape, dtype=torch.float64, device=d.device)
            T = torch.empty(shape, dtype=torch.float64, device=d.device)
            d = d.contiguous()
            tmm_rt(d, nk, wl, sin_t, cos_t, pol_mask=pol_mask, R=R, T=T)
            ctx.save_for_backward(d, nk, wl, sin_t, cos_t)
            ctx.pol_mask = pol_mask
            return R, T

        @staticmethod
        def backward(ctx, gR, gT):
            d, nk, wl, sin_t, cos_t = ctx.saved_tensors
            B, L = d.shape
            want_d, want_n = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            gd = torch.empty((B, L), dtype=torch.float64, device=d.device)
            gn = torch.empty((B, L), dtype=torch.complex128, device=d.device)
            tmm_rt_grad(d, nk, wl, sin_t, cos_t, pol_mask=ctx.pol_mask,
                        dl_dR=None if gR is None else gR.contiguous(),
                        dl_dT=None if gT is None else gT.contiguous(),
                        grad_d=gd, grad_n=gn)
            return (gd if want_d else None, gn if want_n else None) + (None,) * 6

    return TMMFunction


_TMMFunction = None


def rt_differentiable(d, n_layers, n_amb, n_sub, wl, sin_theta, cos_theta, pol: str = "both"):
    """(R, T) as differentiable torch tensors [B, P, n_theta, n_wl] (float64).
    d [B, L] float64 and n_layers [B, L] complex128 on the device (either may
    require grad); n_amb, n_sub complex scalars; sin/cos of the angles in float64."""
    import torch
    global _TMMFunction
    if _TMMFunction is None:
        _TMMFunction = _autograd_function()
    dev = d.device
    as_c = lambda x: torch.as_tensor(x, dtype=torch.complex128, device=dev)
    return _TMMFunction.apply(d, n_layers.to(torch.complex128), as_c(n_amb), as_c(n_sub),
                              wl.contiguous(), sin_theta.contiguous(), cos_theta.contiguous(), POL[pol])


def coh_tmm_torch(pol: str, n, d, theta, wl, device="cuda"):
    """Paper-style differentiable call (App. A.3): n [L+2] or [N, L+2] indices,
    d [L+2] or [N, L+2] thicknesses (the two semi-infinite slots are ignored; a
    torch tensor with requires_grad gets gradients on its finite entries), theta
    in rad, wl in the unit of d.  Returns {'R', 'T'} differentiable tensors."""
    import torch
    if not isinstance(d, torch.Tensor):
        d = torch.as_tensor(np.asarray(d, dtype=np.float64))
    d2 = d if d.dim() == 2 else d.unsqueeze(0)
    N, M = d2.shape
    d_fin = d2[:, 1:M - 1].to(device=device, dtype=torch.float64)
    n_t = torch.as_tensor(n) if not isinstance(n, torch.Tensor) else n
    n_t = n_t.to(device=device, dtype=torch.complex128)
    if n_t.dim() == 1:
        n_t = n_t.unsqueeze(0).expand(N, M)
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    wl_t = torch.as_tensor(np.atleast_1d(np.asarray(wl, dtype=np.float64)), device=device)
    s = torch.as_tensor(np.sin(theta), device=device)
    c = torch.as_tensor(np.cos(theta), device=device)
    # the semi-infinite media must be the same for every stack here
    R, T = rt_differentiable(d_fin, n_t[:, 1:M - 1].contiguous(), n_t[0, 0], n_t[0, M - 1], wl_t, s, c, pol)
    if pol != "both":
        R, T = R[:, 0], T[:, 0]
    return {"R": R, "T": T}
