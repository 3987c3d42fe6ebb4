"""Plain complex128 CPU oracle for the batched transfer-matrix method.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this package, and this package imports nothing from the product path.

The arithmetic lives in ``tmm_oracle.c`` (plain C, ``double complex``, built
without fast-math, OpenMP over stacks); this module only builds it with gcc and
marshals numpy arrays.  See the header of ``tmm_oracle.c`` for the equations it
follows, the readings it takes, and which pins hold it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_tmm.so")
_lib = None


def compile_source(src: str, out: str) -> str:
    """gcc, C11, no fast-math, no FMA contraction, OpenMP."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle_tmm.so``."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


class using:
    """Context manager that points this module at another build of the oracle
    source (the pin-strength tests load deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _bind(ctypes.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _bind(lib):
    P = ctypes.c_void_p
    lib.oracle_rt.restype = ctypes.c_int
    lib.oracle_rt.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, ctypes.c_int,
                                                    P, P, P, P, ctypes.c_uint,
                                                    P, P, P, P, P]
    lib.oracle_rt_points.restype = ctypes.c_int
    lib.oracle_rt_points.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, ctypes.c_int,
                                                           P, P, P, P, ctypes.c_int64,
                                                           P, P, P, P, P, P]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_rt_dir_cs.restype = ctypes.c_int
    lib.oracle_rt_dir_cs.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P, P, P, ctypes.c_uint,
                                                           P, P, P, P, P]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        _lib = _bind(lib)
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def rt(d, nk, wl, sin_t, cos_t, *, mat=None, dispersive=None, pol="both",
       want_amplitudes=True, flip=None):
    """Evaluate R, T (and r, t) for a batch of stacks.

    d        [B, L] float64 thicknesses (same length unit as ``wl``)
    nk       complex table: [n_mat, n_wl] (dispersive) or [n_mat] (constant)
    mat      [B, L+2] int32 row ids into ``nk``; None means row = b*(L+2)+j
    wl       [n_wl] vacuum wavelengths; sin_t, cos_t [n_theta]
    pol      's', 'p' or 'both' (output polarisation axis: s then p)
    Returns a dict with 'R', 'T' [B, P, n_theta, n_wl] float64 and, when
    requested, 'r', 't' complex128 of the same shape, plus 'threads'.
    """
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    if d.ndim != 2:
        raise ValueError("d must be [B, L]")
    B, L = d.shape
    nk = np.ascontiguousarray(nk, dtype=np.complex128)
    wl = np.ascontiguousarray(wl, dtype=np.float64).ravel()
    sin_t = np.ascontiguousarray(sin_t, dtype=np.float64).ravel()
    cos_t = np.ascontiguousarray(cos_t, dtype=np.float64).ravel()
    if sin_t.shape != cos_t.shape:
        raise ValueError("sin_t and cos_t differ in length")
    if dispersive is None:
        dispersive = nk.ndim == 2
    if dispersive and (nk.ndim != 2 or nk.shape[1] != wl.size):
        raise ValueError("dispersive nk must be [n_mat, n_wl]")
    n_mat = nk.shape[0]
    if mat is not None:
        mat = np.ascontiguousarray(mat, dtype=np.int32)
        if mat.shape != (B, L + 2):
            raise ValueError("mat must be [B, L+2]")
    mask = {"s": 1, "p": 2, "both": 3}[pol]
    P = 2 if mask == 3 else 1
    shape = (B, P, sin_t.size, wl.size)
    R = np.empty(shape)
    T = np.empty(shape)
    r = np.empty(shape, np.complex128) if want_amplitudes else None
    t = np.empty(shape, np.complex128) if want_amplitudes else None
    if flip is not None:
        flip = np.ascontiguousarray(flip, dtype=np.uint8)
        if flip.shape != (L + 2,):
            raise ValueError("flip must be [L+2]")
    th = lib.oracle_rt(B, L, wl.size, sin_t.size, _ptr(d), _ptr(nk), n_mat,
                       int(bool(dispersive)), _ptr(mat), _ptr(wl), _ptr(sin_t),
                       _ptr(cos_t), mask, _ptr(R), _ptr(T), _ptr(r), _ptr(t),
                       _ptr(flip))
    if th < 0:
        raise ValueError("oracle_rt rejected its arguments")
    out = {"R": R, "T": T, "threads": th}
    if want_amplitudes:
        out["r"] = r
        out["t"] = t
    return out


def rt_points(d, nk, wl, sin_t, cos_t, b, i, k, pol, *, mat=None, dispersive=None):
    """R, T at an explicit list of points: stack b[m], wavelength index i[m],
    angle index k[m], polarisation pol[m] (0 = s, 1 = p); same inputs as ``rt``.
    Returns (R [n], T [n])."""
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    B, L = d.shape
    nk = np.ascontiguousarray(nk, dtype=np.complex128)
    wl = np.ascontiguousarray(wl, dtype=np.float64).ravel()
    sin_t = np.ascontiguousarray(sin_t, dtype=np.float64).ravel()
    cos_t = np.ascontiguousarray(cos_t, dtype=np.float64).ravel()
    if dispersive is None:
        dispersive = nk.ndim == 2
    if dispersive and (nk.ndim != 2 or nk.shape[1] != wl.size):
        raise ValueError("dispersive nk must be [n_mat, n_wl]")
    if mat is not None:
        mat = np.ascontiguousarray(mat, dtype=np.int32)
        if mat.shape != (B, L + 2):
            raise ValueError("mat must be [B, L+2]")
    idx = [np.ascontiguousarray(x, dtype=np.int32).ravel() for x in (b, i, k, pol)]
    n = idx[0].size
    if any(x.size != n for x in idx):
        raise ValueError("b, i, k, pol differ in length")
    R = np.empty(n)
    T = np.empty(n)
    th = lib.oracle_rt_points(B, L, wl.size, sin_t.size, _ptr(d), _ptr(nk), nk.shape[0],
                              int(bool(dispersive)), _ptr(mat), _ptr(wl), _ptr(sin_t), _ptr(cos_t),
                              n, *[_ptr(x) for x in idx], _ptr(R), _ptr(T))
    if th < 0:
        raise ValueError("oracle_rt_points rejected its arguments")
    return R, T


def rt_dir_cs(d, nk, wl, sin_t, cos_t, *, gR=None, gT=None, vd=None, vn=None, pol="both",
              dispersive=None):
    """Complex-step directional derivative, per stack, of
    sum(gR * R + gT * T) along d -> d + e vd, n_j -> n_j + e vn (finite layers).

    Per-layer index table only: nk has rows b*(L+2)+j ([B*(L+2)] or
    [B*(L+2), n_wl]).  gR, gT: [B, P, n_theta, n_wl]; vd: [B, L] real;
    vn: [B, L] complex.  Returns D [B].
    """
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    B, L = d.shape
    nk = np.ascontiguousarray(nk, dtype=np.complex128)
    wl = np.ascontiguousarray(wl, dtype=np.float64).ravel()
    sin_t = np.ascontiguousarray(sin_t, dtype=np.float64).ravel()
    cos_t = np.ascontiguousarray(cos_t, dtype=np.float64).ravel()
    if dispersive is None:
        dispersive = nk.ndim == 2
    if nk.shape[0] != B * (L + 2):
        raise ValueError("nk must have one row per medium of every stack")
    mask = {"s": 1, "p": 2, "both": 3}[pol]
    P = 2 if mask == 3 else 1
    shape = (B, P, sin_t.size, wl.size)
    conv = lambda a, dt, shp: None if a is None else np.ascontiguousarray(np.broadcast_to(a, shp), dtype=dt)
    gR = conv(gR, np.float64, shape)
    gT = conv(gT, np.float64, shape)
    vd = conv(vd, np.float64, (B, L))
    vn = conv(vn, np.complex128, (B, L))
    D = np.empty(B)
    th = lib.oracle_rt_dir_cs(B, L, wl.size, sin_t.size, _ptr(d), _ptr(nk), int(bool(dispersive)),
                              _ptr(wl), _ptr(sin_t), _ptr(cos_t), mask, _ptr(gR), _ptr(gT),
                              _ptr(vd), _ptr(vn), _ptr(D))
    if th < 0:
        raise ValueError("oracle_rt_dir_cs rejected its arguments")
    return D


def rt_grad_cs(d, nk, wl, sin_t, cos_t, *, gR=None, gT=None, pol="both"):
    """Full gradient per stack by one complex-step pass per parameter:
    returns (grad_d [B, L], grad_n [B, L] complex = dl/dRe n + i dl/dIm n)."""
    d = np.asarray(d, dtype=np.float64)
    B, L = d.shape
    gd = np.empty((B, L))
    gn = np.empty((B, L), np.complex128)
    for j in range(L):
        e = np.zeros((B, L))
        e[:, j] = 1.0
        gd[:, j] = rt_dir_cs(d, nk, wl, sin_t, cos_t, gR=gR, gT=gT, vd=e, pol=pol)
        re = rt_dir_cs(d, nk, wl, sin_t, cos_t, gR=gR, gT=gT, vn=e.astype(complex), pol=pol)
        im = rt_dir_cs(d, nk, wl, sin_t, cos_t, gR=gR, gT=gT, vn=1j * e, pol=pol)
        gn[:, j] = re + 1j * im
    return gd, gn


def max_threads() -> int:
    return _load().oracle_max_threads()
