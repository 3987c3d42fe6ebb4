"""ctypes binding of the ragged-batch interface (include/tmm_ragged.h).

Argument marshalling only; the plan, the work list, the autotuning and the
kernels live in libtmm_rt.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import tmm


class RaggedData(ctypes.Structure):
    _fields_ = [("d", ctypes.c_void_p), ("mat", ctypes.c_void_p), ("ends", ctypes.c_void_p),
                ("wl", ctypes.c_void_p), ("sin_theta", ctypes.c_void_p), ("cos_theta", ctypes.c_void_p),
                ("nk", ctypes.c_void_p), ("n_mat", ctypes.c_int32), ("R", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("r", ctypes.c_void_p), ("t", ctypes.c_void_p)]


_bound = False


def _lib():
    global _bound
    lib = tmm.library()
    if not _bound:
        P = ctypes.c_void_p
        lib.tmm_ragged_plan_create.restype = ctypes.c_int
        lib.tmm_ragged_plan_create.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_uint32, ctypes.POINTER(P)]
        lib.tmm_ragged_plan_destroy.restype = ctypes.c_int
        lib.tmm_ragged_plan_destroy.argtypes = [P]
        lib.tmm_ragged_plan_output_size.restype = ctypes.c_int64
        lib.tmm_ragged_plan_output_size.argtypes = [P]
        lib.tmm_ragged_plan_output_offsets.restype = ctypes.c_int
        lib.tmm_ragged_plan_output_offsets.argtypes = [P, P]
        lib.tmm_ragged_plan_shape.restype = ctypes.c_int
        lib.tmm_ragged_plan_shape.argtypes = [P, ctypes.c_int, P]
        lib.tmm_ragged_plan_set_shape.restype = ctypes.c_int
        lib.tmm_ragged_plan_set_shape.argtypes = [P, ctypes.c_int, P]
        for name in ("tmm_ragged_run", "tmm_rt_ragged", "tmm_ragged_capture"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [P, ctypes.POINTER(RaggedData), ctypes.c_int, P]
        lib.tmm_ragged_replay.restype = ctypes.c_int
        lib.tmm_ragged_replay.argtypes = [P, P]
        _bound = True
    return lib


class RaggedPlan:
    """Plan for one ragged batch shape (host offset arrays [B+1])."""

    def __init__(self, layer_off, wl_off, th_off, pol: str = "both"):
        self.layer_off = np.ascontiguousarray(layer_off, dtype=np.int64)
        self.wl_off = np.ascontiguousarray(wl_off, dtype=np.int64)
        self.th_off = np.ascontiguousarray(th_off, dtype=np.int64)
        self.B = self.layer_off.size - 1
        if self.wl_off.size != self.B + 1 or self.th_off.size != self.B + 1:
            raise ValueError("offset arrays must all have B+1 entries")
        h = ctypes.c_void_p()
        tmm._check(_lib().tmm_ragged_plan_create(self.B, self.layer_off.ctypes.data, self.wl_off.ctypes.data,
                                                 self.th_off.ctypes.data, tmm.POL[pol], ctypes.byref(h)))
        self.h = h
        self.P = 2 if pol == "both" else 1
        self._data = None

    def close(self):
        if self.h:
            _lib().tmm_ragged_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def output_size(self) -> int:
        return int(_lib().tmm_ragged_plan_output_size(self.h))

    def output_offsets(self) -> np.ndarray:
        out = np.empty(self.B + 1, dtype=np.int64)
        tmm._check(_lib().tmm_ragged_plan_output_offsets(self.h, out.ctypes.data))
        return out

    def _pack(self, d, mat, ends, wl, sin_t, cos_t, nk, R, T, r=None, t=None):
        import torch
        n_layers, n_wl, n_th = int(self.layer_off[-1]), int(self.wl_off[-1]), int(self.th_off[-1])
        real = wl.dtype
        cplx = torch.complex128 if real == torch.float64 else torch.complex64
        checks = [("d", d, (n_layers,), real), ("mat", mat, (n_layers,), torch.int32),
                  ("ends", ends, (self.B, 2), torch.int32), ("wl", wl, (n_wl,), real),
                  ("sin_theta", sin_t, (n_th,), real), ("cos_theta", cos_t, (n_th,), real),
                  ("R", R, (self.output_size,), real), ("T", T, (self.output_size,), real),
                  ("r", r, (self.output_size,), cplx), ("t", t, (self.output_size,), cplx)]
        for name, x, shape, dt in checks:
            if x is None:
                continue
            if tuple(x.shape) != shape or x.dtype != dt or not x.is_cuda or not x.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} device tensor of shape {shape}")
        if nk.dim() != 2 or nk.shape[1] != n_wl or nk.dtype != cplx or not nk.is_cuda or not nk.is_contiguous():
            raise ValueError(f"nk must be a contiguous {cplx} device tensor [n_mat, {n_wl}]")
        if R is None and T is None and r is None and t is None:
            raise ValueError("at least one of R, T, r, t")
        if real == torch.float64:
            dt = tmm.TMM_F64
        elif real == torch.float32:
            dt = tmm.TMM_F32
        else:
            raise TypeError("real tensors must be float64 or float32")
        p = tmm._ptr
        return RaggedData(p(d), p(mat), p(ends), p(wl), p(sin_t), p(cos_t), p(nk), nk.shape[0], p(R), p(T), p(r),
                          p(t)), dt

    def run(self, d, mat, ends, wl, sin_t, cos_t, nk, R=None, T=None, r=None, t=None, stream=None):
        """Evaluate every stack into R, T (real) and / or r, t (complex), each
        [output_size] in the plan's output layout."""
        data, dt = self._pack(d, mat, ends, wl, sin_t, cos_t, nk, R, T, r, t)
        tmm._check(_lib().tmm_rt_ragged(self.h, ctypes.byref(data), dt, tmm._stream_handle(stream)))

    def shape(self, dtype="f64") -> dict:
        """The autotuned launch shape for dtype (after the first run)."""
        out = np.zeros(4, dtype=np.int32)
        tmm._check(_lib().tmm_ragged_plan_shape(self.h, tmm.TMM_F64 if dtype == "f64" else tmm.TMM_F32,
                                                out.ctypes.data))
        return {"workgroups_per_cu": int(out[0]), "grain": int(out[1]), "waves_per_workgroup": int(out[2]),
                "lanes_per_point": int(out[3]), "points_per_unit": 64 // int(out[3])}

    def set_shape(self, dtype="f64", *, workgroups_per_cu=1, grain=1, waves_per_workgroup=12, lanes_per_point=1):
        """Fix the launch shape for dtype instead of tuning it on the first run."""
        sh = np.array([workgroups_per_cu, grain, waves_per_workgroup, lanes_per_point], dtype=np.int32)
        tmm._check(_lib().tmm_ragged_plan_set_shape(self.h, tmm.TMM_F64 if dtype == "f64" else tmm.TMM_F32,
                                                    sh.ctypes.data))

    def capture(self, d, mat, ends, wl, sin_t, cos_t, nk, R=None, T=None, r=None, t=None, stream=None):
        """Capture a run into the plan's HIP graph (stream: a non-default torch stream)."""
        data, dt = self._pack(d, mat, ends, wl, sin_t, cos_t, nk, R, T, r, t)
        self._data = (d, mat, ends, wl, sin_t, cos_t, nk, R, T, r, t)  # keep the captured buffers alive
        tmm._check(_lib().tmm_ragged_capture(self.h, ctypes.byref(data), dt, tmm._stream_handle(stream)))

    def replay(self, stream=None):
        tmm._check(_lib().tmm_ragged_replay(self.h, tmm._stream_handle(stream)))


def to_device(rw, dtype="f64", device="cuda"):
    """Device tensors of a workloads.RaggedWorkload: (d, mat, ends, wl, sin, cos, nk)."""
    import torch
    real = torch.float64 if dtype == "f64" else torch.float32
    cplx = torch.complex128 if dtype == "f64" else torch.complex64
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    return (t(rw.d, real), t(rw.mat, torch.int32), t(rw.ends, torch.int32), t(rw.wl, real), t(rw.sin_t, real),
            t(rw.cos_t, real), t(rw.nk, cplx))
