"""ctypes binding of the learned surrogate (include/tmm_surrogate.h) and the
training / calibration driver around it.

Argument marshalling and orchestration only: data generation runs in tmm_rt,
every forward, backward and optimiser step in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import json
import time
from dataclasses import dataclass

import numpy as np

from . import tmm, workloads


class SurrogateConfig(ctypes.Structure):
    _fields_ = [
        ("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_layers", ctypes.c_int32),
        ("n_out", ctypes.c_int32), ("n_members", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("in_shift", ctypes.c_float), ("in_scale", ctypes.c_float),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float), ("weight_decay", ctypes.c_float),
        ("gemm_tile", ctypes.c_int32), ("sigma_window", ctypes.c_int32),
    ]


_bound = False


def _lib():
    global _bound
    lib = tmm.library()
    if not _bound:
        P = ctypes.c_void_p
        lib.tmm_surrogate_create.restype = ctypes.c_int
        lib.tmm_surrogate_create.argtypes = [ctypes.POINTER(SurrogateConfig), ctypes.POINTER(P)]
        lib.tmm_surrogate_destroy.restype = ctypes.c_int
        lib.tmm_surrogate_destroy.argtypes = [P]
        lib.tmm_surrogate_param_count.restype = ctypes.c_size_t
        lib.tmm_surrogate_param_count.argtypes = [P]
        lib.tmm_surrogate_export.restype = ctypes.c_int
        lib.tmm_surrogate_export.argtypes = [P, P, ctypes.c_size_t]
        lib.tmm_surrogate_import.restype = ctypes.c_int
        lib.tmm_surrogate_import.argtypes = [P, P, ctypes.c_size_t]
        lib.tmm_surrogate_train_step.restype = ctypes.c_int
        lib.tmm_surrogate_train_step.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_float, P, P]
        lib.tmm_surrogate_gradients.restype = ctypes.c_int
        lib.tmm_surrogate_gradients.argtypes = [P, P, P, ctypes.c_int32, P, P]
        lib.tmm_surrogate_predict.restype = ctypes.c_int
        lib.tmm_surrogate_predict.argtypes = [P, P, ctypes.c_int32, P, P, P, P]
        lib.tmm_surrogate_predict_fallback.restype = ctypes.c_int
        lib.tmm_surrogate_predict_fallback.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(tmm.TmmRtArgs),
                                                       ctypes.c_float, ctypes.c_float, P,
                                                       ctypes.POINTER(ctypes.c_int64), P]
        _bound = True
    return lib


def _p(x):
    return None if x is None else x.data_ptr()


class Surrogate:
    """Ensemble MLP surrogate living in device memory (one handle)."""

    def __init__(self, n_in, n_out, *, n_hidden=1024, n_layers=5, n_members=5, max_batch=4096, seed=0,
                 in_shift=0.0, in_scale=1.0, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, gemm_tile=0,
                 sigma_window=0):
        self.cfg = SurrogateConfig(n_in, n_hidden, n_layers, n_out, n_members, max_batch, seed,
                                   in_shift, in_scale, 0.0, beta1, beta2, eps, weight_decay, gemm_tile,
                                   sigma_window)
        h = ctypes.c_void_p()
        tmm._check(_lib().tmm_surrogate_create(ctypes.byref(self.cfg), ctypes.byref(h)))
        self.h = h
        self.n_in, self.n_out, self.E = n_in, n_out, n_members
        self.sigma_window = sigma_window

    def close(self):
        if self.h:
            _lib().tmm_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(_lib().tmm_surrogate_param_count(self.h))

    def export(self) -> np.ndarray:
        buf = np.empty(self.param_count * self.E, dtype=np.float32)
        tmm._check(_lib().tmm_surrogate_export(self.h, buf.ctypes.data, buf.size))
        return buf.reshape(self.E, self.param_count)

    def load(self, params: np.ndarray):
        buf = np.ascontiguousarray(params, dtype=np.float32).ravel()
        tmm._check(_lib().tmm_surrogate_import(self.h, buf.ctypes.data, buf.size))

    def _check_xy(self, x, y=None):
        import torch
        for name, t, cols in (("x", x, self.n_in), ("y", y, self.n_out)):
            if t is None:
                continue
            if t.dim() != 2 or t.shape[1] != cols or t.dtype != torch.float32 or not t.is_contiguous() \
                    or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 device tensor [B, {cols}]")
        if y is not None and y.shape[0] != x.shape[0]:
            raise ValueError("x and y differ in batch size")

    def train_step(self, x, y, lr, loss=None):
        self._check_xy(x, y)
        import torch
        if loss is not None and (loss.numel() < self.E or loss.dtype != torch.float32 or not loss.is_cuda):
            raise ValueError("loss must be a device float32 tensor with one entry per member")
        tmm._check(_lib().tmm_surrogate_train_step(self.h, _p(x), _p(y), x.shape[0], lr, _p(loss),
                                                   tmm._stream_handle(None)))

    def gradients(self, x, y):
        import torch
        self._check_xy(x, y)
        g = torch.empty((self.E, self.param_count), dtype=torch.float32, device=x.device)
        tmm._check(_lib().tmm_surrogate_gradients(self.h, _p(x), _p(y), x.shape[0], _p(g),
                                                  tmm._stream_handle(None)))
        return g

    def predict(self, x, *, sigma=True, members=False):
        import torch
        self._check_xy(x)
        B = x.shape[0]
        mean = torch.empty((B, self.n_out), dtype=torch.float32, device=x.device)
        sig = torch.empty_like(mean) if sigma else None
        mem = torch.empty((self.E, B, self.n_out), dtype=torch.float32, device=x.device) if members else None
        tmm._check(_lib().tmm_surrogate_predict(self.h, _p(x), B, _p(mean), _p(sig), _p(mem),
                                                tmm._stream_handle(None)))
        return mean, sig, mem

    def predict_fallback(self, x, task: "Task", err_scale: float, bound: float):
        """Surrogate with transfer-matrix fallback (point granularity) for the stacks
        x [B, n_in] of task.  Returns (out [B, n_out], number of outputs replaced)."""
        import torch
        self._check_xy(x)
        if task.n_out != self.n_out or task.n_layers != self.n_in or task.wl.dtype != torch.float32:
            raise ValueError("task does not match the surrogate (layers, outputs, float32 grids)")
        tmpl = task.args(x.shape[0])
        out = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        nf = ctypes.c_int64(0)
        tmm._check(_lib().tmm_surrogate_predict_fallback(self.h, _p(x), x.shape[0], ctypes.byref(tmpl),
                                                         err_scale, bound, _p(out), ctypes.byref(nf),
                                                         tmm._stream_handle(None)))
        return out, int(nf.value)


# ---------------------------------------------------------------------------
# Surrogate tasks: a fixed material sequence and grids; the thicknesses vary.
#   "surrogate_batch"  30 alternating Cauchy layers -> R over 256 wl x 16 angles x s, p
#   "dataset_example"  the paper's App. A.2 dataset shape: 10 layers 2.0 / 1.4 between
#                      2.5 and 1.0 -> s-polarised R over 128 wl at normal incidence

INSTANCES = {
    "surrogate_batch": dict(pol="both", d_range=(20.0, 250.0), n_wl=256),
    "dataset_example": dict(pol="s", d_range=(5.0, 180.0), n_wl=128),
}


@dataclass
class Task:
    """Device tensors describing the fixed part of the stacks (materials, grids)."""
    n_layers: int
    nk: object
    mat_row: object      # [1, L+2] int32, the material sequence of every stack
    wl: object
    sin_t: object
    cos_t: object
    n_wl: int
    n_theta: int
    pol_mask: int = 3    # tmm.POL: 1 s, 2 p, 3 both

    @property
    def P(self):
        return 2 if self.pol_mask == 3 else 1

    @property
    def n_out(self):
        return self.P * self.n_theta * self.n_wl

    def mat(self, B):
        """Material ids [B, L+2] (a contiguous device tensor with exactly B rows)."""
        cache = self.__dict__.setdefault("_mat_cache", {})
        if B not in cache:
            cache.clear()
            cache[B] = self.mat_row.expand(B, self.n_layers + 2).contiguous()
        return cache[B]

    def args(self, B, d=None, R=None):
        """tmm_rt arguments for B stacks (d [B, L] thicknesses, R output); the
        material-id array it points to has exactly B rows."""
        mat = self.mat(B)
        return tmm.TmmRtArgs(B, self.n_layers, self.n_wl, self.n_theta, tmm._ptr(d), tmm._ptr(self.nk),
                             self.nk.shape[0], int(self.nk.dim() == 2), tmm._ptr(mat),
                             tmm._ptr(self.wl), tmm._ptr(self.sin_t), tmm._ptr(self.cos_t), self.pol_mask,
                             tmm._ptr(R), None, None, None)


def make_task(dtype="f32", device="cuda", L=30, n_wl=None, n_theta=16, instance="surrogate_batch"):
    """The fixed part of a surrogate instance ("surrogate_batch": L alternating
    layers over n_wl x n_theta, s and p; "dataset_example": the paper's App. A.2
    shape over n_wl wavelengths, s only; L and n_theta do not apply to it)."""
    import torch
    if n_wl is None:
        n_wl = INSTANCES[instance]["n_wl"]
    if instance == "surrogate_batch":
        w = workloads.surrogate_batch(B=1, L=L, n_wl=n_wl, n_theta=n_theta)
    elif instance == "dataset_example":
        w = workloads.dataset_example(B=1, n_wl=n_wl)
    else:
        raise ValueError(f"unknown surrogate instance {instance!r}")
    real = torch.float32 if dtype == "f32" else torch.float64
    cplx = torch.complex64 if dtype == "f32" else torch.complex128
    mat_row = torch.as_tensor(w.mat[:1], dtype=torch.int32, device=device)
    return Task(w.L, torch.as_tensor(w.nk, dtype=cplx, device=device), mat_row,
                torch.as_tensor(w.wl, dtype=real, device=device),
                torch.as_tensor(w.sin_t, dtype=real, device=device),
                torch.as_tensor(w.cos_t, dtype=real, device=device), w.wl.size, w.theta.size,
                tmm.POL[INSTANCES[instance]["pol"]])


def generate(task: Task, d, chunk=65536):
    """R spectra [B, n_out] of the stacks with thicknesses d [B, L] (device), by
    tmm_rt in the task's real type."""
    import torch
    real = task.wl.dtype
    B = d.shape[0]
    out = torch.empty((B, task.n_out), dtype=real, device=d.device)
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        dd = d[b0:b1].to(real).contiguous()
        tmm.tmm_rt(dd, task.nk, task.wl, task.sin_t, task.cos_t, mat=task.mat(b1 - b0), pol_mask=task.pol_mask,
                   R=out[b0:b1].view(b1 - b0, task.P, task.n_theta, task.n_wl))
    return out


def window_sigma(sigma, task, window):
    """sigma [B, n_out] -> the largest sigma of each output's spectrum row (one
    stack, polarisation and angle) within `window` wavelengths of it, the
    estimate tmm_surrogate_predict_fallback compares with the bound for a handle
    whose sigma_window is `window` (NaN propagates)."""
    import torch
    if window <= 0:
        return sigma
    B = sigma.shape[0]
    rows = sigma.reshape(B * task.P * task.n_theta, 1, task.n_wl)
    nan = torch.isnan(rows)
    m = torch.nn.functional.max_pool1d(torch.nan_to_num(rows, nan=0.0), 2 * window + 1, stride=1, padding=window)
    if bool(nan.any()):
        nanw = torch.nn.functional.max_pool1d(nan.float(), 2 * window + 1, stride=1, padding=window) > 0
        m = torch.where(nanw, torch.full_like(m, float("nan")), m)
    return m.reshape(B, -1)


def calibrate(mean, sigma, truth, bound, margin=1.0, spread_factor=1.0):
    """Point-level error scale: tau is the smallest sigma among the outputs of this
    set whose error |mean - truth| exceeds margin * bound; err_scale = bound / tau'
    with tau' just below tau / spread_factor, so that accepting the outputs with
    err_scale * sigma <= bound (sigma <= tau') keeps every accepted error of this
    set within margin * bound.  Returns (err_scale, accepted fraction of outputs);
    err_scale is inf (nothing accepted) when the smallest-sigma output is bad, 0
    (everything accepted) when no output is bad.  margin < 1 leaves room in the
    error and spread_factor > 1 in the spread for the held-out data the scale is
    then used on: on new data an output can fall below every bad calibration
    output's spread and still miss the bound."""
    import torch
    bad = (mean - truth).abs() > margin * bound
    if not bool(bad.any()):
        return 0.0, 1.0
    tau = float(sigma[bad].min()) / spread_factor
    tau = float(np.nextafter(np.float32(tau), np.float32(0)))
    if not tau > 0:
        return float("inf"), 0.0
    frac = float((sigma <= tau).double().mean())
    return float(bound / tau), frac


def _log(line):
    print(line, flush=True)


def train(sur: Surrogate, x, y, *, epochs, batch, lr_max=1e-3, lr_min=1e-5, seed=0, log_every=0, log=_log):
    """Adam over shuffled mini-batches with a cosine learning-rate schedule.
    Returns the per-epoch mean training loss of every member."""
    import torch
    N = x.shape[0]
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    loss = torch.zeros(sur.E, dtype=torch.float32, device=x.device)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(x.device)
        acc = torch.zeros(sur.E, dtype=torch.float64, device=x.device)
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            xb = x.index_select(0, idx)
            yb = y.index_select(0, idx)
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + np.cos(np.pi * step / max(1, total)))
            sur.train_step(xb, yb, float(lr), loss)
            acc += loss.double()
            step += 1
        hist.append((acc / steps_per_epoch).cpu().numpy().tolist())
        if log_every and (ep + 1) % log_every == 0:
            log(json.dumps({"epoch": ep + 1, "loss": hist[-1]}))
    return hist


# ---------------------------------------------------------------------------
# End-to-end driver: data from tmm_rt, training, calibration, throughput.

def _timeit(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps / 1e3


def run(n_train=2_000_000, n_cal=34_464, n_test=65_536, epochs=20, batch=4096, hidden=1024, layers=5,
        members=5, lr_max=1e-3, lr_min=1e-5, eval_batch=65536, bounds=(1e-3,), margin=0.5, seed=0,
        infer_batch=16384, instance="surrogate_batch", n_wl=None, sigma_window=4, spread_factor=2.0,
        log=_log):
    """Train the surrogate on tmm_rt data and report accuracy and throughput.
    The held-out stacks (n_cal + n_test, 100 000 by default) are split into a
    calibration part, on which the point-level error scale is fitted with the
    given margin, and a test part (also the throughput batch when it holds
    eval_batch stacks), on which the accepted fraction and the errors are
    measured.  Inference runs on a second handle whose internal batch is
    infer_batch rows (larger GEMMs than the training batch), loaded with the
    trained weights.  instance: "surrogate_batch" (30 layers, 256 wl x 16 angles x
    s, p) or "dataset_example" (the paper's App. A.2 shape, 128 wl, s);
    thicknesses are drawn uniformly over the instance's range.  Every bound of
    `bounds` gets its own calibrated scale, accepted fractions, fallback check
    and fallback throughput (the first also at the top level of the report);
    the error estimate is the ensemble spread maximised over sigma_window
    wavelengths of each spectrum row (window_sigma), calibrated with the given
    margin and spread_factor (calibrate)."""
    import torch
    dev = "cuda"
    bounds = tuple(float(b) for b in bounds)
    report = {"config": dict(instance=instance, n_train=n_train, n_cal=n_cal, n_test=n_test, epochs=epochs,
                             batch=batch, hidden=hidden, layers=layers, members=members, bounds=list(bounds),
                             margin=margin, spread_factor=spread_factor, infer_batch=infer_batch,
                             sigma_window=sigma_window, lr_max=lr_max)}
    kw = {} if n_wl is None else {"n_wl": n_wl}
    task = make_task("f32", instance=instance, **kw)
    task64 = make_task("f64", instance=instance, **kw)
    lo, hi = INSTANCES[instance]["d_range"]
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    N = n_train + n_cal + n_test
    d = (lo + (hi - lo) * torch.rand((N, task.n_layers), generator=g, device=dev, dtype=torch.float32)).contiguous()
    in_shift, in_scale = 0.5 * (lo + hi), float(np.sqrt(12.0) / (hi - lo))  # zero mean, unit variance
    t0 = time.perf_counter()
    y = generate(task, d)
    torch.cuda.synchronize()
    report["datagen_s"] = time.perf_counter() - t0
    log(json.dumps({"stage": "data", "stacks": N, "seconds": round(report["datagen_s"], 3)}))
    xtr, ytr = d[:n_train], y[:n_train]
    xcal, ycal = d[n_train:n_train + n_cal], y[n_train:n_train + n_cal]
    xte, yte = d[n_train + n_cal:], y[n_train + n_cal:]
    sur = Surrogate(task.n_layers, task.n_out, n_hidden=hidden, n_layers=layers, n_members=members,
                    max_batch=max(batch, 4096), seed=seed + 1, in_shift=in_shift, in_scale=in_scale)
    t0 = time.perf_counter()
    hist = train(sur, xtr, ytr, epochs=epochs, batch=batch, lr_max=lr_max, lr_min=lr_min, seed=seed,
                 log_every=1, log=log)
    torch.cuda.synchronize()
    report["train_s"] = time.perf_counter() - t0
    report["loss_per_epoch"] = [h[0] for h in hist]
    steps = epochs * (n_train // batch)
    flop_step = 3 * 2 * batch * members * sum(i * o for i, o in zip(
        [128] + [hidden] * layers, [hidden] * layers + [task.n_out]))
    report["train_tflops"] = flop_step * steps / report["train_s"] / 1e12
    log(json.dumps({"stage": "train", "seconds": round(report["train_s"], 2),
                    "TFLOP/s": round(report["train_tflops"], 1)}))
    params = sur.export()
    sur.close()
    sur = Surrogate(task.n_layers, task.n_out, n_hidden=hidden, n_layers=layers, n_members=members,
                    max_batch=infer_batch, seed=seed + 1, in_shift=in_shift, in_scale=in_scale,
                    sigma_window=sigma_window)
    sur.load(params)
    # accuracy on held-out stacks
    mean, sigma, _ = sur.predict(xte)
    err = (mean - yte).abs()
    base = (ytr[:100000].mean(0, keepdim=True) - yte).abs()
    report["test_mae"] = err.mean().item()
    report["test_rmse"] = err.pow(2).mean().sqrt().item()
    report["test_max_abs"] = err.max().item()
    report["test_frac_within"] = {f"{b:g}": float((err <= b).double().mean()) for b in bounds}
    report["baseline_mean_spectrum_mae"] = base.mean().item()
    report["sigma_window"] = sigma_window
    sw = window_sigma(sigma, task, sigma_window)
    mcal, scal, _ = sur.predict(xcal)
    scal = window_sigma(scal, task, sigma_window)
    y64 = generate(task64, xte.double())
    per = {}
    for bnd in bounds:
        r = {}
        scale, r["accepted_fraction_cal"] = calibrate(mcal, scal, ycal, bnd, margin, spread_factor)
        r["err_scale"] = scale
        acc = sw * scale <= bnd
        r["accepted_fraction_test"] = float(acc.double().mean())
        r["max_abs_accepted_test"] = float(err[acc].max()) if bool(acc.any()) else None
        out, nf = sur.predict_fallback(xte, task, scale, bnd)
        r["fallback_fraction_test"] = nf / (n_test * task.n_out)
        r["max_abs_after_fallback_vs_f64"] = (out.double() - y64).abs().max().item()
        del out, acc
        per[f"{bnd:g}"] = r
        log(json.dumps({"stage": "accuracy", "bound": bnd, **r}))
    del mcal, scal, sw, mean, sigma, err, base, y64
    report["bounds"] = per
    first = per[f"{bounds[0]:g}"]
    report.update({k: first[k] for k in ("err_scale", "accepted_fraction_cal", "accepted_fraction_test",
                                        "max_abs_accepted_test", "fallback_fraction_test",
                                        "max_abs_after_fallback_vs_f64")})
    log(json.dumps({"stage": "accuracy", **{k: report[k] for k in (
        "test_mae", "test_rmse", "test_max_abs", "baseline_mean_spectrum_mae", "test_frac_within")}}))
    # throughput on one batch of eval_batch stacks
    xb = xte[:eval_batch] if n_test >= eval_batch else d[:eval_batch]
    B = xb.shape[0]
    Rf = torch.empty((B, task.n_out), dtype=torch.float32, device=dev)
    Rd = torch.empty((B, task.n_out), dtype=torch.float64, device=dev)
    x64 = xb.double().contiguous()
    t_tmm32 = _timeit(lambda: tmm.tmm_rt(xb, task.nk, task.wl, task.sin_t, task.cos_t, mat=task.mat(B),
                                         pol_mask=task.pol_mask, R=Rf.view(B, task.P, task.n_theta, task.n_wl)))
    t_tmm64 = _timeit(lambda: tmm.tmm_rt(x64, task64.nk, task64.wl, task64.sin_t, task64.cos_t,
                                         mat=task64.mat(B), pol_mask=task.pol_mask,
                                         R=Rd.view(B, task.P, task.n_theta, task.n_wl)))
    t_pred = _timeit(lambda: sur.predict(xb))
    thr = {"tmm_f32": B / t_tmm32, "tmm_f64": B / t_tmm64, "surrogate_only": B / t_pred}
    for bnd in bounds:
        r = per[f"{bnd:g}"]
        nfs = []
        t_fb = _timeit(lambda: nfs.append(sur.predict_fallback(xb, task, r["err_scale"], bnd)[1]))
        r["surrogate_fallback_stacks_per_s"] = B / t_fb
        r["fallback_fraction_eval_batch"] = nfs[-1] / (B * task.n_out)
        r["gain_vs_tmm_f32"] = t_tmm32 / t_fb
        r["gain_vs_tmm_f64"] = t_tmm64 / t_fb
    thr["surrogate_fallback"] = first["surrogate_fallback_stacks_per_s"]
    report["throughput_stacks_per_s"] = thr
    report["fallback_fraction_eval_batch"] = first["fallback_fraction_eval_batch"]
    report["gain_vs_tmm_f32"] = first["gain_vs_tmm_f32"]
    report["gain_vs_tmm_f64"] = first["gain_vs_tmm_f64"]
    log(json.dumps({"stage": "throughput", **thr, "gains": {k: (v["gain_vs_tmm_f32"], v["gain_vs_tmm_f64"])
                                                            for k, v in per.items()}}))
    sur.close()
    return report


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="train and evaluate the surrogate on tmm_rt data")
    ap.add_argument("--n-train", type=int, default=2_000_000)
    ap.add_argument("--n-cal", type=int, default=34_464)
    ap.add_argument("--n-test", type=int, default=65_536)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--hidden", type=int, default=1024)
    ap.add_argument("--layers", type=int, default=5)
    ap.add_argument("--members", type=int, default=5)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--bound", type=float, nargs="+", default=[1e-3])
    ap.add_argument("--sigma-window", type=int, default=4)
    ap.add_argument("--spread-factor", type=float, default=2.0)
    ap.add_argument("--margin", type=float, default=0.5, help="calibration margin (fraction of the bound)")
    ap.add_argument("--infer-batch", type=int, default=16384, help="internal batch of the inference handle")
    ap.add_argument("--instance", choices=sorted(INSTANCES), default="surrogate_batch")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rep = run(n_train=a.n_train, n_cal=a.n_cal, n_test=a.n_test, epochs=a.epochs, batch=a.batch, hidden=a.hidden,
              layers=a.layers, members=a.members, lr_max=a.lr, bounds=a.bound, margin=a.margin,
              infer_batch=a.infer_batch, instance=a.instance, sigma_window=a.sigma_window,
              spread_factor=a.spread_factor)
    print(json.dumps(rep), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rep, f, indent=1)
