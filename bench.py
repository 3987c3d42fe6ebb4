"""Throughput of the batched transfer-matrix forward pass on one MI355X.

One step = one tmm_rt call over the large batch: 4096 stacks x 40 layers from a
4-material Cauchy pool, 1024 wavelengths (300-1200 nm) x 91 angles (0-90 deg),
s and p, R and T written to HBM.  Inputs and outputs are resident in device
memory before the timed region starts.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--dtype f64|f32] [--no-cpu-baseline]

The record carries the roofline of the forward kernel (algorithmic FP64 flops
against the VALU peak, HBM traffic from the profiler's counters), the CPU
oracle on a bounded sample of the same batch, the other precision, the
amplitude variant, the adjoint, ragged batches, the surrogate with its
transfer-matrix fallback against plain TMM (extra records), and the paper's own
CPU timings as labelled context.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TMM points/s (stack·λ·θ·pol) at 40 layers; surrogate vs TMM at 1e-3 R error"

# Algorithmic arithmetic of the division-free layer step (complex products and
# sums of the Fresnel/phase/chain update, FMA counted as 2 flops; elementary
# functions not counted): 55 flops for s and 73 for p per layer step, i.e. 64
# per (point, interface) on average; a point of an L-layer stack crosses L+1
# interfaces.
FLOPS_PER_POINT_STEP = 64.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X vector FP64 / FP32
PEAK_HBM_GBS = 8000.0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def launch_times(fn, steps: int, warmup: int, stream=None):
    """Run fn warmup times, then steps times with a HIP event pair around every
    launch on the stream the work goes to.  Returns (per-launch ms list, wall
    seconds of the bracketed region)."""
    import torch
    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [e0.elapsed_time(e1) for e0, e1 in evs], wall


def summary(ms):
    ms = np.asarray(ms, dtype=np.float64)
    return {"median_ms": round(float(np.median(ms)), 4), "mean_ms": round(float(ms.mean()), 4),
            "min_ms": round(float(ms.min()), 4), "max_ms": round(float(ms.max()), 4), "launches": int(ms.size)}


def device_inputs(w, dtype):
    import torch
    real = torch.float64 if dtype == "f64" else torch.float32
    cplx = torch.complex128 if dtype == "f64" else torch.complex64
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    mat = None if w.mat is None else dev(w.mat, torch.int32)
    return (dev(w.d, real), dev(w.nk, cplx), dev(w.wl, real), dev(w.sin_t, real), dev(w.cos_t, real)), mat, real, cplx


def time_gpu(w, dtype: str, steps: int, warmup: int, amplitudes: bool = False):
    """tmm_rt over the whole batch (one kernel launch), outputs preallocated in
    device memory.  Returns (per-launch ms, wall s, output bytes per launch)."""
    import torch
    from paper_2111_13667_amd import tmm
    args, mat, real, cplx = device_inputs(w, dtype)
    shape = (w.B, 2, w.theta.size, w.wl.size)
    R = torch.empty(shape, dtype=real, device="cuda")
    T = torch.empty(shape, dtype=real, device="cuda")
    r = torch.empty(shape, dtype=cplx, device="cuda") if amplitudes else None
    t = torch.empty(shape, dtype=cplx, device="cuda") if amplitudes else None

    def step():
        tmm.tmm_rt(*args, mat=mat, pol_mask=3, R=R, T=T, r=r, t=t)

    ms, wall = launch_times(step, steps, warmup)  # tmm_rt launches on the current stream
    out_bytes = sum(x.numel() * x.element_size() for x in (R, T, r, t) if x is not None)
    del R, T, r, t
    torch.cuda.empty_cache()
    return ms, wall, out_bytes


def _event_time(fn, steps, warmup, stream=None):
    """Median per-launch milliseconds of fn (event pair around every launch)."""
    ms, _ = launch_times(fn, steps, warmup, stream)
    return float(np.median(ms))


# Algorithmic arithmetic of the adjoint per (point, interface): the forward step
# (64 flops, as above) plus its adjoint.  Chain adjoint per polarisation and
# layer step: two complex sums, two complex differences (8 flops), five complex
# products (30) and one complex multiply-add (8) = 46; per layer step shared by
# both polarisations: the phase-factor adjoint (8), dl/dd (4), the thickness
# term of dl/dq (4), the interface terms of dl/dq (s, 4) and dl/deta (p, 4),
# dl/dn through dq/dn and deta/dn (14) = 38.  (2 x 46 + 38) / 2 = 65 per
# (point, interface); 64 + 65 = 129.  Checkpoint recomputation is not counted.
GRAD_FLOPS_PER_POINT_STEP = 129.0


def time_grad(steps=10, L=60, n_pool=2):
    """Adjoint gradients on the 1024 x 60-layer batch (512 wl x 31 angles, s+p):
    dl/dd and dl/dn of an MSE against a long-pass target, float64.  L: the same
    batch with L layers (120 for the long-stack record); n_pool: layers cycling
    through n_pool materials (5 for the seven-row record)."""
    import torch
    from paper_2111_13667_amd import tmm, workloads
    w = workloads.adjoint_batch(L=L, n_pool=n_pool)
    (d, nk, wl, s, c), mat, _, _ = device_inputs(w, "f64")
    shape = (w.B, 2, w.theta.size, w.wl.size)
    R = torch.empty(shape, dtype=torch.float64, device="cuda")
    tmm.tmm_rt(d, nk, wl, s, c, mat=mat, R=R)
    target = torch.as_tensor(workloads.longpass_target(w.wl), dtype=torch.float64, device="cuda")
    gR = 2.0 * (R - target) / R.numel()
    gd = torch.empty((w.B, w.L), dtype=torch.float64, device="cuda")
    gn = torch.empty((w.B, w.L), dtype=torch.complex128, device="cuda")
    ws = torch.empty(tmm.grad_workspace_size(d, nk, wl, s, c, mat=mat), dtype=torch.uint8, device="cuda")
    gms, _ = launch_times(lambda: tmm.tmm_rt_grad(d, nk, wl, s, c, mat=mat, dl_dR=gR, grad_d=gd, grad_n=gn,
                                                  workspace=ws), steps, 1)
    fms, _ = launch_times(lambda: tmm.tmm_rt(d, nk, wl, s, c, mat=mat, R=R), steps, 1)
    g_med, f_med = float(np.median(gms)), float(np.median(fms))
    units = w.n_points * (w.L + 1)
    flops = units * GRAD_FLOPS_PER_POINT_STEP
    achieved = flops / (float(np.mean(gms)) * 1e-3) / 1e12
    return {"workload": f"adjoint_batch: 1024 stacks x {L} layers, {n_pool + 2} table rows, 512 wl x 31 angles, s+p, "
                        "float64",
            "points": w.n_points, "grad_ms": round(g_med, 3), "forward_ms": round(f_med, 3),
            "grad_timing": summary(gms),
            "grad_points_per_s": round(w.n_points / (g_med * 1e-3), 1), "grad_over_forward": round(g_med / f_med, 2),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f64"],
                         "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f64"], 4),
                         "algorithmic_flops_per_launch": flops,
                         "flops_per_point_interface": GRAD_FLOPS_PER_POINT_STEP},
            "workspace_MB": round(ws.numel() / 1e6, 1)}


def time_ragged(dtype="f64", steps=10, amplitudes=False):
    """Ragged batch: 8192 stacks, 2-100 layers, 256-2048 wl, 1-64 angles, s+p, R and T,
    one persistent launch (autotuned on the first run) and its HIP-graph replay."""
    import torch
    from paper_2111_13667_amd import ragged, workloads
    rw = workloads.ragged_batch()
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off)
    dev = ragged.to_device(rw, dtype)
    real = dev[3].dtype
    out = {"R": torch.empty(plan.output_size, dtype=real, device="cuda"),
           "T": torch.empty(plan.output_size, dtype=real, device="cuda")}
    if amplitudes:
        cplx = torch.complex128 if dtype == "f64" else torch.complex64
        out["r"] = torch.empty(plan.output_size, dtype=cplx, device="cuda")
        out["t"] = torch.empty(plan.output_size, dtype=cplx, device="cuda")
    t0 = time.perf_counter()
    plan.run(*dev, **out)  # tunes
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    # the amplitude kernels tune their own shape (one lane per point), which the plan does not report
    shape = None if amplitudes else plan.shape(dtype)
    rms, _ = launch_times(lambda: plan.run(*dev, **out), steps, 1)
    ms = float(np.median(rms))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan.capture(*dev, stream=st, **out)
    st.synchronize()
    gms = _event_time(lambda: plan.replay(stream=st), steps, 1, stream=st)
    layer_steps = int(((np.diff(rw.layer_off) + 1) * np.diff(rw.wl_off) * np.diff(rw.th_off)).sum()) * 2
    plan.close()
    outputs = "R,T,r,t" if amplitudes else "R,T"
    return {"workload": f"ragged_batch: 8192 stacks, 2-100 layers, 256-2048 wl, 1-64 angles, s+p, {outputs}, {dtype}",
            "points": rw.n_points, "ms": round(ms, 3), "timing": summary(rms), "graph_ms": round(gms, 3),
            "autotuned_shape": shape, "first_run_with_tuning_s": round(tune_s, 3),
            "points_per_s": round(rw.n_points / (ms * 1e-3), 1),
            "algorithmic_TFLOPs": round(layer_steps * FLOPS_PER_POINT_STEP / (ms * 1e-3) / 1e12, 2),
            "frac_of_valu_peak": round(layer_steps * FLOPS_PER_POINT_STEP / (ms * 1e-3) / 1e12
                                       / PEAK_TFLOPS[dtype], 4)}


def time_ragged_layers(dtype="f64", steps=5, layer_counts=(2, 50, 100)):
    """The ragged batch's shape (8192 stacks, 256-2048 wl, 1-64 angles, s+p) with
    every stack at one layer count, in the launch shape the full batch tunes to
    (one workgroup per CU of 12 (FP64) or 16 (FP32) waves, 4 units per claim): the
    time per unit of 64 points against the time per layer step."""
    import torch
    from paper_2111_13667_amd import ragged, workloads
    out = {"workload": f"ragged_batch shape, fixed layer counts {list(layer_counts)}, s+p, {dtype}",
           "shape": {"workgroups_per_cu": 1, "grain": 4, "waves_per_workgroup": 12 if dtype == "f64" else 16}}
    for L in layer_counts:
        rw = workloads.ragged_batch(L_range=(L, L))
        plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off)
        dev = ragged.to_device(rw, dtype)
        R = torch.empty(plan.output_size, dtype=dev[3].dtype, device="cuda")
        T = torch.empty_like(R)
        plan.set_shape(dtype, **out["shape"])
        rms, _ = launch_times(lambda: plan.run(*dev, R=R, T=T), steps, 1)
        npts = np.diff(rw.wl_off) * np.diff(rw.th_off)
        out[f"L={L}"] = {"ms": round(float(np.median(rms)), 3), "units": int(((npts + 63) // 64).sum())}
        plan.close()
    return out


# The paper's own timings (section "Core functionality speedup and dataset
# generation"): CPU only, hardware model not stated, polarisations not stated.
# Points counted as stack x wavelength x angle (one polarisation).  Other
# workloads and machines: context for the reader, not a baseline.
PAPER_CONTEXT = {
    "source": "arXiv 2111.13667, section 'Core functionality speedup and dataset generation' (CPU)",
    "tmm_fast_numpy": {"seconds": 0.168, "workload": "10 stacks x 21 layers, 100 wl (400-700 nm) x 20 angles",
                       "points_per_s": round(10 * 100 * 20 / 0.168, -2)},
    "original_tmm_per_point": {"seconds": 17.5, "workload": "same", "points_per_s": round(10 * 100 * 20 / 17.5, 0)},
    "dask_dataset": {"seconds": 2400, "workload": "1e6 stacks x 9 layers, 100 wl x 10 angles, eight-core machine",
                     "points_per_s": round(1e6 * 100 * 10 / 2400, -3)},
}


def _surrogate_record(rep):
    tp = rep["throughput_stacks_per_s"]
    per = {}
    for k, r in rep["bounds"].items():
        per[k] = {"err_scale": r["err_scale"], "accepted_fraction_cal": r["accepted_fraction_cal"],
                  "accepted_fraction_test": r["accepted_fraction_test"],
                  "max_abs_accepted_test": r["max_abs_accepted_test"],
                  "fallback_fraction_outputs": r["fallback_fraction_eval_batch"],
                  "max_abs_after_fallback_vs_f64": r["max_abs_after_fallback_vs_f64"],
                  "surrogate_fallback_stacks_per_s": round(r["surrogate_fallback_stacks_per_s"], 1),
                  "gain_vs_tmm_f32": round(r["gain_vs_tmm_f32"], 3), "gain_vs_tmm_f64": round(r["gain_vs_tmm_f64"], 3)}
    first = per[next(iter(per))]
    return {"bound": rep["config"]["bounds"][0], "calibration_margin": rep["config"]["margin"],
            "spread_factor": rep["config"]["spread_factor"], "sigma_window": rep["config"]["sigma_window"],
            "surrogate_fallback_stacks_per_s": first["surrogate_fallback_stacks_per_s"],
            "surrogate_only_stacks_per_s": round(tp["surrogate_only"], 1),
            "tmm_f32_stacks_per_s": round(tp["tmm_f32"], 1),
            "tmm_f64_stacks_per_s": round(tp["tmm_f64"], 1),
            "gain_vs_tmm_f32": first["gain_vs_tmm_f32"], "gain_vs_tmm_f64": first["gain_vs_tmm_f64"],
            "accepted_fraction_cal": first["accepted_fraction_cal"],
            "accepted_fraction_test": first["accepted_fraction_test"],
            "fallback_fraction_outputs": first["fallback_fraction_outputs"],
            "max_abs_accepted_test": first["max_abs_accepted_test"],
            "max_abs_after_fallback_vs_f64": first["max_abs_after_fallback_vs_f64"],
            "per_bound": per,
            "test_mae": round(rep["test_mae"], 6), "test_max_abs": round(rep["test_max_abs"], 6),
            "test_frac_within": rep["test_frac_within"],
            "baseline_mean_spectrum_mae": round(rep["baseline_mean_spectrum_mae"], 4),
            "train_s": round(rep["train_s"], 1), "datagen_s": round(rep["datagen_s"], 2),
            "train_tflops": round(rep["train_tflops"], 1)}


def time_surrogate():
    """Surrogate + transfer-matrix fallback against plain TMM on the 30-layer
    surrogate task (256 wavelengths x 16 angles x s,p R outputs per stack):
    2 000 000 TMM-labelled training stacks, 20 epochs, 100 000 held-out stacks
    (34 464 to fit the point-level error scale for a 1e-3 max-abs R bound, 65 536
    to test it, which are also the throughput batch)."""
    from paper_2111_13667_amd import surrogate
    rep = surrogate.run(n_train=2_000_000, n_cal=34_464, n_test=65_536, epochs=20, log=lambda *_: None)
    rec = {"workload": "surrogate_batch: 30 layers, 256 wl x 16 angles x s,p R; ensemble of 5 MLPs "
                       "30 -> 5 x 1024 GELU -> 8192, BF16 MFMA; 2000000 training stacks x 20 epochs, "
                       "100000 held-out (34464 calibration, 65536 test and throughput batch)"}
    rec.update(_surrogate_record(rep))
    return rec


def time_surrogate_dataset():
    """The same surrogate and fallback on the paper's dataset-generation shape
    (App. A.2: ten layers 2.0 / 1.4 between 2.5 and 1.0, d ~ U[5,180] nm, s-polarised
    R at normal incidence, 128 wavelengths 1000-1700 nm): 1 000 000 training
    stacks (the paper's dataset size), 100 epochs at a 3e-4 peak learning rate,
    100 000 held-out; bounds 1e-3 and 1e-2."""
    from paper_2111_13667_amd import surrogate
    rep = surrogate.run(n_train=1_000_000, n_cal=34_464, n_test=65_536, epochs=100, lr_max=3e-4,
                        bounds=(1e-3, 1e-2), instance="dataset_example", log=lambda *_: None)
    rec = {"workload": "dataset_example (App. A.2 shape): 10 layers, 128 wl x 1 angle x s R; ensemble of 5 MLPs "
                       "10 -> 5 x 1024 GELU -> 128, BF16 MFMA; 1000000 training stacks x 100 epochs, "
                       "100000 held-out (34464 calibration, 65536 test and throughput batch)"}
    rec.update(_surrogate_record(rep))
    return rec


# Arithmetic the forward pair kernel executes on the benchmark batch, from its
# instruction counters (profiles/fwd_pair_kernel_large_batch_4096x40.md: 64 lanes x
# (2 FMA + MUL + ADD) per launch): FP64 72.6 flops per lane-step, 36.3 per point and
# interface; FP32 kernel 2.1e10 float and 2.1e9 double instructions' worth.
EXECUTED_FLOPS_PER_LAUNCH = {
    "f64": {"fp64": 64 * (2 * 5.018e9 + 3.454e9 + 4.246e9)},
    "f32": {"fp32": 64 * (2 * 3.822e9 + 3.472e9 + 4.761e9), "fp64": 64 * (2 * 3.62e8 + 2.20e8 + 1.93e8)},
}


def roofline(w, dtype, kernel_ms, out_bytes, traffic=None, executed=None):
    """kernel_ms: the average launch duration of the forward kernel.  executed:
    the kernel's executed flops per launch by precision (instruction counters of
    the same kernel on the same batch), reported beside the algorithmic figure."""
    flops = w.n_points * (w.L + 1) * FLOPS_PER_POINT_STEP
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    rec = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic,
           "algorithmic_flops_per_launch": flops,
           "output_GBps": round(out_bytes / (kernel_ms * 1e-3) / 1e9, 1),
           "output_frac_of_hbm": round(out_bytes / (kernel_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    if executed:
        ex = {}
        for prec, f in executed.items():
            tf = f / (kernel_ms * 1e-3) / 1e12
            ex[prec] = {"flops_per_launch": f, "TFLOPs": round(tf, 3),
                        "frac_of_peak": round(tf / PEAK_TFLOPS["f64" if prec == "fp64" else "f32"], 4)}
        rec["executed"] = ex
        rec["executed_source"] = "instruction counters, profiles/fwd_pair_kernel_large_batch_4096x40.md"
    return rec


def time_oracle(w, runs=3, amplitudes=False):
    """The CPU oracle (complex128, OpenMP over stacks) on workload w: one
    warm-up run, then the median wall time of `runs` runs.  Returns
    (median seconds, all timed seconds, threads)."""
    import oracle
    oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, want_amplitudes=amplitudes)
    times, threads = [], 0
    for _ in range(runs):
        t0 = time.perf_counter()
        out = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, want_amplitudes=amplitudes)
        times.append(time.perf_counter() - t0)
        threads = int(out["threads"])
    return float(np.median(times)), [round(t, 4) for t in times], threads


def cpu_baseline(w, n_stacks: int):
    """The CPU oracle on the first n_stacks stacks of the same workload, all
    wavelengths, angles and polarisations (median of 3 after a warm-up)."""
    sub = w.take(slice(0, n_stacks))
    dt, times, threads = time_oracle(sub)
    pts = sub.n_points
    return {"value": round(pts / dt, 1), "unit": "points/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n_stacks} of {w.B} stacks, all {w.wl.size} wavelengths x "
                      f"{w.theta.size} angles x 2 pol ({pts} points); median of 3 runs after a warm-up "
                      f"({dt:.2f} s; runs {times})",
            "full_batch_s_extrapolated": round(dt * w.B / n_stacks, 1),
            "cpu_model": cpu_model()}


def gpu_and_oracle(w, label, steps=20, amplitudes=False, paper_s=None):
    """A small workload timed in full on both sides: tmm_rt in float64 (median
    of per-launch events) and the oracle (median of 3 after a warm-up)."""
    ms, _, _ = time_gpu(w, "f64", steps, 3, amplitudes=amplitudes)
    cpu_s, times, threads = time_oracle(w, amplitudes=amplitudes)
    g_s = float(np.median(ms)) * 1e-3
    rec = {"workload": label, "points": w.n_points, "outputs": "R,T,r,t" if amplitudes else "R,T",
           "gpu_f64": {**summary(ms), "points_per_s": round(w.n_points / g_s, 1)},
           "oracle": {"median_s": round(cpu_s, 6), "runs_s": times, "cores": threads,
                      "points_per_s": round(w.n_points / cpu_s, 1)},
           "gpu_over_oracle": round(cpu_s / g_s, 1)}
    if paper_s is not None:
        rec["paper_numpy_s"] = paper_s
        rec["note"] = ("the paper's time is its NumPy code on an unstated CPU; different hardware, "
                       "not a like-for-like comparison")
    return rec


def material_variant(n_pool, steps=5):
    """The large batch with a larger material pool (n_pool + ambient + substrate
    table rows), FP64 and FP32: the forward kernel's per-material table path."""
    from paper_2111_13667_amd import workloads
    w = workloads.large_batch(n_pool=n_pool)
    rec = {"workload": f"large_batch with a {n_pool}-material pool ({n_pool + 2} table rows)"}
    for dt in ("f64", "f32"):
        ms, _, ob = time_gpu(w, dt, steps, 1)
        rf = roofline(w, dt, float(np.mean(ms)), ob)
        rec[dt] = {**summary(ms), "points_per_s": round(w.n_points / (np.median(ms) * 1e-3), 1),
                   "frac": rf["frac"]}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other-precision, amplitude, adjoint, ragged, material-pool and surrogate records")
    ap.add_argument("--cpu-stacks", type=int, default=128,
                    help="stacks of the CPU oracle sample (median of 3 runs after a warm-up)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--only", choices=["adjoint", "adjoint_long", "adjoint_rows", "ragged_f64", "ragged_f32", "ragged_rt_f64", "ragged_rt_f32", "ragged_layers_f64", "ragged_layers_f32",
                                       "surrogate", "surrogate_dataset", "materials"],
                    default=None, help="run only this extra measurement and print its record (for profiling)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run a plain N-MiB elementwise copy kernel (profiler calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only; every point is independent and "
              "stacks would shard across GPUs with no exchange, but no multi-GPU run is "
              "provided. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.only:
        if args.only == "adjoint":
            rec = time_grad(max(1, args.steps))
        elif args.only == "adjoint_long":
            rec = time_grad(max(1, args.steps), L=120)
        elif args.only == "adjoint_rows":
            rec = time_grad(max(1, args.steps), n_pool=5)
        elif args.only == "surrogate":
            rec = time_surrogate()
        elif args.only == "surrogate_dataset":
            rec = time_surrogate_dataset()
        elif args.only.startswith("ragged_layers_"):
            rec = time_ragged_layers(args.only.split("_")[2], max(1, args.steps))
        elif args.only == "materials":
            rec = {"7": material_variant(7, max(1, args.steps)), "12": material_variant(12, max(1, args.steps))}
        elif args.only.startswith("ragged_rt_"):
            rec = time_ragged(args.only.split("_")[2], max(1, args.steps), amplitudes=True)
        else:
            rec = time_ragged(args.only.split("_")[1], max(1, args.steps))
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    from paper_2111_13667_amd import workloads
    w = workloads.large_batch()

    if args.calibrate_copy_mib > 0:
        # A plain elementwise kernel of known traffic (reads and writes N bytes),
        # for scaling the FETCH_SIZE / WRITE_SIZE counters of a profiler run.
        n = args.calibrate_copy_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y

    # HBM bytes per launch from the profiler's FETCH_SIZE + WRITE_SIZE (scaled by a
    # copy kernel), per dtype; null for a dtype that has not been measured.
    traffic_all = {}
    if os.path.exists(args.traffic_json):
        try:
            traffic_all = json.load(open(args.traffic_json))
        except (OSError, ValueError):
            traffic_all = {}
    traffic = traffic_all.get(args.dtype)

    ms, wall, out_bytes = time_gpu(w, args.dtype, args.steps, args.warmup)
    med, mean = float(np.median(ms)), float(np.mean(ms))
    value = w.n_points / (med * 1e-3)
    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med, 4),
        "timing": {**summary(ms), "wall_ms_per_step": round(wall * 1e3 / args.steps, 4),
                   "note": "value and ms_per_step use the median of the per-launch HIP-event times; "
                           "roofline.achieved uses their mean"},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "large_batch: 4096 stacks x 40 layers (4-material Cauchy pool), "
                               "1024 wavelengths 300-1200 nm x 91 angles 0-90 deg, s+p, R and T",
                   "stacks": w.B, "layers": w.L, "n_wl": int(w.wl.size), "n_theta": int(w.theta.size),
                   "points": w.n_points, "outputs": "R,T"},
        "roofline": roofline(w, args.dtype, mean, out_bytes, traffic, EXECUTED_FLOPS_PER_LAUNCH[args.dtype]),
    }
    if not args.no_extra:
        extra = {}
        other = "f32" if args.dtype == "f64" else "f64"
        oms, _, ob = time_gpu(w, other, max(10, args.steps // 2), 1)
        extra[other] = {"value": round(w.n_points / (np.median(oms) * 1e-3), 1), **summary(oms),
                        "roofline": roofline(w, other, float(np.mean(oms)), ob, traffic_all.get(other),
                                             EXECUTED_FLOPS_PER_LAUNCH[other])}
        ams, _, ob = time_gpu(w, args.dtype, max(10, args.steps // 2), 1, amplitudes=True)
        extra[args.dtype + "_with_r_t"] = {"value": round(w.n_points / (np.median(ams) * 1e-3), 1), **summary(ams),
                                           "roofline": roofline(w, args.dtype, float(np.mean(ams)), ob)}
        extra["small_batch"] = gpu_and_oracle(
            workloads.small_batch(), "small_batch: 16 stacks x 10 layers, 128 wl x 8 angles, s+p, R,T,r,t "
            "(timed in full on both sides)", amplitudes=True)
        extra["speedup_example"] = gpu_and_oracle(
            workloads.speedup_example(), "speedup_example: the paper's speed-up shape, 10 stacks x 21 media, "
            "100 wl 400-700 nm x 20 angles 0-90 deg (points counted with both polarisations)", paper_s=0.168)
        extra["adjoint_f64"] = time_grad()
        extra["adjoint_f64_120_layers"] = time_grad(L=120)
        extra["adjoint_f64_7_rows"] = time_grad(n_pool=5)
        extra["ragged_f64"] = time_ragged("f64")
        extra["ragged_f32"] = time_ragged("f32")
        extra["ragged_f64_with_r_t"] = time_ragged("f64", amplitudes=True)
        extra["material_pool_7"] = material_variant(7)
        extra["material_pool_12"] = material_variant(12)
        extra["surrogate"] = time_surrogate()
        extra["surrogate_dataset_example"] = time_surrogate_dataset()
        rec["extra"] = extra
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_stacks)
    rec["paper_context"] = PAPER_CONTEXT
    rec["gpu"] = torch.cuda.get_device_name(0)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
