"""Ragged batches (one persistent launch) against the oracle, stack by stack;
autotuning, HIP-graph replay and invalid inputs."""
import numpy as np
import pytest

import oracle
from paper_2111_13667_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(rw, dtype="f64", pol="both", lpp=None):
    from paper_2111_13667_amd import ragged
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off, pol=pol)
    if lpp is not None:
        # 2 workgroups of 6 waves per CU: fits the LDS of any table up to 8 rows
        plan.set_shape(dtype, workgroups_per_cu=2, grain=2, waves_per_workgroup=6, lanes_per_point=lpp)
    dev = ragged.to_device(rw, dtype)
    real = dev[3].dtype
    R = torch.empty(plan.output_size, dtype=real, device="cuda")
    T = torch.empty(plan.output_size, dtype=real, device="cuda")
    plan.run(*dev, R=R, T=T)
    torch.cuda.synchronize()
    return plan, dev, R, T


def check_stacks(rw, plan, R, T, stacks, dtype="f64", pol="both"):
    off = plan.output_offsets()
    Rh, Th = R.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    tol = 1e-12 if dtype == "f64" else 2e-5
    for b in stacks:
        w = rw.stack(b)
        if dtype == "f32":
            w = w.rounded_f32()
        ref = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, pol=pol, want_amplitudes=False)
        shape = ref["R"].shape[1:]
        got_R = Rh[off[b]:off[b + 1]].reshape(shape)
        got_T = Th[off[b]:off[b + 1]].reshape(shape)
        assert np.abs(got_R - ref["R"][0]).max() <= tol, (b, np.abs(got_R - ref["R"][0]).max())
        assert np.abs(got_T - ref["T"][0]).max() <= tol, b


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_small_ragged_batch_every_stack(dtype):
    rw = workloads.ragged_batch(seed=3, B=37, L_range=(0, 12), wl_range=(1, 150), th_range=(1, 5))
    plan, _, R, T = run(rw, dtype)
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("pol", ["s", "p"])
def test_single_polarisation(pol):
    rw = workloads.ragged_batch(seed=4, B=9, L_range=(1, 20), wl_range=(30, 100), th_range=(1, 4))
    plan, _, R, T = run(rw, "f64", pol)
    check_stacks(rw, plan, R, T, range(rw.B), "f64", pol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_ragged_batch_sampled_stacks(dtype):
    # 8192 stacks, 2-100 layers, 256-2048 wavelengths, 1-64 angles (6.1e8 points),
    # checked on 12 seeded random stacks plus the longest and the shortest.
    rw = workloads.ragged_batch()
    plan, _, R, T = run(rw, dtype)
    L = np.diff(rw.layer_off)
    rng = np.random.default_rng(7)
    stacks = list(rng.choice(rw.B, 12, replace=False)) + [int(L.argmax()), int(L.argmin())]
    assert np.isfinite(R.cpu().numpy()).all()
    check_stacks(rw, plan, R, T, stacks, dtype)


def test_graph_replay_matches_eager_every_time():
    rw = workloads.ragged_batch(seed=5, B=300, L_range=(2, 30), wl_range=(64, 300), th_range=(1, 8))
    from paper_2111_13667_amd import ragged
    plan, dev, R0, T0 = run(rw)
    R = torch.empty_like(R0)
    T = torch.empty_like(T0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(*dev, R=R, T=T, stream=s)
    s.synchronize()
    for rep in range(3):
        R.zero_()
        T.fill_(-1.0)
        torch.cuda.synchronize()
        plan.replay(stream=s)
        s.synchronize()
        assert torch.equal(R, R0) and torch.equal(T, T0), rep
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()


def test_second_run_reuses_tuned_shape_and_is_identical():
    rw = workloads.ragged_batch(seed=6, B=64, L_range=(5, 40), wl_range=(100, 400), th_range=(1, 6))
    plan, dev, R1, T1 = run(rw)
    R2, T2 = torch.empty_like(R1), torch.empty_like(T1)
    plan.run(*dev, R=R2, T=T2)
    torch.cuda.synchronize()
    assert torch.equal(R1, R2) and torch.equal(T1, T2)


def test_invalid_material_row_is_nan_for_that_stack_only():
    rw = workloads.ragged_batch(seed=8, B=6, L_range=(3, 6), wl_range=(10, 70), th_range=(1, 3))
    rw.mat[rw.layer_off[2]] = 17
    rw.ends[4, 1] = -1
    plan, _, R, T = run(rw)
    off = plan.output_offsets()
    Rh = R.cpu().numpy()
    for b in range(rw.B):
        seg = Rh[off[b]:off[b + 1]]
        assert np.isnan(seg).all() if b in (2, 4) else np.isfinite(seg).all(), b


@pytest.mark.parametrize("seed", range(6))
def test_seeded_sweep_ragged(seed):
    # Six seeded batches drawn at random: 5-40 stacks, layer counts up to 100,
    # 1-300 wavelengths and 1-9 angles per stack, one or both polarisations,
    # both precisions; every stack against the oracle.
    rng = np.random.default_rng(4000 + seed)
    B = int(rng.integers(5, 41))
    lo = int(rng.integers(0, 20))
    hi = lo + int(rng.integers(0, 81))
    pol = ["s", "p", "both"][int(rng.integers(0, 3))]
    dtype = ["f64", "f32"][seed % 2]
    rw = workloads.ragged_batch(seed=4100 + seed, B=B, L_range=(lo, hi), wl_range=(1, 300), th_range=(1, 9))
    plan, _, R, T = run(rw, dtype, pol)
    check_stacks(rw, plan, R, T, range(rw.B), dtype, pol)


@pytest.mark.parametrize("lpp", [1, 2, 4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lanes_per_point(lpp, dtype):
    # Every launch shape of the autotuner's space by hand: one lane per point,
    # or the stack's layers split across two or four lanes of a point (32- and
    # 16-point tiles) with the segments' 2x2 operators composed across lanes.
    # Layer counts 0-70 cover empty segments (L < lanes per point) and segments
    # longer than a renormalisation block; every stack against the oracle.
    rw = workloads.ragged_batch(seed=50 + lpp, B=23, L_range=(0, 70), wl_range=(1, 90), th_range=(1, 5))
    plan, _, R, T = run(rw, dtype, lpp=lpp)
    assert plan.shape(dtype)["lanes_per_point"] == lpp
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("pol", ["s", "p"])
def test_lanes_per_point_single_polarisation(pol):
    rw = workloads.ragged_batch(seed=60, B=11, L_range=(1, 40), wl_range=(5, 70), th_range=(1, 3))
    plan, _, R, T = run(rw, "f64", pol, lpp=4)
    check_stacks(rw, plan, R, T, range(rw.B), "f64", pol)


def test_autotuned_shape_is_reported():
    rw = workloads.ragged_batch(seed=61, B=40, L_range=(2, 30), wl_range=(64, 200), th_range=(1, 4))
    plan, _, R, T = run(rw)
    sh = plan.shape("f64")
    assert sh["lanes_per_point"] in (1, 2, 4) and sh["points_per_unit"] * sh["lanes_per_point"] == 64
    check_stacks(rw, plan, R, T, [0, rw.B - 1])


def test_first_run_of_a_plan_with_a_cached_shape_computes_its_output():
    # A second plan of the same kind (dtype, polarisation, layer and size
    # buckets) takes the tuned shape from the process-wide cache without timing
    # anything; its first run must still write the whole output.
    rw = workloads.ragged_batch(seed=62, B=40, L_range=(2, 30), wl_range=(64, 200), th_range=(1, 4))
    run(rw)                                   # tunes and caches the shape
    plan, _, R, T = run(rw)                   # new plan, cached shape
    check_stacks(rw, plan, R, T, range(rw.B))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scaled_lengths_take_the_exact_phase_reduction(dtype):
    # Only d / lambda matters.  Thicknesses and wavelengths scaled by 1e-6 leave
    # every phase as it was, but the phase coefficient per unit thickness
    # (1024 Re q / lambda) exceeds 2^20, so every unit reduces its phases
    # modulo a full turn before the table lookup; every stack against the oracle.
    import dataclasses
    rw = workloads.ragged_batch(seed=70, B=21, L_range=(0, 80), wl_range=(1, 120), th_range=(1, 6))
    rw = dataclasses.replace(rw, d=rw.d * 1e-6, wl=rw.wl * 1e-6)
    plan, _, R, T = run(rw, dtype)
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ambient_and_substrate_rows_as_layer_materials(dtype):
    # Layers made of the ambient's or the substrate's table row (rows 4, 5):
    # the unit builds exactly the rows its stack uses.
    rw = workloads.ragged_batch(seed=71, B=17, L_range=(1, 70), wl_range=(20, 150), th_range=(1, 5))
    rng = np.random.default_rng(71)
    pick = rng.random(rw.mat.size) < 0.3
    rw.mat[pick] = rng.integers(4, 6, int(pick.sum())).astype(np.int32)
    plan, _, R, T = run(rw, dtype)
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_metal_rows_and_grazing_angles(dtype):
    # Strongly absorbing rows (metal-like 0.2+3.5i and 1.5+5.8i in place of
    # materials 1 and 3), 5-40 nm films and angles up to 89.9 deg, where eta
    # grows to hundreds and the units fall back to the shorter renormalisation
    # period; every stack against the oracle.
    import dataclasses
    rw = workloads.ragged_batch(seed=72, B=15, L_range=(1, 60), wl_range=(10, 120), th_range=(2, 7))
    rng = np.random.default_rng(72)
    nk = rw.nk.copy()
    nk[1] = 0.2 + 3.5j
    nk[3] = 1.5 + 5.8j
    d = rw.d.copy()
    metal = np.isin(rw.mat, [1, 3])
    d[metal] = rng.uniform(5.0, 40.0, int(metal.sum()))
    theta = np.concatenate([np.deg2rad(np.linspace(0.0, 89.9, n)) for n in np.diff(rw.th_off)])
    s, c = workloads.angles(theta)
    rw = dataclasses.replace(rw, nk=nk, d=d, theta=theta, sin_t=s, cos_t=c)
    plan, _, R, T = run(rw, dtype)
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("grain", [1, 3, 16])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_eight_rows_and_claim_batches_across_stacks(dtype, grain):
    # The most rows a unit's table holds (8: two more rows, one of them
    # absorbing), stacks of one to four units so that a claimed batch of units
    # spans several stacks and the wave's kept stack record changes within the
    # batch, empty stacks, and layer counts to 90 (top 64-layer chunks that
    # start above layer 1); every stack against the oracle.
    import dataclasses
    from paper_2111_13667_amd import ragged
    rw = workloads.ragged_batch(seed=73, B=45, L_range=(0, 90), wl_range=(1, 120), th_range=(1, 3))
    rng = np.random.default_rng(73)
    extra = np.stack([np.full(rw.wl.size, 1.8 + 0.0j), np.full(rw.wl.size, 2.1 + 0.02j)])
    mat = rw.mat.copy()
    pick = rng.random(mat.size) < 0.3
    mat[pick] = rng.integers(6, 8, int(pick.sum())).astype(np.int32)
    rw = dataclasses.replace(rw, nk=np.concatenate([rw.nk, extra]), mat=mat)
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off)
    plan.set_shape(dtype, workgroups_per_cu=1, grain=grain, waves_per_workgroup=8)
    dev = ragged.to_device(rw, dtype)
    R = torch.empty(plan.output_size, dtype=dev[3].dtype, device="cuda")
    T = torch.empty_like(R)
    plan.run(*dev, R=R, T=T)
    torch.cuda.synchronize()
    check_stacks(rw, plan, R, T, range(rw.B), dtype)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_one_row_table_and_empty_stacks(dtype):
    # A one-row table (ambient, every layer and the substrate the same medium):
    # R = 0 and T = 1 at every point, against the oracle too; then a batch in
    # which every stack is empty (L = 0: the bare interface).
    import dataclasses
    rw = workloads.ragged_batch(seed=74, B=12, L_range=(0, 70), wl_range=(1, 90), th_range=(1, 4))
    one = dataclasses.replace(rw, nk=rw.nk[5:6].copy(), mat=np.zeros_like(rw.mat),
                              ends=np.zeros_like(rw.ends))
    plan, _, R, T = run(one, dtype)
    check_stacks(one, plan, R, T, range(one.B), dtype)
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert np.abs(R.cpu().numpy()).max() <= tol
    assert np.abs(T.cpu().numpy() - 1.0).max() <= tol
    empty = workloads.ragged_batch(seed=75, B=20, L_range=(0, 0), wl_range=(1, 130), th_range=(1, 5))
    plan, _, R, T = run(empty, dtype)
    check_stacks(empty, plan, R, T, range(empty.B), dtype)


# --- r and t (the amplitude kernels: one lane per point, their own shape) ---

def run_amp(rw, dtype="f64", pol="both", outputs=("R", "T", "r", "t")):
    from paper_2111_13667_amd import ragged
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off, pol=pol)
    dev = ragged.to_device(rw, dtype)
    real = dev[3].dtype
    cplx = torch.complex128 if real == torch.float64 else torch.complex64
    out = {k: torch.full((plan.output_size,), float("nan"), dtype=real if k in ("R", "T") else cplx, device="cuda")
           for k in outputs}
    plan.run(*dev, **out)
    torch.cuda.synchronize()
    return plan, dev, out


def check_amplitudes(rw, plan, out, stacks, dtype="f64", pol="both"):
    # tmm_rt's bounds: R, T absolute; r, t relative to max(1, |ref|)
    off = plan.output_offsets()
    host = {k: v.cpu().numpy() for k, v in out.items()}
    tol = 1e-12 if dtype == "f64" else 2e-5
    for b in stacks:
        w = rw.stack(b)
        if dtype == "f32":
            w = w.rounded_f32()
        ref = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, pol=pol, want_amplitudes=True)
        for k, v in host.items():
            want = ref[k][0]
            got = v[off[b]:off[b + 1]].reshape(want.shape).astype(want.dtype)
            err = np.abs(got - want)
            bound = tol * (np.maximum(1.0, np.abs(want)) if k in ("r", "t") else 1.0)
            assert (err <= bound).all(), (k, b, float(err.max()))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_amplitudes_every_stack(dtype):
    # R, T, r, t in one run: empty stacks, stacks of one and of two 64-layer
    # chunks, absorbing and lossless rows; every stack against the oracle.
    rw = workloads.ragged_batch(seed=80, B=31, L_range=(0, 100), wl_range=(1, 140), th_range=(1, 5))
    plan, _, out = run_amp(rw, dtype)
    check_amplitudes(rw, plan, out, range(rw.B), dtype)


@pytest.mark.parametrize("pol", ["s", "p"])
def test_amplitudes_single_polarisation(pol):
    rw = workloads.ragged_batch(seed=81, B=13, L_range=(0, 40), wl_range=(10, 90), th_range=(1, 4))
    plan, _, out = run_amp(rw, "f64", pol)
    check_amplitudes(rw, plan, out, range(rw.B), "f64", pol)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_amplitudes_exact_phase_reduction_and_metals(dtype):
    # Thicknesses and wavelengths scaled by 1e-6 (every unit reduces its phases
    # exactly before the table lookup: t's phase sum must keep two turns), then
    # metal-like rows at angles up to 89.9 deg; every stack against the oracle.
    import dataclasses
    rw = workloads.ragged_batch(seed=82, B=17, L_range=(0, 80), wl_range=(1, 100), th_range=(1, 5))
    scaled = dataclasses.replace(rw, d=rw.d * 1e-6, wl=rw.wl * 1e-6)
    plan, _, out = run_amp(scaled, dtype)
    check_amplitudes(scaled, plan, out, range(scaled.B), dtype)
    rng = np.random.default_rng(83)
    nk = rw.nk.copy()
    nk[1] = 0.2 + 3.5j
    nk[3] = 1.5 + 5.8j
    d = rw.d.copy()
    metal = np.isin(rw.mat, [1, 3])
    d[metal] = rng.uniform(5.0, 40.0, int(metal.sum()))
    theta = np.concatenate([np.deg2rad(np.linspace(0.0, 89.9, n)) for n in np.diff(rw.th_off)])
    s, c = workloads.angles(theta)
    metals = dataclasses.replace(rw, nk=nk, d=d, theta=theta, sin_t=s, cos_t=c)
    plan, _, out = run_amp(metals, dtype)
    check_amplitudes(metals, plan, out, range(metals.B), dtype)


def test_amplitude_outputs_alone_and_rt_runs_unchanged():
    # r alone, then t alone (the other outputs untouched); an R, T run of the
    # same plan afterwards keeps its own tuned shape and its bits.
    rw = workloads.ragged_batch(seed=84, B=19, L_range=(1, 70), wl_range=(20, 150), th_range=(1, 4))
    plan, dev, R0, T0 = run(rw)
    shape0 = plan.shape("f64")
    for k in ("r", "t"):
        x = torch.full((plan.output_size,), complex(7.0, 7.0), dtype=torch.complex128, device="cuda")
        plan.run(*dev, **{k: x})
        torch.cuda.synchronize()
        check_amplitudes(rw, plan, {k: x}, range(rw.B))
    R1, T1 = torch.empty_like(R0), torch.empty_like(T0)
    plan.run(*dev, R=R1, T=T1)
    torch.cuda.synchronize()
    assert plan.shape("f64") == shape0
    assert torch.equal(R0, R1) and torch.equal(T0, T1)


def test_amplitude_graph_replay_matches_eager():
    rw = workloads.ragged_batch(seed=85, B=60, L_range=(2, 70), wl_range=(32, 200), th_range=(1, 6))
    plan, dev, out0 = run_amp(rw)
    out = {k: torch.empty_like(v) for k, v in out0.items()}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(*dev, stream=s, **out)
    s.synchronize()
    for rep in range(3):
        for v in out.values():
            v.fill_(-1.0)
        torch.cuda.synchronize()
        plan.replay(stream=s)
        s.synchronize()
        for k in out:
            assert torch.equal(out[k], out0[k]), (k, rep)
        x = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
    check_amplitudes(rw, plan, out, [0, rw.B // 2, rw.B - 1])


def test_fixed_rt_shape_leaves_amplitude_runs_their_own():
    # A plan whose R, T shape is fixed at four lanes per point: an amplitude run
    # of the same plan still takes the one-lane-per-point kernels (its own
    # tuned shape), and the R, T shape stays as set.
    from paper_2111_13667_amd import ragged
    rw = workloads.ragged_batch(seed=86, B=14, L_range=(0, 50), wl_range=(8, 90), th_range=(1, 4))
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off)
    plan.set_shape("f64", workgroups_per_cu=2, grain=2, waves_per_workgroup=6, lanes_per_point=4)
    dev = ragged.to_device(rw, "f64")
    out = {k: torch.empty(plan.output_size, dtype=torch.float64 if k in ("R", "T") else torch.complex128,
                          device="cuda") for k in ("R", "r", "t")}
    plan.run(*dev, **out)
    torch.cuda.synchronize()
    check_amplitudes(rw, plan, out, range(rw.B))
    assert plan.shape("f64")["lanes_per_point"] == 4


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_amplitudes_full_ragged_batch_sampled_stacks(dtype):
    # The 8192-stack batch with R, T, r, t in the tuned amplitude shape (the
    # bench's launch); ten seeded stacks plus the longest and the shortest
    # against the oracle, copying only their slices to the host.
    from paper_2111_13667_amd import ragged
    rw = workloads.ragged_batch()
    plan = ragged.RaggedPlan(rw.layer_off, rw.wl_off, rw.th_off)
    dev = ragged.to_device(rw, dtype)
    real = dev[3].dtype
    cplx = torch.complex128 if real == torch.float64 else torch.complex64
    out = {k: torch.empty(plan.output_size, dtype=real if k in ("R", "T") else cplx, device="cuda")
           for k in ("R", "T", "r", "t")}
    plan.run(*dev, **out)
    torch.cuda.synchronize()
    off = plan.output_offsets()
    L = np.diff(rw.layer_off)
    stacks = list(np.random.default_rng(87).choice(rw.B, 10, replace=False)) + [int(L.argmax()), int(L.argmin())]
    tol = 1e-12 if dtype == "f64" else 2e-5
    for b in stacks:
        w = rw.stack(b)
        if dtype == "f32":
            w = w.rounded_f32()
        ref = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, want_amplitudes=True)
        for k, v in out.items():
            want = ref[k][0]
            got = v[int(off[b]):int(off[b + 1])].cpu().numpy().reshape(want.shape).astype(want.dtype)
            bound = tol * (np.maximum(1.0, np.abs(want)) if k in ("r", "t") else 1.0)
            assert (np.abs(got - want) <= bound).all(), (k, b, float(np.abs(got - want).max()))
    del out
    plan.close()
