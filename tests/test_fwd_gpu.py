"""GPU parity of the forward kernels against the CPU oracle (element by element).

Tolerances: float64 kernels agree with the complex128 oracle to 1e-12 absolute
on R and T and 1e-12 * max(1, |ref|) on r and t; float32 kernels agree to 2e-5
absolute on R and T with the oracle fed the float32-rounded inputs.
"""
import numpy as np
import pytest

import oracle
from paper_2111_13667_amd import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5


def run_gpu(w, dtype="f64", amplitudes=False, pol="both"):
    from paper_2111_13667_amd import tmm
    out = tmm.evaluate_workload(w, dtype=dtype, amplitudes=amplitudes, pol=pol)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def run_oracle(w, amplitudes=False, pol="both"):
    return oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat, pol=pol,
                     want_amplitudes=amplitudes)


def assert_close64(got, ref, keys=("R", "T")):
    for k in keys:
        g, r = got[k], ref[k]
        assert g.shape == r.shape, k
        if k in ("r", "t"):
            err = np.abs(g - r) / np.maximum(1.0, np.abs(r))
        else:
            err = np.abs(g - r)
        assert np.isfinite(g).all(), f"{k}: non-finite GPU values"
        assert err.max() <= TOL64, f"{k}: max error {err.max():.3e}"


def assert_close32(got, ref):
    for k in ("R", "T"):
        err = np.abs(got[k].astype(np.float64) - ref[k])
        assert np.isfinite(got[k]).all(), f"{k}: non-finite GPU values"
        assert err.max() <= TOL32, f"{k}: max error {err.max():.3e}"


def test_small_batch_f64_with_amplitudes():
    w = workloads.small_batch()
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_small_batch_f32():
    w = workloads.small_batch()
    assert_close32(run_gpu(w, dtype="f32"), run_oracle(w.rounded_f32()))


def test_large_batch_amplitudes_f64():
    w = workloads.large_batch().take(slice(8, 11))
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_large_batch_full_size(dtype):
    # The full 4096 x 40 x 1024 x 91 x 2 batch in the benchmark's launch
    # configuration: the first 64 stacks element by element over the whole
    # grid (1.19e7 points), and 1e5 seeded random points of the other 4032
    # stacks against the oracle evaluated at those points.
    from paper_2111_13667_amd import tmm
    w = workloads.large_batch()
    out = tmm.evaluate_workload(w, dtype=dtype)
    torch.cuda.synchronize()
    wr = w.rounded_f32() if dtype == "f32" else w
    tol = TOL64 if dtype == "f64" else TOL32
    head = {key: out[key][:64].cpu().numpy().astype(np.float64) for key in ("R", "T")}
    ref = run_oracle(wr.take(slice(0, 64)))
    for key in ("R", "T"):
        assert np.isfinite(head[key]).all(), key
        err = np.abs(head[key] - ref[key])
        assert err.max() <= tol, (key, err.max(), np.unravel_index(err.argmax(), err.shape))
    rng = np.random.default_rng(1234)
    n = 100_000
    b = rng.integers(64, w.B, n)
    p = rng.integers(0, 2, n)
    k = rng.integers(0, w.theta.size, n)
    i = rng.integers(0, w.wl.size, n)
    idx = [torch.as_tensor(x, device="cuda") for x in (b, p, k, i)]
    got = {key: out[key][tuple(idx)].cpu().numpy().astype(np.float64) for key in ("R", "T")}
    del out
    R, T = oracle.rt_points(wr.d, wr.nk, wr.wl, wr.sin_t, wr.cos_t, b, i, k, p, mat=wr.mat)
    for key, r in (("R", R), ("T", T)):
        err = np.abs(got[key] - r)
        j = int(err.argmax())
        assert err[j] <= tol, (key, err[j], b[j], p[j], k[j], i[j])


@pytest.mark.parametrize("L", [0, 1, 2, 7])
def test_few_layers_ragged_grids(L):
    # Bare interface and thin stacks; wavelength counts that leave ragged tiles.
    w = workloads.random_stacks(10 + L, B=5, L=L, n_wl=67, n_theta=3)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_single_wavelength_single_angle():
    w = workloads.random_stacks(3, B=3, L=5, n_wl=1, n_theta=1)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dispersive_per_layer_table(dtype):
    w = workloads.random_stacks(21, B=6, L=23, n_wl=130, n_theta=4, dispersive=True)
    if dtype == "f64":
        assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))
    else:
        assert_close32(run_gpu(w, dtype="f32"), run_oracle(w.rounded_f32()))


def test_appendix_example_total_internal_reflection():
    # Dense injection medium, exit into air: evanescent layers and TIR.
    w = workloads.appendix_example(B=2, n_wl=101, n_theta=91)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


@pytest.mark.parametrize("pol", ["s", "p"])
def test_single_polarisation(pol):
    w = workloads.large_batch(B=5, L=9, n_wl=70, n_theta=6)
    assert_close64(run_gpu(w, amplitudes=True, pol=pol), run_oracle(w, amplitudes=True, pol=pol),
                   ("R", "T", "r", "t"))


def test_table_path_with_mixed_ambients():
    # Stacks whose ambient differs from the first stack's take the inline source.
    w = workloads.large_batch(B=9, L=12, n_wl=64, n_theta=5)
    w.mat[3, 0] = 5
    w.mat[5, 0] = 2
    w.mat[5, -1] = 4
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_large_material_table_inline_with_ids():
    # More rows than the LDS table holds: inline source with material ids.
    rng = np.random.default_rng(5)
    w = workloads.large_batch(B=7, L=15, n_wl=90, n_theta=4)
    n_mat = 40
    nk = np.empty((n_mat, w.wl.size), np.complex128)
    nk[:] = workloads.cauchy(rng.uniform(1.3, 2.5, n_mat), rng.uniform(0, 0.03, n_mat),
                             rng.uniform(0, 0.01, n_mat), w.wl)
    nk[0] = 1.0
    mat = rng.integers(1, n_mat, w.mat.shape).astype(np.int32)
    mat[:, 0] = 0
    from dataclasses import replace
    w = replace(w, nk=nk, mat=mat)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_zero_thickness_layers():
    w = workloads.random_stacks(8, B=4, L=9, n_wl=40, n_theta=5)
    w.d[:, ::3] = 0.0
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_grazing_incidence_finite():
    w = workloads.large_batch(B=3, L=40, n_wl=64, n_theta=91)
    got = run_gpu(w, amplitudes=True)
    for k in ("R", "T", "r", "t"):
        assert np.isfinite(got[k]).all()
    np.testing.assert_allclose(got["R"][:, :, -1], 1.0, atol=1e-12)


def test_invalid_values_give_nan_not_fault():
    w = workloads.large_batch(B=4, L=6, n_wl=64, n_theta=3)
    w.d[1, 2] = -5.0
    w.d[2, 0] = np.nan
    w.mat[3, 4] = 99
    got = run_gpu(w, amplitudes=True)
    assert np.isfinite(got["R"][0]).all()
    for b in (1, 2, 3):
        assert np.isnan(got["R"][b]).all() and np.isnan(got["r"][b]).all()
    ref = run_oracle(w)
    assert np.isnan(ref["R"][1:]).all()


def _checked_call(w, dtype="f64", **mod):
    """tmm_rt with TMM_CHECK_FINITE on w (after the in-place edits in mod); returns
    the status and whether the R output was left untouched."""
    from paper_2111_13667_amd import tmm
    real = torch.float64 if dtype == "f64" else torch.float32
    cplx = torch.complex128 if dtype == "f64" else torch.complex64
    d, nk = dev(w.d, real), dev(w.nk, cplx)
    wl, s, c = dev(w.wl, real), dev(w.sin_t, real), dev(w.cos_t, real)
    mat = None if w.mat is None else dev(w.mat, torch.int32)
    R = torch.full((w.B, 2, w.theta.size, w.wl.size), 7.0, dtype=real, device="cuda")
    try:
        tmm.tmm_rt(d, nk, wl, s, c, mat=mat, R=R, flags=tmm.TMM_CHECK_FINITE)
        st = tmm.TMM_OK
    except tmm.TmmError as e:
        st = e.status
    torch.cuda.synchronize()
    return st, bool((R == 7.0).all().item()), R.cpu().numpy()


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_check_finite_flag(dtype):
    # TMM_CHECK_FINITE: valid inputs give the unchecked results; a NaN or
    # infinity gives TMM_ERR_NONFINITE, a finite out-of-range value
    # TMM_ERR_INVALID_ARG, and the output is untouched in both cases.
    from paper_2111_13667_amd import tmm
    w0 = workloads.large_batch(B=5, L=7, n_wl=70, n_theta=4)
    st, untouched, R = _checked_call(w0, dtype)
    assert st == tmm.TMM_OK and not untouched
    ref = run_gpu(w0, dtype=dtype)["R"]
    assert np.array_equal(R, ref)
    cases = [
        ("d", (3, 2), np.nan, tmm.TMM_ERR_NONFINITE),
        ("d", (0, 6), np.inf, tmm.TMM_ERR_NONFINITE),
        ("d", (4, 0), -1.0, tmm.TMM_ERR_INVALID_ARG),
        ("wl", (17,), np.nan, tmm.TMM_ERR_NONFINITE),
        ("wl", (0,), 0.0, tmm.TMM_ERR_INVALID_ARG),
        ("cos_t", (2,), -0.1, tmm.TMM_ERR_INVALID_ARG),
        ("sin_t", (1,), np.inf, tmm.TMM_ERR_NONFINITE),
        ("nk", (1, 33), complex(1.5, np.nan), tmm.TMM_ERR_NONFINITE),
        ("mat", (2, 3), 6, tmm.TMM_ERR_INVALID_ARG),
        ("mat", (1, 0), -1, tmm.TMM_ERR_INVALID_ARG),
        ("nk", (4, 10), complex(1.0, 0.01), tmm.TMM_ERR_INVALID_ARG),  # absorbing ambient row, oblique angles
    ]
    for field, idx, val, want in cases:
        from dataclasses import replace
        arr = getattr(w0, field).copy()
        arr[idx] = val
        st, untouched, _ = _checked_call(replace(w0, **{field: arr}), dtype)
        assert st == want and untouched, (field, idx, val, st)


def test_check_finite_flag_gradient():
    from paper_2111_13667_amd import tmm
    w = workloads.large_batch(B=3, L=5, n_wl=40, n_theta=2)
    args = (dev(w.d, torch.float64), dev(w.nk, torch.complex128), dev(w.wl, torch.float64),
            dev(w.sin_t, torch.float64), dev(w.cos_t, torch.float64))
    mat = dev(w.mat, torch.int32)
    gR = torch.ones((w.B, 2, w.theta.size, w.wl.size), dtype=torch.float64, device="cuda")
    gd = torch.full((w.B, w.L), 7.0, dtype=torch.float64, device="cuda")
    gd0 = torch.empty_like(gd)
    tmm.tmm_rt_grad(*args, mat=mat, dl_dR=gR, grad_d=gd0)
    tmm.tmm_rt_grad(*args, mat=mat, dl_dR=gR, grad_d=gd, flags=tmm.TMM_CHECK_FINITE)
    assert torch.equal(gd, gd0)
    gd.fill_(7.0)
    gR[1, 0, 1, 5] = float("nan")
    with pytest.raises(tmm.TmmError) as e:
        tmm.tmm_rt_grad(*args, mat=mat, dl_dR=gR, grad_d=gd, flags=tmm.TMM_CHECK_FINITE)
    assert e.value.status == tmm.TMM_ERR_NONFINITE
    torch.cuda.synchronize()
    assert (gd == 7.0).all()


def test_absorbing_ambient_only_at_normal_incidence():
    w = workloads.random_stacks(9, B=2, L=3, n_wl=20, n_theta=3, n_amb=1.2 + 0.05j)
    w.sin_t[0], w.cos_t[0] = 0.0, 1.0
    got = run_gpu(w)
    ref = run_oracle(w)
    assert np.isfinite(got["R"][:, :, 0]).all()
    assert np.isnan(got["R"][:, :, 1:]).all() and np.isnan(ref["R"][:, :, 1:]).all()
    assert np.abs(got["R"][:, :, 0] - ref["R"][:, :, 0]).max() <= TOL64


def test_empty_batch():
    from paper_2111_13667_amd import tmm
    w = workloads.small_batch(B=1)
    d = torch.zeros((0, w.L), dtype=torch.float64, device="cuda")
    R = torch.empty((0, 2, 8, 128), dtype=torch.float64, device="cuda")
    nk = torch.ones(1, dtype=torch.complex128, device="cuda")
    wl = torch.as_tensor(w.wl, device="cuda")
    s = torch.as_tensor(w.sin_t, device="cuda")
    c = torch.as_tensor(w.cos_t, device="cuda")
    tmm.tmm_rt(d, nk, wl, s, c, R=R)


def test_bitwise_deterministic():
    w = workloads.large_batch().take(slice(0, 16))
    a = run_gpu(w, amplitudes=True)
    b = run_gpu(w, amplitudes=True)
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_paper_style_call():
    from paper_2111_13667_amd import tmm
    rng = np.random.default_rng(2)
    d = rng.uniform(20, 150, 12)
    d[0] = d[-1] = np.inf
    n = rng.uniform(1.2, 5, 12)
    n[-1] = 1.0
    wl = np.linspace(500, 900, 31)
    th = np.deg2rad(np.linspace(0, 90, 17))
    out = tmm.coh_tmm("s", n, d, th, wl)
    ref = oracle.rt(d[None, 1:-1], n.astype(complex), wl, np.sin(th), np.cos(th), pol="s")
    assert np.abs(out["R"].cpu().numpy() - ref["R"][:, 0]).max() <= TOL64


def test_binding_rejects_arrays_smaller_than_the_batch():
    # The C interface cannot see device array sizes; the binding checks them
    # before any launch (here: 3 rows of material ids for 5 stacks).
    from paper_2111_13667_amd import tmm
    w = workloads.large_batch(B=5, L=4, n_wl=8, n_theta=2)
    dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    R = torch.empty((5, 2, 2, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        tmm.tmm_rt(dev(w.d, torch.float64), dev(w.nk, torch.complex128), dev(w.wl, torch.float64),
                   dev(w.sin_t, torch.float64), dev(w.cos_t, torch.float64), mat=dev(w.mat[:3], torch.int32), R=R)
    with pytest.raises(ValueError):
        tmm.tmm_rt(dev(w.d, torch.float64), dev(w.nk[:, :4], torch.complex128), dev(w.wl, torch.float64),
                   dev(w.sin_t, torch.float64), dev(w.cos_t, torch.float64), mat=dev(w.mat, torch.int32), R=R)


# --- material-table (pair) path ---------------------------------------------
# With material ids and a small table the forward kernel runs the ratio form of
# the recursion on per-pair LDS blocks (up to 6 materials in float64, 8 in
# float32); these cases cover the table sizes on both sides of those limits,
# the workgroup shapes they select, layer counts across renormalisation blocks
# and 64-layer chunks, and the fallbacks.

def _material_workload(seed, B, L, n_wl, n_theta, n_inner, *, theta_max_deg=89.0, n_amb=1.0, n_sub=1.52,
                       k_max=0.02):
    from dataclasses import replace
    rng = np.random.default_rng(seed)
    w = workloads.random_stacks(seed, B=B, L=L, n_wl=n_wl, n_theta=n_theta, theta_max_deg=theta_max_deg)
    k = np.where(rng.random(n_inner) < 0.5, 0.0, rng.uniform(0.0, k_max, n_inner))
    nk = np.empty((n_inner + 2, n_wl), np.complex128)
    nk[:n_inner] = workloads.cauchy(rng.uniform(1.3, 2.6, n_inner), rng.uniform(0.0, 0.03, n_inner), k, w.wl)
    nk[n_inner] = n_amb
    nk[n_inner + 1] = n_sub
    mat = np.empty((B, L + 2), np.int32)
    mat[:, 0] = n_inner
    mat[:, 1:L + 1] = rng.integers(0, n_inner, (B, L))
    mat[:, L + 1] = n_inner + 1
    return replace(w, nk=nk, mat=mat)


@pytest.mark.parametrize("n_inner,L", [(1, 5), (2, 33), (4, 70), (5, 40), (6, 17)])
def test_material_table_sizes_f64(n_inner, L):
    w = _material_workload(40 + n_inner, B=29, L=L, n_wl=97, n_theta=3, n_inner=n_inner)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))
    assert_close64(run_gpu(w), run_oracle(w))


@pytest.mark.parametrize("n_inner,L", [(2, 9), (6, 66), (7, 24)])
def test_material_table_sizes_f32(n_inner, L):
    w = _material_workload(50 + n_inner, B=21, L=L, n_wl=70, n_theta=2, n_inner=n_inner)
    assert_close32(run_gpu(w, dtype="f32"), run_oracle(w.rounded_f32()))


def test_many_stacks_per_workgroup_with_ragged_chunk():
    # 200 stacks: several stack chunks per (angle, wavelength tile), the last one partial
    w = _material_workload(60, B=200, L=12, n_wl=64, n_theta=2, n_inner=4)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


def test_near_critical_layer_takes_the_division_free_path():
    # Dense ambient (n = 1.5) and one air layer per stack at 4e-6 (relative)
    # from its critical angle: q of the air layer is ~2.5e-3 (real or
    # imaginary), so the pair ratios exceed their bound and those workgroups
    # evaluate their stacks with the division-free recursion (the angle 0.3
    # rad stays on the pair path).  One such layer per stack keeps the problem
    # well conditioned: k of them amplify rounding by about (1/|t|)^k.
    from dataclasses import replace
    w = _material_workload(61, B=6, L=8, n_wl=64, n_theta=3, n_inner=3, n_amb=1.5, k_max=0.0)
    nk = w.nk.copy()
    nk[0] = 1.0
    mat = w.mat.copy()
    inner = mat[:, 1:-1]
    inner[inner == 0] = 1
    inner[np.arange(w.B), np.arange(w.B) % w.L] = 0
    th_c = np.arcsin(1.0 / 1.5)
    theta = np.array([0.3, th_c * (1 + 4e-6), th_c * (1 - 4e-6)])
    s, c = workloads.angles(theta)
    w = replace(w, nk=nk, mat=mat, theta=theta, sin_t=s, cos_t=c)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))


@pytest.mark.parametrize("d_thick", [1e9, 1e16])
def test_thick_lossless_layer_conserves_energy(d_thick):
    # A 1 m layer stays on the fast phase reduction, a 1e16 nm layer takes the
    # exact one (phase beyond 2^49 / 256 half-turns).  The phase of such layers
    # is ill-conditioned (its rounding alone is ~1e-8 rad at 1 m), so the check
    # is the property that holds for any phase: R + T = 1 without absorption.
    w = _material_workload(62, B=4, L=6, n_wl=64, n_theta=3, n_inner=3, k_max=0.0)
    w.d[:, 2] = d_thick
    got = run_gpu(w)
    for k in ("R", "T"):
        assert np.isfinite(got[k]).all(), k
    assert np.abs(got["R"] + got["T"] - 1.0).max() <= 1e-12


def test_float_pair_phase_range_f32():
    # Float R and T reduce the phase d * 1024 Re q / lambda as a float pair below
    # 2^21: a 0.1 mm layer stays on it, a 1 mm layer (phase about 2^22) sends its
    # stack to the exact reduction; both against the oracle element by element,
    # and R + T = 1 (no absorption).
    w = _material_workload(63, B=6, L=8, n_wl=64, n_theta=3, n_inner=3, k_max=0.0)
    w.d[0:2, 3] = 1e5
    w.d[2:4, 5] = 1e6
    w = w.rounded_f32()
    got = run_gpu(w, dtype="f32")
    assert_close32(got, run_oracle(w))
    assert np.abs(got["R"] + got["T"] - 1.0).max() <= 2e-5


@pytest.mark.parametrize("pol", ["s", "p"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_material_table_single_polarisation_rt(pol, dtype):
    # single-polarisation pair-path variants without amplitudes
    w = _material_workload(70, B=11, L=37, n_wl=80, n_theta=3, n_inner=4)
    if dtype == "f64":
        assert_close64(run_gpu(w, pol=pol), run_oracle(w, pol=pol))
    else:
        assert_close32(run_gpu(w, dtype="f32", pol=pol), run_oracle(w.rounded_f32(), pol=pol))


@pytest.mark.parametrize("pol", ["both", "s", "p"])
def test_material_table_float_amplitudes(pol):
    # float pair path with r, t: 2e-5 * max(1, |ref|) against the oracle fed the
    # float32-rounded inputs (the same bar as R and T)
    w = _material_workload(71, B=9, L=21, n_wl=70, n_theta=3, n_inner=5)
    got = run_gpu(w, dtype="f32", amplitudes=True, pol=pol)
    ref = run_oracle(w.rounded_f32(), amplitudes=True, pol=pol)
    assert_close32(got, ref)
    for k in ("r", "t"):
        g = got[k].astype(np.complex128)
        assert np.isfinite(g).all(), k
        err = np.abs(g - ref[k]) / np.maximum(1.0, np.abs(ref[k]))
        assert err.max() <= TOL32, f"{k}: max error {err.max():.3e}"


@pytest.mark.parametrize("L,B", [(0, 1), (0, 3), (1, 1), (1, 5)])
def test_material_table_degenerate_stacks(L, B):
    # bare interface and one layer with material ids, fewer stacks than the
    # workgroup has waves, one layer material
    w = _material_workload(90 + L + B, B=B, L=L, n_wl=67, n_theta=3, n_inner=1)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))
    assert_close32(run_gpu(w, dtype="f32"), run_oracle(w.rounded_f32()))


@pytest.mark.parametrize("seed", range(24))
def test_seeded_sweep_material_ids(seed):
    # Twenty-four seeded configurations drawn at random: 1-12 inner materials (pair path
    # up to 6, table path above), 0-64 layers, 1-130 wavelengths (ragged tiles),
    # 1-5 angles, one or both polarisations, with or without r and t, both
    # precisions; four seeds use a dense ambient (n = 1.5) below every critical
    # angle of the inner media (theta <= 40 deg, n_inner >= 1.3).
    rng = np.random.default_rng(1000 + seed)
    n_inner = int(rng.integers(1, 13))
    L = int(rng.integers(0, 65))
    n_wl = int(rng.integers(1, 131))
    n_theta = int(rng.integers(1, 6))
    B = int(rng.integers(1, 40))
    pol = ["s", "p", "both"][int(rng.integers(0, 3))]
    dense = seed in (3, 7, 15, 21)
    w = _material_workload(2000 + seed, B=B, L=L, n_wl=n_wl, n_theta=n_theta, n_inner=n_inner,
                           theta_max_deg=40.0 if dense else 89.0, n_amb=1.5 if dense else 1.0)
    if seed % 2 == 0:
        amps = bool(rng.integers(0, 2))
        keys = ("R", "T", "r", "t") if amps else ("R", "T")
        assert_close64(run_gpu(w, amplitudes=amps, pol=pol), run_oracle(w, amplitudes=amps, pol=pol), keys)
    else:
        got = run_gpu(w, dtype="f32", pol=pol)
        ref = run_oracle(w.rounded_f32(), pol=pol)
        assert_close32(got, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_strongly_absorbing_metal_layers(dtype):
    # Metal-like media (n' in [0.1, 1], k in [1, 6]) between dielectrics: the
    # attenuation leaves the weak-absorption series for the full 2^y evaluation,
    # and thin metal films (5-40 nm) keep T measurable.  Material ids (pair path)
    # and per-layer indices (inline path).
    from dataclasses import replace
    rng = np.random.default_rng(77)
    B, L, n_wl, n_theta = 13, 9, 83, 4
    w = workloads.random_stacks(77, B=B, L=L, n_wl=n_wl, n_theta=n_theta, theta_max_deg=80.0)
    nk = np.empty((6, n_wl), np.complex128)
    nk[0] = workloads.cauchy(np.array([0.15]), np.array([0.0]), np.array([3.5]), w.wl)[0]
    nk[1] = workloads.cauchy(np.array([0.9]), np.array([0.0]), np.array([5.8]), w.wl)[0]
    nk[2] = workloads.cauchy(np.array([2.3]), np.array([0.02]), np.array([0.0]), w.wl)[0]
    nk[3] = workloads.cauchy(np.array([1.46]), np.array([0.004]), np.array([1.2]), w.wl)[0]
    nk[4] = 1.0
    nk[5] = 1.52
    mat = np.empty((B, L + 2), np.int32)
    mat[:, 0], mat[:, L + 1] = 4, 5
    mat[:, 1:L + 1] = rng.integers(0, 4, (B, L))
    d = np.where(mat[:, 1:L + 1] < 2, rng.uniform(5.0, 40.0, (B, L)), rng.uniform(20.0, 250.0, (B, L)))
    w = replace(w, d=d, nk=nk, mat=mat)
    for ww in (w, w.per_layer()):
        if dtype == "f64":
            assert_close64(run_gpu(ww, amplitudes=True), run_oracle(ww, amplitudes=True), ("R", "T", "r", "t"))
        else:
            assert_close32(run_gpu(ww, dtype="f32"), run_oracle(ww.rounded_f32()))


@pytest.mark.parametrize("n_sub", [1.52 + 0.05j, 0.2 + 3.5j])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_absorbing_exit_medium(dtype, n_sub):
    # Absorbing substrates (weakly lossy glass, metal-like): T_p is the flux form
    # with conj(cos) of the exit medium, the case the 50-digit admittance pin
    # covers for the oracle.  Material ids (pair path) and per-layer rows.
    w = _material_workload(130, B=7, L=12, n_wl=75, n_theta=5, n_inner=3, theta_max_deg=85.0,
                           n_sub=n_sub, k_max=0.01)
    for ww in (w, w.per_layer()):
        if dtype == "f64":
            assert_close64(run_gpu(ww, amplitudes=True), run_oracle(ww, amplitudes=True), ("R", "T", "r", "t"))
        else:
            assert_close32(run_gpu(ww, dtype="f32"), run_oracle(ww.rounded_f32()))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_long_stacks_many_renormalisation_blocks(dtype):
    # 400 layers: thirteen 32-step renormalisation blocks in double (fifty of 8
    # in float) and seven 64-layer chunks of the per-wave layer broadcast, on the
    # pair path (material ids) and the inline path (per-layer rows).
    w = _material_workload(95, B=3, L=400, n_wl=70, n_theta=3, n_inner=4, theta_max_deg=70.0, k_max=0.002)
    for ww in (w, w.per_layer()):
        if dtype == "f64":
            assert_close64(run_gpu(ww, amplitudes=True), run_oracle(ww, amplitudes=True), ("R", "T", "r", "t"))
        else:
            assert_close32(run_gpu(ww, dtype="f32"), run_oracle(ww.rounded_f32()))


@pytest.mark.parametrize("n_inner,L", [(5, 31), (10, 64), (14, 45)])
def test_row_blocks_f64(n_inner, L):
    # 7, 12 and 16 table rows (above the pair blocks' six in double): one block per
    # row with q, eta, their reciprocals and the phase coefficients, the ratios
    # formed per step; ragged wavelength tile, angles to 89 deg, r and t.
    w = _material_workload(140 + n_inner, B=23, L=L, n_wl=97, n_theta=4, n_inner=n_inner)
    assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))
    assert_close64(run_gpu(w), run_oracle(w))


@pytest.mark.parametrize("n_inner,L", [(7, 40), (14, 66)])
def test_row_blocks_f32(n_inner, L):
    # 9 and 16 rows in float (above the pair blocks' eight), with r and t
    w = _material_workload(150 + n_inner, B=19, L=L, n_wl=70, n_theta=3, n_inner=n_inner)
    assert_close32(run_gpu(w, dtype="f32"), run_oracle(w.rounded_f32()))
    assert_close32(run_gpu(w, dtype="f32", amplitudes=True), run_oracle(w.rounded_f32(), amplitudes=True))


@pytest.mark.parametrize("pol", ["s", "p"])
def test_row_blocks_single_polarisation(pol):
    # The row-block kernels for one polarisation (11 rows), R, T, r and t in
    # double, R and T in float; then 18 rows (above the row blocks' 16: the
    # per-step media path) for the same polarisation.
    w = _material_workload(170, B=13, L=26, n_wl=75, n_theta=3, n_inner=9)
    assert_close64(run_gpu(w, amplitudes=True, pol=pol), run_oracle(w, amplitudes=True, pol=pol),
                   ("R", "T", "r", "t"))
    assert_close32(run_gpu(w, dtype="f32", pol=pol), run_oracle(w.rounded_f32(), pol=pol))
    w = _material_workload(171, B=7, L=21, n_wl=40, n_theta=2, n_inner=16)
    assert_close64(run_gpu(w, amplitudes=True, pol=pol), run_oracle(w, amplitudes=True, pol=pol),
                   ("R", "T", "r", "t"))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_row_blocks_metal_rows_and_critical_fallback(dtype):
    # Ten rows: metal-like media (0.15+3.5i, 0.9+5.8i) in thin films with the
    # strong-attenuation path, under a dense ambient (n = 1.5) with one air layer
    # per stack at 4e-6 from its critical angle (q ~ 2.5e-3: the row ratios exceed
    # their bound and those workgroups take the division-free recursion), beside an
    # angle that stays on the row blocks.
    from dataclasses import replace
    rng = np.random.default_rng(160)
    w = _material_workload(160, B=8, L=10, n_wl=66, n_theta=3, n_inner=8, n_amb=1.5, k_max=0.005)
    nk = w.nk.copy()
    nk[0] = 1.0
    nk[1] = workloads.cauchy(np.array([0.15]), np.array([0.0]), np.array([3.5]), w.wl)[0]
    nk[2] = workloads.cauchy(np.array([0.9]), np.array([0.0]), np.array([5.8]), w.wl)[0]
    mat = w.mat.copy()
    inner = mat[:, 1:-1]
    inner[inner == 0] = 3
    inner[np.arange(w.B), np.arange(w.B) % w.L] = 0
    d = w.d.copy()
    metal = np.isin(inner, [1, 2])
    d[metal] = rng.uniform(5.0, 40.0, int(metal.sum()))
    th_c = np.arcsin(1.0 / 1.5)
    theta = np.array([0.3, th_c * (1 + 4e-6), th_c * (1 - 4e-6)])
    s, c = workloads.angles(theta)
    w = replace(w, nk=nk, mat=mat, d=d, theta=theta, sin_t=s, cos_t=c)
    if dtype == "f64":
        assert_close64(run_gpu(w, amplitudes=True), run_oracle(w, amplitudes=True), ("R", "T", "r", "t"))
    else:
        ww = replace(w, theta=theta[:1], sin_t=s[:1], cos_t=c[:1])  # float: away from the critical angle
        assert_close32(run_gpu(ww, dtype="f32"), run_oracle(ww.rounded_f32()))
