"""Seeded synthetic workloads shaped like the paper's random thin-film stacks.

This module only draws inputs: thicknesses, refractive-index tables (including
the Cauchy material model n(lambda) = A + B / lambda^2 that defines the
dispersive materials), material ids and the wavelength / angle grids.  It holds
none of the transfer-matrix arithmetic, so both the HIP path and the CPU oracle
consume its output.  Every array is drawn in float64 from
``numpy.random.default_rng(seed)`` in a fixed order.  Lengths are in nm; Cauchy
B coefficients are in um^2.

The paper measures on random stacks it draws itself (speed-up section: random
21-layer films; appendix examples: uniform thicknesses and indices), and names no
public dataset; these generators stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Optional

import numpy as np


@dataclass
class Workload:
    """One batch: B stacks of L finite layers over n_wl wavelengths x n_theta angles.

    d      [B, L] float64 thicknesses (nm)
    nk     complex128 index table, [n_mat, n_wl] if ``dispersive`` else [n_mat]
    mat    [B, L+2] int32 row ids into ``nk`` (media 0 and L+1 are the ambient and
           the substrate) or None, meaning row = b*(L+2)+j
    wl     [n_wl] vacuum wavelengths (nm)
    theta  [n_theta] incidence angles in the ambient (rad)
    sin_t, cos_t  [n_theta] float64 sine / cosine of ``theta``
    """
    name: str
    d: np.ndarray
    nk: np.ndarray
    mat: Optional[np.ndarray]
    wl: np.ndarray
    theta: np.ndarray
    sin_t: np.ndarray
    cos_t: np.ndarray

    @property
    def B(self) -> int:
        return self.d.shape[0]

    @property
    def L(self) -> int:
        return self.d.shape[1]

    @property
    def dispersive(self) -> bool:
        return self.nk.ndim == 2

    @property
    def n_points(self) -> int:
        return self.B * self.wl.size * self.theta.size * 2

    def take(self, stacks) -> "Workload":
        """Subset of stacks (index array or slice); per-layer tables are re-packed."""
        idx = np.arange(self.B)[stacks]
        d = self.d[idx]
        if self.mat is not None:
            return replace(self, d=d, mat=np.ascontiguousarray(self.mat[idx]))
        L2 = self.L + 2
        rows = (idx[:, None] * L2 + np.arange(L2)[None, :]).ravel()
        return replace(self, d=d, nk=np.ascontiguousarray(self.nk[rows]))

    def per_layer(self) -> "Workload":
        """Same stacks with one index-table row per medium (row b*(L+2)+j, mat None)."""
        if self.mat is None:
            return self
        nk = np.ascontiguousarray(self.nk[self.mat.ravel()])
        return replace(self, nk=nk, mat=None)

    def rounded_f32(self) -> "Workload":
        """Every real input rounded to float32 and widened back to float64.

        The oracle is fed these when it checks the float32 kernels, so that the
        rounding of the inputs is not charged to the kernel."""
        f = lambda a: a.astype(np.float32).astype(np.float64)
        nk = (self.nk.real.astype(np.float32).astype(np.float64)
              + 1j * self.nk.imag.astype(np.float32).astype(np.float64))
        return replace(self, d=f(self.d), nk=nk, wl=f(self.wl),
                       sin_t=f(self.sin_t), cos_t=f(self.cos_t))


def angles(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    return np.sin(theta), np.cos(theta)


def cauchy(A, Bc, k, wl_nm):
    """n_m(lambda) = A_m + B_m / lambda^2 + i k_m with lambda in um; [n_mat, n_wl]."""
    lam_um = np.asarray(wl_nm, dtype=np.float64) / 1000.0
    A = np.asarray(A, dtype=np.float64)[:, None]
    Bc = np.asarray(Bc, dtype=np.float64)[:, None]
    k = np.asarray(k, dtype=np.float64)[:, None]
    return (A + Bc / lam_um[None, :] ** 2) + 1j * k * np.ones_like(lam_um)[None, :]


def _per_layer_table(n_inner: np.ndarray, n_amb: complex, n_sub: complex) -> np.ndarray:
    """Per-layer constant indices packed as rows b*(L+2)+j, j = 0..L+1."""
    B, L = n_inner.shape
    tab = np.empty((B, L + 2), dtype=np.complex128)
    tab[:, 0] = n_amb
    tab[:, 1:L + 1] = n_inner
    tab[:, L + 1] = n_sub
    return tab.ravel()


def small_batch(seed: int = 0, B: int = 16, L: int = 10, n_wl: int = 128,
                n_theta: int = 8) -> Workload:
    """Small complex128 batch: 16 stacks x 10 layers, d ~ U[10,300] nm,
    n ~ U[1.3,2.5] + i U[0,0.01] per layer (constant in lambda), ambient 1.0,
    substrate 1.52, 128 wavelengths 400-900 nm, 8 angles 0-60 deg."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(10.0, 300.0, (B, L))
    nr = rng.uniform(1.3, 2.5, (B, L))
    k = rng.uniform(0.0, 0.01, (B, L))
    nk = _per_layer_table(nr + 1j * k, 1.0, 1.52)
    wl = np.linspace(400.0, 900.0, n_wl)
    theta = np.deg2rad(np.linspace(0.0, 60.0, n_theta))
    s, c = angles(theta)
    return Workload("small_batch_16x10", d, nk, None, wl, theta, s, c)


def large_batch(seed: int = 0, B: int = 4096, L: int = 40, n_wl: int = 1024,
                n_theta: int = 91, n_pool: int = 4) -> Workload:
    """Large batch: 4096 stacks x 40 layers from a 4-material Cauchy pool
    (A ~ U[1.4,2.4], B ~ U[0.003,0.03] um^2, k = 0, 1e-3, 0, 1e-3), d ~ U[20,250] nm,
    1024 wavelengths 300-1200 nm, 91 angles 0-90 deg in 1 deg steps (grazing
    incidence included), ambient 1.0, substrate 1.52.  Table rows 0..n_pool-1 are
    the pool, row n_pool the ambient, row n_pool+1 the substrate.  n_pool other
    than 4 draws a larger (or smaller) pool the same way, k alternating 0 / 1e-3
    (the material-count variants of the benchmark)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(1.4, 2.4, n_pool)
    Bc = rng.uniform(0.003, 0.03, n_pool)
    k = np.where(np.arange(n_pool) % 2 == 1, 1e-3, 0.0)
    mat_inner = rng.integers(0, n_pool, (B, L))
    d = rng.uniform(20.0, 250.0, (B, L))
    wl = np.linspace(300.0, 1200.0, n_wl)
    nk = np.empty((n_pool + 2, n_wl), dtype=np.complex128)
    nk[:n_pool] = cauchy(A, Bc, k, wl)
    nk[n_pool] = 1.0
    nk[n_pool + 1] = 1.52
    mat = np.empty((B, L + 2), dtype=np.int32)
    mat[:, 0] = n_pool
    mat[:, 1:L + 1] = mat_inner
    mat[:, L + 1] = n_pool + 1
    theta = np.deg2rad(np.arange(0, n_theta, dtype=np.float64))
    s, c = angles(theta)
    name = "large_batch_4096x40" if n_pool == 4 else f"large_batch_4096x40_{n_pool}mat"
    return Workload(name, d, nk, mat, wl, theta, s, c)


def adjoint_batch(seed: int = 0, B: int = 1024, L: int = 60, n_wl: int = 512,
                  n_theta: int = 31, n_pool: int = 2) -> Workload:
    """Gradient workload: 1024 stacks x 60 alternating high/low layers (high first,
    n_H = 2.35, n_L = 1.46, k = 0), d ~ U[30,200] nm, 512 wavelengths 400-800 nm x
    31 angles 0-60 deg, ambient 1.0, substrate 1.52.  Table rows: 0 high, 1 low,
    2 ambient, 3 substrate.  n_pool > 2: the layers cycle through a pool of
    n_pool lossless indices (2.35, 1.46, then 2.0, 1.7, 2.2, 1.6, ...), rows
    n_pool and n_pool + 1 the ambient and the substrate (the thicknesses are the
    same draws)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(30.0, 200.0, (B, L))
    pool = [2.35, 1.46, 2.0, 1.7, 2.2, 1.6, 1.9, 2.5, 1.55, 2.1][:n_pool]
    if len(pool) < n_pool:
        raise ValueError("n_pool <= 10")
    nk = np.array(pool + [1.0, 1.52], dtype=np.complex128)
    mat = np.empty((B, L + 2), dtype=np.int32)
    mat[:, 0] = n_pool
    mat[:, 1:L + 1] = np.arange(L) % n_pool
    mat[:, L + 1] = n_pool + 1
    wl = np.linspace(400.0, 800.0, n_wl)
    theta = np.deg2rad(np.linspace(0.0, 60.0, n_theta))
    s, c = angles(theta)
    return Workload("adjoint_batch_1024x60", d, nk, mat, wl, theta, s, c)


def longpass_target(wl: np.ndarray, edge_nm: float = 600.0) -> np.ndarray:
    """Target reflectance of the gradient workload: 1 below the edge, 0 above."""
    return (np.asarray(wl) < edge_nm).astype(np.float64)


def surrogate_batch(seed: int = 0, B: int = 65536, L: int = 30, n_wl: int = 256,
                    n_theta: int = 16) -> Workload:
    """Surrogate workload: B stacks of 30 layers, d ~ U[20,250] nm, fixed
    alternating Cauchy materials (high first: A = 2.3, B = 0.02 um^2; low:
    A = 1.45, B = 0.004 um^2; lossless), 256 wavelengths 400-900 nm x 16 angles
    0-60 deg, ambient 1.0, substrate 1.52.  Table rows: 0 high, 1 low,
    2 ambient, 3 substrate."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(20.0, 250.0, (B, L))
    wl = np.linspace(400.0, 900.0, n_wl)
    nk = np.empty((4, n_wl), dtype=np.complex128)
    nk[:2] = cauchy([2.3, 1.45], [0.02, 0.004], [0.0, 0.0], wl)
    nk[2] = 1.0
    nk[3] = 1.52
    mat = np.empty((B, L + 2), dtype=np.int32)
    mat[:, 0] = 2
    mat[:, 1:L + 1] = np.arange(L) % 2
    mat[:, L + 1] = 3
    theta = np.deg2rad(np.linspace(0.0, 60.0, n_theta))
    s, c = angles(theta)
    return Workload("surrogate_batch_30", d, nk, mat, wl, theta, s, c)


def dataset_example(seed: int = 0, B: int = 65536, n_wl: int = 128) -> Workload:
    """Shape of the paper's dataset-generation example (App. A.2): ten finite
    layers alternating n = 2.0 / 1.4 between an injection medium n = 2.5 and an
    exit medium n = 1.0, d ~ U[5,180] nm, wavelengths 1000-1700 nm at normal
    incidence (the paper's example takes s-polarised R at 100 wavelengths;
    128 here, the surrogate's output tile).  Table rows: 0 high, 1 low,
    2 injection, 3 exit."""
    rng = np.random.default_rng(seed)
    L = 10
    d = rng.uniform(5.0, 180.0, (B, L))
    wl = np.linspace(1000.0, 1700.0, n_wl)
    nk = np.array([2.0, 1.4, 2.5, 1.0], dtype=np.complex128)
    mat = np.empty((B, L + 2), dtype=np.int32)
    mat[:, 0] = 2
    mat[:, 1:L + 1] = np.arange(L) % 2
    mat[:, L + 1] = 3
    theta = np.zeros(1)
    s, c = angles(theta)
    return Workload("dataset_example_10", d, nk, mat, wl, theta, s, c)


@dataclass
class RaggedWorkload:
    """Stacks with their own layer counts and grids, packed flat (CSR style).

    Stack b: finite layers layer_off[b]..layer_off[b+1]-1 of d and mat,
    wavelengths wl_off[b]..wl_off[b+1]-1 of wl, angles th_off[b]..th_off[b+1]-1
    of theta / sin_t / cos_t; ends[b] = (ambient row, substrate row); nk
    [n_mat, wl_off[B]] holds every material at every stack's wavelengths.
    """
    name: str
    layer_off: np.ndarray
    wl_off: np.ndarray
    th_off: np.ndarray
    d: np.ndarray
    mat: np.ndarray
    ends: np.ndarray
    wl: np.ndarray
    theta: np.ndarray
    sin_t: np.ndarray
    cos_t: np.ndarray
    nk: np.ndarray

    @property
    def B(self) -> int:
        return len(self.layer_off) - 1

    @property
    def n_points(self) -> int:
        nw = np.diff(self.wl_off)
        nt = np.diff(self.th_off)
        return int(2 * (nw * nt).sum())

    def stack(self, b: int) -> Workload:
        """Stack b as a dense one-stack workload (for the oracle)."""
        l0, l1 = self.layer_off[b], self.layer_off[b + 1]
        w0, w1 = self.wl_off[b], self.wl_off[b + 1]
        t0, t1 = self.th_off[b], self.th_off[b + 1]
        L = int(l1 - l0)
        mat = np.empty((1, L + 2), dtype=np.int32)
        mat[0, 0] = self.ends[b, 0]
        mat[0, 1:L + 1] = self.mat[l0:l1]
        mat[0, L + 1] = self.ends[b, 1]
        return Workload(f"{self.name}[{b}]", self.d[None, l0:l1].copy(), np.ascontiguousarray(self.nk[:, w0:w1]),
                        mat, self.wl[w0:w1].copy(), self.theta[t0:t1].copy(), self.sin_t[t0:t1].copy(),
                        self.cos_t[t0:t1].copy())


def ragged_batch(seed: int = 0, B: int = 8192, L_range=(2, 100), wl_range=(256, 2048), th_range=(1, 64),
                 wl_span=(350.0, 1100.0), th_max_deg=80.0) -> RaggedWorkload:
    """Ragged batch: layer counts ~ integers in L_range (inclusive), per-stack
    wavelength counts in wl_range over linspace(350, 1100 nm) and angle counts in
    th_range over linspace(0, 80 deg) (one angle means normal incidence); the
    4-material Cauchy pool of large_batch (rows 0-3) plus ambient 1.0 (row 4) and
    substrate 1.52 (row 5); d ~ U[20,250] nm; material ids uniform over the pool.
    Draw order: layer counts, wavelength counts, angle counts, A, B, thicknesses,
    material ids."""
    rng = np.random.default_rng(seed)
    Ls = rng.integers(L_range[0], L_range[1] + 1, B)
    nws = rng.integers(wl_range[0], wl_range[1] + 1, B)
    nts = rng.integers(th_range[0], th_range[1] + 1, B)
    A = rng.uniform(1.4, 2.4, 4)
    Bc = rng.uniform(0.003, 0.03, 4)
    k = np.array([0.0, 1e-3, 0.0, 1e-3])
    layer_off = np.concatenate([[0], np.cumsum(Ls)]).astype(np.int64)
    wl_off = np.concatenate([[0], np.cumsum(nws)]).astype(np.int64)
    th_off = np.concatenate([[0], np.cumsum(nts)]).astype(np.int64)
    d = rng.uniform(20.0, 250.0, int(layer_off[-1]))
    mat = rng.integers(0, 4, int(layer_off[-1])).astype(np.int32)
    wl = np.concatenate([np.linspace(wl_span[0], wl_span[1], n) for n in nws])
    theta = np.concatenate([np.deg2rad(np.linspace(0.0, th_max_deg, n)) if n > 1 else np.zeros(1) for n in nts])
    s, c = angles(theta)
    nk = np.empty((6, wl.size), dtype=np.complex128)
    nk[:4] = cauchy(A, Bc, k, wl)
    nk[4] = 1.0
    nk[5] = 1.52
    ends = np.tile(np.array([[4, 5]], dtype=np.int32), (B, 1))
    return RaggedWorkload(f"ragged_batch_{B}", layer_off, wl_off, th_off, d, mat, ends, wl, theta, s, c, nk)


def appendix_example(seed: int = 0, B: int = 1, n_media: int = 12, n_wl: int = 301,
                     n_theta: int = 301) -> Workload:
    """Shape of the paper's appendix TMM-Fast example: 12 media including the two
    semi-infinite ones, d ~ U[20,150] nm, n ~ U[1.2,5] constant (the first draw is
    the injection medium), exit medium n = 1, 301 wavelengths 500-900 nm and 301
    angles 0-90 deg.  Light goes from a dense into a thin medium, so total
    internal reflection and evanescent layers occur."""
    rng = np.random.default_rng(seed)
    L = n_media - 2
    d = rng.uniform(20.0, 150.0, (B, L))
    n = rng.uniform(1.2, 5.0, (B, n_media))
    n[:, -1] = 1.0
    nk = n.astype(np.complex128).ravel()
    wl = np.linspace(500.0, 900.0, n_wl)
    theta = np.deg2rad(np.linspace(0.0, 90.0, n_theta))
    s, c = angles(theta)
    return Workload("appendix_example_12media", d, nk, None, wl, theta, s, c)


def speedup_example(seed: int = 0, B: int = 10, n_media: int = 21, n_wl: int = 100,
                    n_theta: int = 20) -> Workload:
    """Shape of the paper's speed-up timing (section "Core functionality speedup
    and dataset generation"): ten stacks of 21 media (read as 19 finite layers
    plus the two semi-infinite ones, as the paper's listings count them), 100
    wavelengths 400-700 nm x 20 angles 0-90 deg.  The paper states no indices or
    thicknesses for it; the appendix example's recipe stands in: d ~ U[20,150]
    nm, constant n ~ U[1.2,5] (the first draw is the injection medium), exit
    medium n = 1."""
    rng = np.random.default_rng(seed)
    L = n_media - 2
    d = rng.uniform(20.0, 150.0, (B, L))
    n = rng.uniform(1.2, 5.0, (B, n_media))
    n[:, -1] = 1.0
    nk = n.astype(np.complex128).ravel()
    wl = np.linspace(400.0, 700.0, n_wl)
    theta = np.deg2rad(np.linspace(0.0, 90.0, n_theta))
    s, c = angles(theta)
    return Workload("speedup_example_10x21", d, nk, None, wl, theta, s, c)


def random_stacks(seed: int, B: int, L: int, n_wl: int, n_theta: int, *,
                  dispersive: bool = False, lossy: bool = True, theta_max_deg=89.0,
                  n_amb: float = 1.0, n_sub: complex = 1.52) -> Workload:
    """Generic random per-layer stacks for parity edge cases (ragged tails, L = 0,
    L = 1, dispersive per-layer tables)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(5.0, 300.0, (B, L))
    wl = np.sort(rng.uniform(350.0, 1100.0, n_wl))
    theta = np.sort(rng.uniform(0.0, np.deg2rad(theta_max_deg), n_theta))
    s, c = angles(theta)
    if dispersive:
        A = rng.uniform(1.3, 2.6, (B, L))
        Bc = rng.uniform(0.0, 0.03, (B, L))
        k = rng.uniform(0.0, 0.02, (B, L)) if lossy else np.zeros((B, L))
        lam = wl / 1000.0
        inner = A[..., None] + Bc[..., None] / lam ** 2 + 1j * k[..., None]
        tab = np.empty((B, L + 2, n_wl), dtype=np.complex128)
        tab[:, 0, :] = n_amb
        tab[:, 1:L + 1, :] = inner
        tab[:, L + 1, :] = n_sub
        nk = tab.reshape(B * (L + 2), n_wl)
    else:
        nr = rng.uniform(1.3, 2.6, (B, L))
        k = rng.uniform(0.0, 0.02, (B, L)) if lossy else np.zeros((B, L))
        nk = _per_layer_table(nr + 1j * k, n_amb, n_sub)
    return Workload(f"random_{B}x{L}", d, nk, None, wl, theta, s, c)
