/*
 * Plain complex128 CPU oracle for the batched transfer-matrix method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (libtmm_rt, the HIP kernels and their Python binding) never calls it and
 * shares no code, header, helper or constant with it.
 *
 * What it computes (paper: "Physical Background of the Transfer Matrix Method"):
 *   - Snell's law with the complex refraction angle for every medium,
 *   - the Fresnel coefficients r, t of every interface, Eq. (1)-(2), with mu_r = 1,
 *   - the layer phase delta_l = d_l k_z, the layer matrices M_l, Eq. (4),
 *   - the characteristic matrix M~ as an explicit left-to-right product of 2x2
 *     complex matrices, Eq. (5),
 *   - r = M~10 / M~00 and t = 1 / M~00, Eq. (6)-(7),
 *   - R and T from Eq. (3) read as |r|^2 and the Poynting-flux ratio.
 * The arithmetic is the literal definition: one point at a time, the full 2x2
 * matrix-matrix product, no blocking, fusion or reordering.
 *
 * Readings of passages where the paper is silent or garbled (each also listed
 * in the design notes):
 *   - mu_r = 1 everywhere (non-magnetic media).
 *   - n = n' + i k with k >= 0 absorbing; k_z = 2 pi n_l cos(theta_l) / lambda.
 *   - M~ = M_0 M_1 ... M_L over the L+1 interfaces of L finite layers, with no
 *     phase in the ambient (delta_0 = 0): the paper's product bound counts the
 *     two semi-infinite media as layers.
 *   - Forward branch of n_j cos(theta_j): if |Im q| > 100 * 2^-52 the decaying
 *     root (Im q > 0), else the root with Re q > 0.
 *   - T_s = |t|^2 Re(n_out cos_out) / Re(n_in cos_in),
 *     T_p = |t|^2 Re(n_out conj(cos_out)) / Re(n_in conj(cos_in)).
 *   - Im(delta) is capped at 35 so that exp(-i delta) cannot overflow for opaque
 *     layers (the dropped relative term is below e^-70).
 *   - Invalid points produce NaN in every output: an absorbing ambient at
 *     oblique incidence, a negative or non-finite thickness, a material id
 *     outside the table.
 *
 * Parity pins (tests/test_oracle_pins.py): single-interface Brewster / TIR /
 * normal-incidence values, the Airy single-layer formula, the quarter-wave
 * stack closed form, R + T = 1, zero-thickness and split-layer invariance,
 * reciprocity of T, the half-wave absentee layer, the inner-branch flip,
 * normal-incidence s/p relations, passivity, and a 50-digit evaluation of the
 * independent Abeles characteristic-matrix formulation, whose exit media
 * include lossless glass, an evanescent exit (air behind a dense ambient
 * beyond the critical angle) and absorbing exits (lossy glass, a metal-like
 * medium): there T = 4 eta_0 Re(eta_sub) / |eta_0 B + C|^2 with the tilted
 * admittances fixes the flux form of T_s and T_p, conj(cos) included.
 *
 * oracle_rt_dir_cs (bottom of this file) repeats the same steps in bicomplex
 * arithmetic to give complex-step directional derivatives of R and T; it is
 * pinned against central finite differences of oracle_rt
 * (tests/test_oracle_grad_pins.py).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORACLE_BRANCH_EPS (100.0 * 2.220446049250313e-16)
#define ORACLE_IM_DELTA_CAP 35.0
#define ORACLE_PI 3.14159265358979323846

/* Refractive index of medium j of stack b at wavelength i.  Layout shared with
 * the public interface: row m of the table holds n_m(lambda_i) at
 * nk[m * n_wl + i] when dispersive, else the single value nk[m]. */
static int material_row(int b, int j, int L, const int32_t *mat) {
    return mat ? mat[(int64_t)b * (L + 2) + j] : b * (L + 2) + j;
}

static cplx nk_at(const double *nk, int dispersive, int n_wl, int row, int i) {
    int64_t k = dispersive ? (int64_t)row * n_wl + i : row;
    return nk[2 * k] + I * nk[2 * k + 1];
}

/* Forward wave criterion for q = n cos(theta) (the branch reading above). */
static int is_forward(cplx q) {
    if (fabs(cimag(q)) > ORACLE_BRANCH_EPS) return cimag(q) > 0.0;
    return creal(q) > 0.0;
}

/* 2x2 complex matrix product C = A B (row-major a00 a01 a10 a11). */
static void mat2_mul(const cplx A[4], const cplx B[4], cplx C[4]) {
    cplx c00 = A[0] * B[0] + A[1] * B[2];
    cplx c01 = A[0] * B[1] + A[1] * B[3];
    cplx c10 = A[2] * B[0] + A[3] * B[2];
    cplx c11 = A[2] * B[1] + A[3] * B[3];
    C[0] = c00; C[1] = c01; C[2] = c10; C[3] = c11;
}

/*
 * One (stack, wavelength, angle, polarisation) point.
 *   n[0..L+1]   refractive indices, d[0..L-1] finite-layer thicknesses,
 *   lam         vacuum wavelength (same unit as d),
 *   sin_t/cos_t sine and cosine of the incidence angle in the ambient,
 *   pol         0 = s, 1 = p,
 *   flip        optional [L+2] mask: 1 forces the other root of q_j for an
 *               inner layer (used only by the branch-invariance pin).
 * Returns 0, or -1 for an invalid point (outputs then NaN).
 */
static int oracle_point(int L, const cplx *n, const double *d, double lam,
                        double sin_t, double cos_t, int pol, const uint8_t *flip,
                        cplx *cos_buf, cplx *r_out, cplx *t_out,
                        double *R_out, double *T_out) {
    const double nan = NAN;
    if (cimag(n[0]) != 0.0 && sin_t != 0.0) goto invalid;
    if (!(lam > 0.0) || !isfinite(lam)) goto invalid;
    for (int j = 0; j < L; ++j)
        if (!(d[j] >= 0.0) || !isfinite(d[j])) goto invalid;

    /* Snell's law: n_0 sin(theta_0) = n_j sin(theta_j) (Physical Background,
     * the law of refraction).  cos(theta_0) is the given value. */
    {
        cplx kx = n[0] * sin_t;
        cos_buf[0] = cos_t;
        for (int j = 1; j <= L + 1; ++j) {
            cplx s = kx / n[j];
            cplx c = csqrt(1.0 - s * s);
            if (!is_forward(n[j] * c)) c = -c;
            if (flip && flip[j] && j <= L) c = -c;
            cos_buf[j] = c;
        }
    }

    /* Characteristic matrix M~ = M_0 M_1 ... M_L, Eq. (4)-(5). */
    cplx Mt[4] = {1.0, 0.0, 0.0, 1.0};
    for (int j = 0; j <= L; ++j) {
        cplx n1 = n[j], n2 = n[j + 1];
        cplx c1 = cos_buf[j], c2 = cos_buf[j + 1];
        cplx r, t;
        if (pol == 0) { /* Eq. (1) */
            cplx den = n1 * c1 + n2 * c2;
            t = 2.0 * n1 * c1 / den;
            r = (n1 * c1 - n2 * c2) / den;
        } else { /* Eq. (2) */
            cplx den = n2 * c1 + n1 * c2;
            t = 2.0 * n1 * c1 / den;
            r = (n2 * c1 - n1 * c2) / den;
        }
        cplx delta = 0.0;
        if (j > 0) { /* delta_l = d_l k_z with k_z = 2 pi n_l cos(theta_l) / lambda */
            delta = 2.0 * ORACLE_PI * n1 * d[j - 1] * c1 / lam;
            if (cimag(delta) > ORACLE_IM_DELTA_CAP)
                delta = creal(delta) + I * ORACLE_IM_DELTA_CAP;
        }
        cplx em = cexp(-I * delta), ep = cexp(I * delta);
        cplx Mj[4] = {em / t, em * r / t, ep * r / t, ep / t};
        mat2_mul(Mt, Mj, Mt);
    }

    /* Eq. (6)-(7): (1, r)^T = M~ (t, 0)^T. */
    cplx r = Mt[2] / Mt[0];
    cplx t = 1.0 / Mt[0];
    double R = creal(r) * creal(r) + cimag(r) * cimag(r);
    double tt = creal(t) * creal(t) + cimag(t) * cimag(t);
    double T;
    /* Eq. (3), Poynting-flux reading. */
    if (pol == 0)
        T = tt * creal(n[L + 1] * cos_buf[L + 1]) / creal(n[0] * cos_buf[0]);
    else
        T = tt * creal(n[L + 1] * conj(cos_buf[L + 1])) / creal(n[0] * conj(cos_buf[0]));
    *r_out = r; *t_out = t; *R_out = R; *T_out = T;
    return 0;

invalid:
    *r_out = nan + I * nan; *t_out = nan + I * nan; *R_out = nan; *T_out = nan;
    return -1;
}

/*
 * Batched evaluation over B stacks x n_wl wavelengths x n_theta angles and the
 * polarisations in pol_mask (bit 0 = s, bit 1 = p).  All pointers are host
 * pointers; complex arrays are interleaved (re, im) doubles.
 *   d      [B][L]                 thicknesses
 *   nk     [n_mat][n_wl] or [n_mat] refractive-index table (see nk_at)
 *   mat    [B][L+2] row ids or NULL (row = b*(L+2)+j)
 *   wl     [n_wl]; sin_t, cos_t [n_theta]
 *   R, T   [B][P][n_theta][n_wl] (either may be NULL)
 *   r, t   [B][P][n_theta][n_wl] complex (either may be NULL)
 *   flip   optional [L+2] inner-branch flip mask (NULL in normal use)
 * Returns the number of OpenMP threads used, or -1 on a bad argument.
 */
int oracle_rt(int B, int L, int n_wl, int n_theta,
              const double *d, const double *nk, int n_mat, int dispersive,
              const int32_t *mat, const double *wl,
              const double *sin_t, const double *cos_t, unsigned pol_mask,
              double *R, double *T, double *r, double *t, const uint8_t *flip) {
    if (B < 0 || L < 0 || n_wl < 0 || n_theta < 0 || (pol_mask & ~3u) || !pol_mask)
        return -1;
    int P = (pol_mask & 1u) + ((pol_mask >> 1) & 1u);
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
        cplx *nbuf = (cplx *)malloc(sizeof(cplx) * (size_t)(L + 2));
        cplx *cbuf = (cplx *)malloc(sizeof(cplx) * (size_t)(L + 2));
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < B; ++b) {
            int bad_row = 0;
            for (int j = 0; j < L + 2; ++j) {
                int row = material_row(b, j, L, mat);
                if (row < 0 || row >= n_mat) bad_row = 1;
            }
            for (int i = 0; i < n_wl; ++i) {
                for (int j = 0; j < L + 2 && !bad_row; ++j)
                    nbuf[j] = nk_at(nk, dispersive, n_wl, material_row(b, j, L, mat), i);
                for (int k = 0; k < n_theta; ++k) {
                    int pi = 0;
                    for (int pol = 0; pol < 2; ++pol) {
                        if (!(pol_mask & (1u << pol))) continue;
                        cplx rr, tt;
                        double RR, TT;
                        if (bad_row) {
                            rr = NAN + I * NAN; tt = rr; RR = NAN; TT = NAN;
                        } else {
                            oracle_point(L, nbuf, d + (int64_t)b * L, wl[i], sin_t[k],
                                         cos_t[k], pol, flip, cbuf, &rr, &tt, &RR, &TT);
                        }
                        int64_t o = (((int64_t)b * P + pi) * n_theta + k) * n_wl + i;
                        if (R) R[o] = RR;
                        if (T) T[o] = TT;
                        if (r) { r[2 * o] = creal(rr); r[2 * o + 1] = cimag(rr); }
                        if (t) { t[2 * o] = creal(tt); t[2 * o + 1] = cimag(tt); }
                        ++pi;
                    }
                }
            }
        }
        free(nbuf);
        free(cbuf);
    }
    return threads;
}

/*
 * The same point definition at an explicit list of n_pts points (sampled
 * checks of large batches): point m is stack b[m], wavelength index i[m],
 * angle index k[m], polarisation pol[m] (0 = s, 1 = p), with the grids and
 * tables laid out as for oracle_rt.  R, T [n_pts] (either may be NULL).
 * Returns the number of OpenMP threads used, or -1 on a bad argument.
 */
int oracle_rt_points(int B, int L, int n_wl, int n_theta,
                     const double *d, const double *nk, int n_mat, int dispersive,
                     const int32_t *mat, const double *wl,
                     const double *sin_t, const double *cos_t, int64_t n_pts,
                     const int32_t *pb, const int32_t *pi_wl, const int32_t *pk, const int32_t *ppol,
                     double *R, double *T) {
    if (B < 0 || L < 0 || n_wl < 0 || n_theta < 0 || n_pts < 0) return -1;
    for (int64_t m = 0; m < n_pts; ++m)
        if (pb[m] < 0 || pb[m] >= B || pi_wl[m] < 0 || pi_wl[m] >= n_wl || pk[m] < 0 ||
            pk[m] >= n_theta || ppol[m] < 0 || ppol[m] > 1)
            return -1;
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
        cplx *nbuf = (cplx *)malloc(sizeof(cplx) * (size_t)(L + 2));
        cplx *cbuf = (cplx *)malloc(sizeof(cplx) * (size_t)(L + 2));
#pragma omp for schedule(dynamic, 64)
        for (int64_t m = 0; m < n_pts; ++m) {
            const int b = pb[m], i = pi_wl[m], k = pk[m];
            int bad_row = 0;
            for (int j = 0; j < L + 2; ++j) {
                int row = material_row(b, j, L, mat);
                if (row < 0 || row >= n_mat) bad_row = 1;
                else nbuf[j] = nk_at(nk, dispersive, n_wl, row, i);
            }
            cplx rr, tt;
            double RR = NAN, TT = NAN;
            if (!bad_row)
                oracle_point(L, nbuf, d + (int64_t)b * L, wl[i], sin_t[k], cos_t[k], ppol[m],
                             NULL, cbuf, &rr, &tt, &RR, &TT);
            if (R) R[m] = RR;
            if (T) T[m] = TT;
        }
        free(nbuf);
        free(cbuf);
    }
    return threads;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ===========================================================================
 * Complex-step derivative oracle (bicomplex arithmetic).
 *
 * The same steps as oracle_point, carried out on bicomplex numbers
 * z = z1 + z2 j (z1, z2 complex in i, j^2 = -1, i j = j i).  A real parameter p
 * of the stack is replaced by p + h v j with h = 1e-20; every output quantity
 * then has a j-part equal to h times its derivative along v, free of
 * cancellation (complex-step differentiation in its multicomplex form).  R and
 * T are formed from the i-real and i-imaginary parts treated as j-complex
 * numbers, so their j-parts are h dR/de and h dT/de.
 * Used to check the adjoint kernel's gradients (TMM-Torch section: gradients
 * of R, T w.r.t. thicknesses and refractive indices).
 * =========================================================================== */

typedef struct { cplx a, b; } bicplx; /* a + b j */

static bicplx bc(cplx a, cplx b) { bicplx r = {a, b}; return r; }
static bicplx bc_add(bicplx x, bicplx y) { return bc(x.a + y.a, x.b + y.b); }
static bicplx bc_sub(bicplx x, bicplx y) { return bc(x.a - y.a, x.b - y.b); }
static bicplx bc_mul(bicplx x, bicplx y) {
    return bc(x.a * y.a - x.b * y.b, x.a * y.b + x.b * y.a);
}
static bicplx bc_scale(cplx s, bicplx x) { return bc(s * x.a, s * x.b); }
static bicplx bc_div(bicplx x, bicplx y) {
    /* x / y = x * (y.a - y.b j) / (y.a^2 + y.b^2) */
    cplx den = y.a * y.a + y.b * y.b;
    bicplx c = bc(y.a, -y.b);
    bicplx n = bc_mul(x, c);
    return bc(n.a / den, n.b / den);
}
/* sqrt with the same principal branch on the value part; w1^2 - w2^2 = z1,
 * 2 w1 w2 = z2.  The j-part is O(h), so w1 = sqrt(z1 + w2^2) = sqrt(z1) to
 * double precision. */
static bicplx bc_sqrt(bicplx z) {
    cplx w1 = csqrt(z.a);
    cplx w2 = z.b / (2.0 * w1);
    return bc(w1, w2);
}
/* exp(z1 + z2 j) = exp(z1) (cos z2 + j sin z2) */
static bicplx bc_exp(bicplx z) {
    cplx e = cexp(z.a);
    return bc(e * ccos(z.b), e * csin(z.b));
}

/* One point in bicomplex arithmetic; n[j], d[j] already carry their j-parts.
 * Outputs R, T as j-complex numbers (value, j-part). */
static int oracle_point_bc(int L, const bicplx *n, const bicplx *d, double lam,
                           double sin_t, double cos_t, int pol, bicplx *cos_buf,
                           double R_out[2], double T_out[2]) {
    if (cimag(n[0].a) != 0.0 && sin_t != 0.0) return -1;
    bicplx kx = bc_scale(sin_t, n[0]);
    cos_buf[0] = bc(cos_t, 0.0);
    for (int j = 1; j <= L + 1; ++j) {
        bicplx s = bc_div(kx, n[j]);
        bicplx c = bc_sqrt(bc_sub(bc(1.0, 0.0), bc_mul(s, s)));
        if (!is_forward(n[j].a * c.a)) c = bc_scale(-1.0, c);
        cos_buf[j] = c;
    }
    bicplx M[4] = {bc(1.0, 0.0), bc(0.0, 0.0), bc(0.0, 0.0), bc(1.0, 0.0)};
    for (int j = 0; j <= L; ++j) {
        bicplx n1 = n[j], n2 = n[j + 1], c1 = cos_buf[j], c2 = cos_buf[j + 1];
        bicplx r, t, den;
        if (pol == 0) {
            den = bc_add(bc_mul(n1, c1), bc_mul(n2, c2));
            t = bc_div(bc_scale(2.0, bc_mul(n1, c1)), den);
            r = bc_div(bc_sub(bc_mul(n1, c1), bc_mul(n2, c2)), den);
        } else {
            den = bc_add(bc_mul(n2, c1), bc_mul(n1, c2));
            t = bc_div(bc_scale(2.0, bc_mul(n1, c1)), den);
            r = bc_div(bc_sub(bc_mul(n2, c1), bc_mul(n1, c2)), den);
        }
        bicplx delta = bc(0.0, 0.0);
        if (j > 0) {
            delta = bc_scale(2.0 * ORACLE_PI / lam, bc_mul(bc_mul(n1, d[j - 1]), c1));
            if (cimag(delta.a) > ORACLE_IM_DELTA_CAP) return -1;
        }
        bicplx em = bc_exp(bc_scale(-I, delta)), ep = bc_exp(bc_scale(I, delta));
        bicplx it = bc_div(bc(1.0, 0.0), t);
        bicplx Mj[4] = {bc_mul(em, it), bc_mul(bc_mul(em, r), it), bc_mul(bc_mul(ep, r), it),
                        bc_mul(ep, it)};
        bicplx C[4];
        C[0] = bc_add(bc_mul(M[0], Mj[0]), bc_mul(M[1], Mj[2]));
        C[1] = bc_add(bc_mul(M[0], Mj[1]), bc_mul(M[1], Mj[3]));
        C[2] = bc_add(bc_mul(M[2], Mj[0]), bc_mul(M[3], Mj[2]));
        C[3] = bc_add(bc_mul(M[2], Mj[1]), bc_mul(M[3], Mj[3]));
        for (int q = 0; q < 4; ++q) M[q] = C[q];
    }
    bicplx r = bc_div(M[2], M[0]);
    bicplx t = bc_div(bc(1.0, 0.0), M[0]);
    /* i-real / i-imaginary parts as j-complex numbers (value, j-part), squared. */
    double rr0 = creal(r.a), rr1 = creal(r.b), ri0 = cimag(r.a), ri1 = cimag(r.b);
    double tr0 = creal(t.a), tr1 = creal(t.b), ti0 = cimag(t.a), ti1 = cimag(t.b);
    double R0 = rr0 * rr0 + ri0 * ri0, R1 = 2.0 * (rr0 * rr1 + ri0 * ri1);
    double tt0 = tr0 * tr0 + ti0 * ti0, tt1 = 2.0 * (tr0 * tr1 + ti0 * ti1);
    /* flux ratio f = Re(num) / Re(den), each a j-complex number */
    bicplx num, den;
    if (pol == 0) {
        num = bc_mul(n[L + 1], cos_buf[L + 1]);
        den = bc_mul(n[0], cos_buf[0]);
    } else {
        bicplx cc = bc(conj(cos_buf[L + 1].a), conj(cos_buf[L + 1].b));
        bicplx c0 = bc(conj(cos_buf[0].a), conj(cos_buf[0].b));
        num = bc_mul(n[L + 1], cc);
        den = bc_mul(n[0], c0);
    }
    double nu0 = creal(num.a), nu1 = creal(num.b), de0 = creal(den.a), de1 = creal(den.b);
    double f0 = nu0 / de0, f1 = (nu1 * de0 - nu0 * de1) / (de0 * de0);
    R_out[0] = R0; R_out[1] = R1;
    T_out[0] = tt0 * f0; T_out[1] = tt1 * f0 + tt0 * f1;
    return 0;
}

/*
 * Directional derivative of a weighted sum of outputs, per stack:
 *   D[b] = sum over (pol, theta, lambda) of gR * dR/de + gT * dT/de
 * for the perturbation d_j -> d_j + e vd[b][j], n_j -> n_j + e vn[b][j] of the
 * finite layers j = 1..L (vn complex; n_j shifted at every wavelength).
 * Per-layer index table only (row b*(L+2)+j), as in oracle_rt with mat = NULL.
 *   gR, gT  [B][P][n_theta][n_wl] weights (either may be NULL = 0)
 *   vd      [B][L] real, vn [B][L] complex interleaved (either may be NULL = 0)
 * Returns the number of threads used, or -1 on a bad argument.
 */
int oracle_rt_dir_cs(int B, int L, int n_wl, int n_theta, const double *d, const double *nk,
                     int dispersive, const double *wl, const double *sin_t,
                     const double *cos_t, unsigned pol_mask, const double *gR,
                     const double *gT, const double *vd, const double *vn, double *D) {
    if (B < 0 || L < 0 || n_wl < 0 || n_theta < 0 || (pol_mask & ~3u) || !pol_mask) return -1;
    const double h = 1e-20;
    int P = (pol_mask & 1u) + ((pol_mask >> 1) & 1u);
    int threads = 1;
#pragma omp parallel
    {
#ifdef _OPENMP
#pragma omp single
        threads = omp_get_num_threads();
#endif
        bicplx *nb = (bicplx *)malloc(sizeof(bicplx) * (size_t)(L + 2));
        bicplx *db = (bicplx *)malloc(sizeof(bicplx) * (size_t)(L + 1));
        bicplx *cb = (bicplx *)malloc(sizeof(bicplx) * (size_t)(L + 2));
#pragma omp for schedule(dynamic, 1)
        for (int b = 0; b < B; ++b) {
            double acc = 0.0;
            for (int j = 0; j < L; ++j)
                db[j] = bc(d[(int64_t)b * L + j], vd ? h * vd[(int64_t)b * L + j] : 0.0);
            for (int i = 0; i < n_wl; ++i) {
                for (int j = 0; j < L + 2; ++j) {
                    cplx v = nk_at(nk, dispersive, n_wl, b * (L + 2) + j, i);
                    cplx dv = 0.0;
                    if (vn && j >= 1 && j <= L) {
                        int64_t q = (int64_t)b * L + (j - 1);
                        dv = h * (vn[2 * q] + I * vn[2 * q + 1]);
                    }
                    nb[j] = bc(v, dv);
                }
                for (int k = 0; k < n_theta; ++k) {
                    int pi = 0;
                    for (int pol = 0; pol < 2; ++pol) {
                        if (!(pol_mask & (1u << pol))) continue;
                        double R[2], T[2];
                        int64_t o = (((int64_t)b * P + pi) * n_theta + k) * n_wl + i;
                        if (oracle_point_bc(L, nb, db, wl[i], sin_t[k], cos_t[k], pol, cb, R, T) == 0) {
                            if (gR) acc += gR[o] * R[1] / h;
                            if (gT) acc += gT[o] * T[1] / h;
                        } else {
                            acc = NAN;
                        }
                        ++pi;
                    }
                }
            }
            D[b] = acc;
        }
        free(nb);
        free(db);
        free(cb);
    }
    return threads;
}
