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
 * independent Abeles characteristic-matrix formulation.
 * Parity unpinned: T_p when the exit medium is absorbing or evanescent (only
 * the passivity inequality applies there).
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

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
