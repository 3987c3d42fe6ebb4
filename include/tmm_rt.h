/*
 * tmm_rt -- batched transfer-matrix evaluation of thin-film stacks on one
 * MI355X (gfx950) GPU.  Plain C interface: plain pointers and sizes only.
 *
 * The method (paper: "Physical Background of the Transfer Matrix Method"):
 * for every stack b, vacuum wavelength lambda_i, incidence angle theta_k and
 * polarisation (s, p), light enters from a semi-infinite ambient (medium 0),
 * crosses L finite layers (media 1..L, thicknesses d) and leaves into a
 * semi-infinite substrate (medium L+1).  The angle in each medium follows
 * Snell's law; each interface contributes the Fresnel coefficients of
 * Eq. (1)-(2) (non-magnetic media); each layer the phase delta = d k_z with
 * k_z = 2 pi n cos(theta) / lambda; the characteristic matrix is the product of
 * the layer matrices of Eq. (4)-(5); r and t follow from Eq. (6)-(7); R = |r|^2
 * and T is the transmitted Poynting flux over the incident one (Eq. (3)).
 * Refractive indices are n = n' + i k with k >= 0 for absorbing media.
 *
 * Conventions shared by every entry point:
 *  - Every data pointer is a DEVICE pointer (hipMalloc'ed, or a torch CUDA
 *    tensor's data_ptr) unless marked "host".  The caller owns all memory;
 *    the library keeps no pointer after a call returns.
 *  - Calls are asynchronous on the given stream (a hipStream_t passed as
 *    void*; NULL is the default stream).  Forward calls allocate nothing.
 *  - Complex arrays are interleaved (re, im) pairs of the call's real type.
 *  - Lengths (thicknesses, wavelengths) share one arbitrary unit (nm is usual).
 *  - All argument checks run on the host before any HIP call.  On a nonzero
 *    status nothing is launched and the outputs are untouched; a message is
 *    available from tmm_last_error() in the calling thread.  No exception
 *    crosses this interface.
 *  - Values that live in device memory cannot be checked on the host.  The
 *    kernels turn the following into NaN in every output of the affected
 *    stack or point, and never fault: a thickness that is negative or not
 *    finite, a material id outside [0, n_mat), an absorbing ambient
 *    (Im n_0 != 0) at oblique incidence, a non-positive wavelength.
 *  - An interface where n_j cos(theta_j) = 0 exactly (a medium whose index
 *    equals the conserved n_0 sin(theta_0)) is degenerate and yields NaN.
 */
#ifndef TMM_RT_H
#define TMM_RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tmm_status {
    TMM_OK = 0,
    TMM_ERR_INVALID_ARG = 1, /* a size, pointer or flag is out of its documented range */
    TMM_ERR_UNSUPPORTED = 2, /* a valid request the library does not handle          */
    TMM_ERR_NONFINITE = 3,   /* TMM_CHECK_FINITE found a NaN or infinity in an input   */
    TMM_ERR_HIP = 4,         /* the HIP runtime reported an error on launch            */
    TMM_ERR_WORKSPACE = 5    /* a caller-provided workspace is missing or too small    */
} tmm_status;

typedef enum tmm_dtype {
    TMM_F64 = 0, /* every real / complex buffer is double                       */
    TMM_F32 = 1  /* every real / complex buffer is float (wl, sin, cos included) */
} tmm_dtype;

enum { TMM_POL_S = 1u, TMM_POL_P = 2u, TMM_POL_BOTH = 3u };

/* Bits of tmm_rt_args.flags. */
enum {
    /* Validate the device-resident inputs before launching: one scan kernel and
     * one read-back (the call then synchronises the stream once).  A NaN or
     * infinity in d, nk, wl, sin_theta, cos_theta (or, for tmm_rt_grad, in
     * dl_dR / dl_dT) returns TMM_ERR_NONFINITE; a finite value outside its
     * range (d < 0, wl <= 0, a material id outside [0, n_mat), sin or cos of
     * the angle outside [0, 1], an absorbing ambient row when some angle is
     * oblique) returns TMM_ERR_INVALID_ARG.  Nothing is launched after a failed
     * check and the outputs are untouched.  Off by default: without it such
     * values give NaN in the affected outputs (see above).  The check keeps its
     * status word in a small static device array (no allocation). */
    TMM_CHECK_FINITE = 1u
};

/*
 * One batch of B stacks with the same number L of finite layers.
 *
 *  d          [B][L] real thicknesses (L = 0: a bare interface; d may be NULL).
 *  nk         complex refractive-index table with n_mat rows.  If dispersive,
 *             row m holds n_m(lambda_i) at element m*n_wl + i; otherwise row m
 *             is the single element m (the same index at every wavelength).
 *  mat        [B][L+2] int32 row of nk for each medium j = 0..L+1 of each stack
 *             (0 = ambient, L+1 = substrate), or NULL, meaning row b*(L+2)+j
 *             (one table row per medium of every stack).
 *  wl         [n_wl] vacuum wavelengths, > 0.
 *  sin_theta, cos_theta
 *             [n_theta] sine and cosine of the incidence angle in the ambient,
 *             0 <= theta <= pi/2.  Computed by the caller in double precision
 *             from theta and then cast, so that grazing incidence keeps
 *             cos(pi/2) = 6.1e-17 rather than a rounded-to-zero or negative value.
 *  pol_mask   TMM_POL_S, TMM_POL_P or TMM_POL_BOTH.  The output polarisation
 *             axis has P = popcount(pol_mask) entries: s first, then p.
 *  R, T       [B][P][n_theta][n_wl] real reflectance / transmittance, or NULL.
 *  r, t       [B][P][n_theta][n_wl] complex amplitude coefficients, or NULL.
 *             r is referred to the ambient side of the first interface, t to
 *             the substrate side of the last one.  The p coefficients follow
 *             the sign convention of Eq. (2), so r_p = -r_s at normal incidence.
 *             At least one of R, T, r, t must be non-NULL.
 *  flags      0 or TMM_CHECK_FINITE (any other bit: TMM_ERR_INVALID_ARG).
 */
typedef struct tmm_rt_args {
    int32_t B, L, n_wl, n_theta;
    const void *d;
    const void *nk;
    int32_t n_mat;
    int32_t dispersive;
    const int32_t *mat;
    const void *wl;
    const void *sin_theta;
    const void *cos_theta;
    uint32_t pol_mask;
    void *R, *T, *r, *t;
    uint32_t flags;
} tmm_rt_args;

/*
 * Forward evaluation: R, T (and r, t) for every (stack, wavelength, angle,
 * polarisation) point of the batch -- the paper's batched coh_tmm_fast /
 * coh_tmm_fast_disp (sections "Physical Background" and "Implementation in
 * Numpy"), Eq. (1)-(7).
 *  a       host pointer to the arguments (read during the call only).
 *  dtype   real type of every buffer (TMM_F64 or TMM_F32).
 *  stream  hipStream_t as void*, NULL = default stream.
 * Sizes: B, n_wl, n_theta >= 0 (zero: nothing to do, TMM_OK); 0 <= L <= 1<<20;
 * n_mat >= 1; the output element count B*P*n_theta*n_wl must fit in int64.
 * Returns TMM_OK or a tmm_status error (TMM_ERR_NONFINITE only with
 * TMM_CHECK_FINITE in a->flags).
 */
tmm_status tmm_rt(const tmm_rt_args *a, tmm_dtype dtype, void *stream);

/*
 * Preferred workspace bytes of tmm_rt_grad for these arguments (0 if there is
 * nothing to compute): checkpoints of the persistent grid plus partial sums for
 * all stacks, or for as many stacks as fit in 512 MiB of partial sums (the
 * batch then runs in several launches).  Depends on B, L, n_wl, n_theta only.
 */
size_t tmm_rt_grad_workspace_size(const tmm_rt_args *a);

/*
 * Smallest workspace tmm_rt_grad accepts (partial sums for four stacks per
 * launch).  Any size between this and tmm_rt_grad_workspace_size works; a
 * smaller workspace means more launches, the results are the same bits.
 */
size_t tmm_rt_grad_workspace_min_size(const tmm_rt_args *a);

/*
 * Reverse-mode gradients of a loss l(R, T) w.r.t. the layer thicknesses and
 * the layer refractive indices -- the gradients the paper obtains through
 * PyTorch autograd (section "TMM-Torch", appendix example: dl/dd of an MSE
 * against a target reflectance), computed here by a hand-written adjoint of
 * the forward recursion (Eq. (1)-(7)).  float64 only.
 *  a            the forward arguments (as for tmm_rt).  r and t must be NULL;
 *               R and T, if given, receive the forward values as a by-product.
 *  dl_dR, dl_dT [B][P][n_theta][n_wl] upstream gradients (device; either may
 *               be NULL, meaning zero; not both).
 *  grad_d       [B][L] real: dl/dd_j of every finite layer (device, or NULL).
 *  grad_n       [B][L] complex interleaved: dl/dRe n_j + i dl/dIm n_j, where
 *               n_j is shifted at every wavelength (for a constant index this
 *               is the derivative w.r.t. that index) (device, or NULL).
 *               The ambient and substrate get no gradient.
 *  workspace    device scratch of at least tmm_rt_grad_workspace_min_size(a)
 *               bytes (tmm_rt_grad_workspace_size(a) preferred), owned by the
 *               caller, contents irrelevant on entry; too small: TMM_ERR_WORKSPACE.
 *  dtype        TMM_F64 (TMM_F32 returns TMM_ERR_UNSUPPORTED).
 * The gradient outputs are overwritten.  Each gradient is a sum over the
 * (wavelength, angle) points taken in a fixed order, so repeated calls give the
 * same bits (also with a smaller workspace).  Points that are invalid
 * (see the NaN rules above) make their stack's gradients NaN.
 * With TMM_CHECK_FINITE in a->flags, dl_dR and dl_dT are checked for
 * finiteness along with the forward inputs.
 * Returns TMM_OK, TMM_ERR_INVALID_ARG, TMM_ERR_UNSUPPORTED, TMM_ERR_WORKSPACE,
 * TMM_ERR_NONFINITE or TMM_ERR_HIP.
 */
tmm_status tmm_rt_grad(const tmm_rt_args *a, const void *dl_dR, const void *dl_dT, void *grad_d,
                       void *grad_n, void *workspace, size_t workspace_bytes, tmm_dtype dtype,
                       void *stream);

/*
 * tmm_rt at an explicit list of points: R, T, r, t (for the polarisations of
 * a->pol_mask) of the listed (stack, angle, wavelength) points of the batch a
 * describes -- the same quantities as tmm_rt (Eq. (1)-(7)), for callers that
 * need only scattered points, such as a surrogate model's fallback, which
 * recomputes exactly the outputs it does not trust (paper: App. A.2, datasets
 * of reflectance spectra for machine learning).
 *  a        as for tmm_rt; a->R, a->T, a->r, a->t (any of them NULL, not all
 *           four) are laid out as tmm_rt's outputs, [B][P][n_theta][n_wl], and
 *           only the elements of the listed points are written.
 *  points   [n_points] int64 device array of flat indices
 *           (b * n_theta + k) * n_wl + i.  An index outside [0, B*n_theta*n_wl)
 *           is skipped (nothing written); a repeated index is evaluated twice.
 * Asynchronous, allocates nothing.  Returns TMM_OK or a tmm_status error
 * (TMM_CHECK_FINITE in a->flags validates the batch's inputs first).
 */
tmm_status tmm_rt_points(const tmm_rt_args *a, const int64_t *points, int64_t n_points, tmm_dtype dtype,
                         void *stream);

/*
 * tmm_rt_grad without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and errors as tmm_rt_grad (the gradients are the same bits); the
 * workspace is a static device array of tmm_rt_grad_noalloc_scratch_bytes()
 * (192 MiB) that every GPU the library runs on holds until the process ends.
 * A batch whose checkpoints of one persistent block plus the partial sums of
 * four stacks do not fit in it returns TMM_ERR_WORKSPACE; larger batches run
 * with a capped persistent grid and several launches.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (several streams or
 * threads) race and give wrong gradients -- serialise them.  Nothing in the
 * array needs clearing between calls (every value is written before it is
 * read).  The first call on a device looks up the array's address there.
 */
tmm_status tmm_rt_grad_noalloc(const tmm_rt_args *a, const void *dl_dR, const void *dl_dT, void *grad_d,
                               void *grad_n, tmm_dtype dtype, void *stream);

/* Size in bytes of tmm_rt_grad_noalloc's static scratch array. */
size_t tmm_rt_grad_noalloc_scratch_bytes(void);

/* Static description of a status code (never NULL). */
const char *tmm_status_string(tmm_status s);

/* Message describing the last error returned in the calling thread ("" if none). */
const char *tmm_last_error(void);

/* Library version as "major.minor.patch" (static string). */
const char *tmm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TMM_RT_H */
