/*
 * tmm_surrogate -- learned surrogate of the transfer-matrix method with a
 * transfer-matrix fallback, on one MI355X (gfx950).  Plain C interface.
 *
 * The paper's fast TMM exists to make machine learning on thin-film data
 * practical (sections "Core functionality speedup and dataset generation" and
 * App. A.2, which generates a dataset of reflectance spectra of random
 * stacks).  This interface trains such a model on data produced by tmm_rt and
 * uses it in place of tmm_rt where its ensemble agrees to within a bound:
 *
 *   an ensemble of E multilayer perceptrons, each
 *     x (n_in thicknesses, normalised as (x - in_shift) * in_scale)
 *     -> n_layers x [Linear(n_hidden) + GELU in its erf form, x Phi(x)
 *        (erf evaluated to 1.2e-7 absolute)] -> Linear(n_out),
 *   trained with Adam on the squared error summed over the outputs and averaged
 *   over the batch (the reported loss is the mean squared error per output);
 *   BF16 weights and activations
 *   with FP32 accumulation (hand-written MFMA kernels), FP32 master weights,
 *   FP32 outputs.
 *
 * Conventions are those of tmm_rt.h: device pointers unless marked host,
 * asynchronous on the given stream unless stated, status codes, no exceptions,
 * tmm_last_error() for messages.  A handle owns its device memory from create
 * to destroy (allocated on the device current at create); calls on one handle
 * must not overlap.
 */
#ifndef TMM_SURROGATE_H
#define TMM_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "tmm_rt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmm_surrogate tmm_surrogate;

typedef struct tmm_surrogate_config {
    int32_t n_in;       /* input features (layer thicknesses), >= 1; padded to a multiple of 128 inside */
    int32_t n_hidden;   /* width of every hidden layer, multiple of 128                              */
    int32_t n_layers;   /* number of hidden layers, >= 1                                              */
    int32_t n_out;      /* outputs per sample, multiple of 128                                        */
    int32_t n_members;  /* ensemble size E, >= 1                                                      */
    int32_t max_batch;  /* rows per internal batch, multiple of 128                                   */
    uint64_t seed;      /* weight initialisation                                                      */
    float in_shift, in_scale;                  /* input normalisation                                 */
    float lr, beta1, beta2, eps, weight_decay; /* Adam (lr here is informative; train_step takes lr) */
    int32_t gemm_tile;  /* GEMM workgroup tile: 0 automatic; 1 = 256 x 256 (eight waves), 2 = 256 x 128
                           (eight waves), 3 = 128 x 128 (four waves).  A forced tile that does not
                           divide a product's M and N falls back to the automatic choice for it.   */
    int32_t sigma_window; /* 0 .. 4096: half-width, in wavelengths, of the window over which
                           tmm_surrogate_predict_fallback takes the largest sigma of a spectrum
                           row (one stack, angle, polarisation) before comparing it with the
                           bound; 0 = each output's own sigma.  The members' curves can cross at
                           an isolated wavelength where their spread is tiny and the error is
                           not; the window maximum closes those gaps.                          */
} tmm_surrogate_config;

/* Allocate and initialise (weights U(-a, a), a = sqrt(6/fan_in) for hidden layers
 * and sqrt(3/fan_in) for the output layer, zero biases) on the current device.
 * Synchronous.  *out receives the handle. */
tmm_status tmm_surrogate_create(const tmm_surrogate_config *cfg, tmm_surrogate **out);

/* Free the handle and its device memory (synchronises the device).  NULL is a no-op. */
tmm_status tmm_surrogate_destroy(tmm_surrogate *h);

/* Parameters per member: every layer's weights [out][in] (layer 0 with the input
 * padded to a multiple of 128; padded columns are zero) followed by every layer's
 * biases [out].  0 for a NULL handle. */
size_t tmm_surrogate_param_count(const tmm_surrogate *h);

/* Copy the FP32 master parameters of all members to / from host memory, member
 * after member in the layout above (n_floats >= E * param_count).  Synchronous.
 * Import resets the optimiser state. */
tmm_status tmm_surrogate_export(const tmm_surrogate *h, float *host, size_t n_floats);
tmm_status tmm_surrogate_import(tmm_surrogate *h, const float *host, size_t n_floats);

/* One Adam step of every member on the same batch: x [B][n_in], y [B][n_out]
 * FP32 targets, 1 <= B <= max_batch; lr >= 0.  loss (device, [E] floats, or
 * NULL) receives each member's mean squared error on the batch before the step. */
tmm_status tmm_surrogate_train_step(tmm_surrogate *h, const float *x, const float *y, int32_t B, float lr,
                                    float *loss, void *stream);

/* Gradients of the batch objective (sum over outputs, mean over the batch of the
 * squared error) w.r.t. every parameter, no update:
 * grads (device) [E][param_count] FP32 in the export layout. */
tmm_status tmm_surrogate_gradients(tmm_surrogate *h, const float *x, const float *y, int32_t B, float *grads,
                                   void *stream);

/* Inference on x [B][n_in] (any B >= 0, processed in chunks of max_batch):
 * mean [B][n_out] ensemble mean, sigma [B][n_out] sample standard deviation
 * over members (0 for E = 1), members [E][B][n_out] every member's output.
 * Any of the three may be NULL, not both mean and members. */
tmm_status tmm_surrogate_predict(tmm_surrogate *h, const float *x, int32_t B, float *mean, float *sigma,
                                 float *members, void *stream);

/* Surrogate with transfer-matrix fallback at point granularity: predict as
 * above, then every output whose error estimate err_scale * sigma_w exceeds
 * bound (or whose sigma_w is NaN) is recomputed by the transfer-matrix kernels,
 * where sigma_w is the largest sigma of the output's spectrum row within
 * cfg.sigma_window wavelengths of it (the output's own sigma for a window of 0)
 * (float32), and replaced in out.  A unit is one (stack, angle, wavelength) with
 * its P polarisation outputs; a unit is recomputed when any of its outputs is
 * flagged.  A stack whose units are all flagged goes through tmm_rt on the
 * gathered stacks; the flagged units of the other stacks go through the
 * point-list kernel of tmm_rt_points, which writes into out in place.
 * tmpl describes the same B stacks for tmm_rt: L = n_in layers whose
 * thicknesses are x, material ids (mat, required), the index table, the grids
 * and pol_mask, with P * n_theta * n_wl = n_out so that out [B][n_out] has the
 * layout of tmm_rt's R; its d and output fields are ignored.  n_fallback (host,
 * may be NULL) receives the number of outputs replaced.  Synchronises the
 * stream once per max_batch chunk (to size the fallback launches).  Allocates
 * nothing: the lists and staging buffers belong to the handle (created with it). */
tmm_status tmm_surrogate_predict_fallback(tmm_surrogate *h, const float *x, int32_t B, const tmm_rt_args *tmpl,
                                          float err_scale, float bound, float *out, int64_t *n_fallback,
                                          void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TMM_SURROGATE_H */
