/*
 * tmm_ragged -- transfer-matrix evaluation of ragged batches: stacks with
 * different numbers of layers, wavelength grids and angle grids, in one
 * persistent launch on one MI355X (gfx950).  Plain C interface; conventions of
 * tmm_rt.h (device pointers unless marked host, status codes, tmm_last_error).
 *
 * The physics is that of tmm_rt (paper: "Physical Background", Eq. (1)-(7));
 * the paper evaluates one dense [N, L] batch at a time (section
 * "Implementation in Numpy", App. A.2), and its reinforcement-learning
 * environment builds stacks of varying length (section "Environment"), which
 * is what a ragged batch serves.
 *
 * A plan is made once per batch shape from host copies of three offset
 * arrays; it owns device copies of them, the work lists and the launch shape
 * an autotuner picks on the first run (timing a few shapes on the real data
 * and caching the winner per (dtype, polarisation, mean layer count, size)).
 * A work unit is a tile of consecutive (angle, wavelength) points of one
 * stack, longest stacks first.  The autotuner chooses the workgroup shape, the
 * units taken per counter update, and the lanes per point: 1 (64-point
 * tiles), or 2 / 4 (32- / 16-point tiles, the stack's layers split across the
 * lanes of a point and their 2x2 transfer operators composed across lanes).
 */
#ifndef TMM_RAGGED_H
#define TMM_RAGGED_H

#include <stddef.h>
#include <stdint.h>

#include "tmm_rt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tmm_ragged_plan tmm_ragged_plan;

/*
 * Per-call data (device pointers).  Stack b (0 <= b < B) has the finite layers
 * layer_off[b] .. layer_off[b+1]-1, the wavelengths wl_off[b] .. wl_off[b+1]-1
 * and the angles th_off[b] .. th_off[b+1]-1 of the plan's offset arrays.
 *  d          [layer_off[B]] real thicknesses.
 *  mat        [layer_off[B]] int32 index-table rows of the finite layers.
 *  ends       [B][2] int32 rows of the ambient and the substrate.
 *  wl         [wl_off[B]] vacuum wavelengths.
 *  sin_theta, cos_theta  [th_off[B]] (computed in double precision, then cast).
 *  nk         [n_mat][wl_off[B]] complex interleaved: row m, column wl_off[b]+i
 *             is the index of material m at stack b's i-th wavelength.
 *  n_mat      1 .. 8.
 *  R, T       [output_size] real: stack b's block starts at its output
 *             offset and is [P][n_theta_b][n_wl_b].
 *  r, t       [output_size] complex interleaved, the same layout: the
 *             amplitudes of tmm_rt (Eq. (7); the same phase convention).
 * Any of R, T, r, t may be NULL, not all four.  A run that asks for r or t uses
 * the amplitude kernels: one lane per point, with a launch shape tuned (and
 * cached) for them separately from the R and T runs' shape, which is the one
 * tmm_ragged_plan_shape reports and tmm_ragged_plan_set_shape fixes.
 * Invalid values (negative / non-finite thickness, row out of range, absorbing
 * ambient at oblique incidence) give NaN, as in tmm_rt.
 */
typedef struct tmm_ragged_data {
    const void *d;
    const int32_t *mat;
    const int32_t *ends;
    const void *wl;
    const void *sin_theta;
    const void *cos_theta;
    const void *nk;
    int32_t n_mat;
    void *R, *T;
    void *r, *t;
} tmm_ragged_data;

/* Build a plan.  layer_off, wl_off, th_off: HOST arrays [B+1] starting at 0
 * (non-decreasing; every stack has at least one wavelength and one angle).
 * pol_mask: TMM_POL_S, TMM_POL_P or TMM_POL_BOTH.  Allocates device memory on
 * the current device.  Synchronous. */
tmm_status tmm_ragged_plan_create(int32_t B, const int64_t *layer_off, const int64_t *wl_off,
                                  const int64_t *th_off, uint32_t pol_mask, tmm_ragged_plan **out);

/* Free a plan (synchronises the device).  NULL is a no-op. */
tmm_status tmm_ragged_plan_destroy(tmm_ragged_plan *plan);

/* Number of elements of R (and of T): sum over stacks of P * n_theta_b * n_wl_b
 * (-1 for a NULL plan). */
int64_t tmm_ragged_plan_output_size(const tmm_ragged_plan *plan);

/* The output offsets [B+1] into host memory. */
tmm_status tmm_ragged_plan_output_offsets(const tmm_ragged_plan *plan, int64_t *host_out_off);

/* Evaluate every stack: asynchronous on the stream, except that the first run
 * of a plan for a dtype (when the shape is not cached yet) times several launch
 * shapes and synchronises; every one of those launches writes the full output,
 * and the output left is that of the chosen shape (the same bits as later runs). */
tmm_status tmm_ragged_run(tmm_ragged_plan *plan, const tmm_ragged_data *data, tmm_dtype dtype, void *stream);

/* The same call under the name of the paper-style entry points (tmm_rt,
 * tmm_rt_grad, tmm_rt_points): ragged batches of the section "Environment"
 * (stacks of varying length). */
tmm_status tmm_rt_ragged(tmm_ragged_plan *plan, const tmm_ragged_data *data, tmm_dtype dtype, void *stream);

/* The launch shape the autotuner chose for dtype (after the first run):
 * host_shape[4] = {workgroups per CU, units per counter update, waves per
 * workgroup, lanes per point}.  TMM_ERR_INVALID_ARG before tuning. */
tmm_status tmm_ragged_plan_shape(const tmm_ragged_plan *plan, tmm_dtype dtype, int32_t *host_shape);

/* Set the launch shape for dtype instead of tuning (same layout as above):
 * at most 12 waves per workgroup in TMM_F64 and 16 in TMM_F32 (the kernels'
 * register limits), at most 32 waves per CU.  The LDS of a workgroup must fit
 * the CU (TMM_F64: 8 KiB phase table plus 2 KiB per index-table row and wave;
 * TMM_F32: 4 KiB plus 1.5 KiB); an oversized shape fails at launch with
 * TMM_ERR_HIP. */
tmm_status tmm_ragged_plan_set_shape(tmm_ragged_plan *plan, tmm_dtype dtype, const int32_t *host_shape);

/* Capture the run (counter reset + persistent kernel) into a HIP graph owned by
 * the plan, replacing any earlier capture; tunes first if needed.  stream must
 * not be the default stream.  The graph keeps the data pointers given here. */
tmm_status tmm_ragged_capture(tmm_ragged_plan *plan, const tmm_ragged_data *data, tmm_dtype dtype, void *stream);

/* Launch the captured graph on the stream. */
tmm_status tmm_ragged_replay(tmm_ragged_plan *plan, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TMM_RAGGED_H */
