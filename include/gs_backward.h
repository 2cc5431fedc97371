/*
 * gs_backward.h -- C ABI of the backward pass of the compositing (training side of the
 * renderer declared in gs.h).
 *
 * The paper trains models at FP16 as well as FP32, but states no backward pass of its own.
 * This call is the derivative of gs_rasterize's forward recurrence (Background: alpha =
 * min(0.99, o exp(power)), power = -1/2 d^T conic d with d = pixel centre - projected
 * centre (eq. power_d, eq. power), pairs with alpha < 1/255 skipped, C = sum alpha_i T_i
 * c_i + T_end bg, the stop before the Gaussian that would take T below 1e-4).  It is exact
 * on the branch the forward takes: clamped alphas, skipped pairs and the stop are held fixed.
 * Per pixel and blended Gaussian i, with S_i = sum over later Gaussians j of c_j alpha_j T_j:
 *   dC/dc_i     = alpha_i T_i
 *   dC/dalpha_i = c_i T_i - (S_i + T_end bg) / (1 - alpha_i)
 * and, where alpha_i is not clamped, dalpha/do = alpha / o, dalpha/dpower = alpha,
 * dpower/d(a, b, c) = -(dx^2 / 2, dx dy, dy^2 / 2), dpower/d(x, y) = (a dx + b dy, b dx + c dy).
 *
 * Conventions are those of gs.h (device pointers, caller-owned buffers, stream as void*,
 * host-side validation before any HIP call, messages in gs_last_error()), except that the
 * gradients are summed with floating-point atomics: repeated calls agree to rounding, not
 * bit for bit.
 */
#ifndef GS_BACKWARD_H
#define GS_BACKWARD_H

#include "gs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Per-Gaussian gradients, FP32, indexed like the gs_projected records (n entries each). */
typedef struct {
  float *rgb;               /* n x 3: dL/d(r, g, b) of the colour record */
  float *opacity;           /* n: dL/d(opacity) */
  float *conic;             /* n x 3: dL/d(a, b, c) of the conic [[a, b], [b, c]] */
  float *xy;                /* n x 2: dL/d(x, y) of the projected centre, in pixels */
} gs_grads;

/* Gradients of L = sum over channels and pixels of dimage * image, where image is what
 * gs_rasterize writes for (proj, bins, cam, opt) with opt->precision = GS_PREC_FP32; the
 * power is evaluated in FP32 exactly as that rasterizer does, so both take the same
 * branch at every pair.  dimage: 3 x H x W FP32 planes (the image's layout).
 * The gradients are ADDED to *grads (zero them before the first call; several views or
 * frames can be summed into one set of buffers) with hardware FP32 atomic adds, so the
 * four buffers must be ordinary (coarse-grained) device memory, as hipMalloc returns.
 * proj and bins are what gs_preprocess and gs_bin_sort wrote (opacity-aware bins, from
 * GS_OPT_TIGHT, give the same gradients).  Reads opt->group, which must be 1 (tile bins;
 * GS_ERR_UNSUPPORTED otherwise), and opt->bg; ignores the precision and the aux flags.
 * Asynchronous on `stream`. */
gs_status gs_rasterize_backward(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam,
                                const gs_options *opt, const float *dimage, const gs_grads *grads,
                                void *stream);

/* The same gradients for the image of the tensorized forward (opt->precision GS_PREC_FP16_MFMA or
 * GS_PREC_BF16_MFMA with opt->splits as in gs_rasterize; Background: eq. power as the MFMA
 * contraction of the design section).  The power of each pair is the forward's own MFMA result
 * (same Gaussian-side rows, same pixel-side operand), so the backward takes the forward's branch
 * at every pair; instead of replaying the forward it starts from the forward's state:
 *   t_final  H x W FP32: the forward's GS_AUX_TFINAL plane (final transmittance);
 *   last     H x W FP32: the forward's GS_AUX_LAST plane (end of the blended prefix),
 * both from gs_rasterize of the same (proj, bins, cam, opt) with aux_flags holding
 * GS_AUX_TFINAL | GS_AUX_LAST.  Tile bins only (opt->group 1, else GS_ERR_UNSUPPORTED);
 * GS_OPT_ALL_ROWS turns quadrant culling off (same gradients up to the order of the atomic sums).
 * Gradients are ADDED to *grads with FP32 atomics, as in gs_rasterize_backward.  Asynchronous. */
gs_status gs_rasterize_backward_mfma(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam,
                                     const gs_options *opt, const float *dimage, const float *t_final,
                                     const float *last, const gs_grads *grads, void *stream);

#ifdef __cplusplus
}
#endif

#endif
