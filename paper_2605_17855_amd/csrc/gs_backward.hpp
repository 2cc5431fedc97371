// Backward pass of the FP32 compositing: the job one launch processes and its launcher.
#pragma once

#include "gs_backward.h"
#include "gs_internal.hpp"

namespace gsi {

struct BackwardJob {
  const double2 *xy;       // n projected centres (FP64)
  const float4 *conic;     // n x (a, b, c, opacity)
  const float4 *rgb;       // n x (r, g, b, depth)
  const uint32_t *vals;    // Gaussian index of each sorted entry
  const uint32_t *ranges;  // per tile [start, end) of its depth-sorted entries
  const float *dimage;     // 3 x H x W
  float *g_rgb, *g_op, *g_conic, *g_xy;
  int W, H, TX, TY;
  float bg[3];
  // MFMA backward only: the forward's final transmittance and blended-prefix end planes (H x W)
  const float *t_final;
  const float *last;
};

hipError_t launch_raster_backward(const BackwardJob &j, hipStream_t st);
// The backward of the MFMA forward (precision GS_PREC_FP16_MFMA or GS_PREC_BF16_MFMA, 1..3
// splits): the power from the same MFMA contraction as the forward, the forward's state in
// place of a replay; all_rows runs every row in every quadrant (no quadrant culling).
hipError_t launch_raster_backward_mfma(const BackwardJob &j, int prec, int splits, bool all_rows, hipStream_t st);

}  // namespace gsi
