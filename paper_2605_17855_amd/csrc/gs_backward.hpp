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
};

hipError_t launch_raster_backward(const BackwardJob &j, hipStream_t st);

}  // namespace gsi
