// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gsi {

constexpr int kTile = 16;            // tile side in pixels (Background: 16x16 tiles)
constexpr int kBlock = 256;          // threads per workgroup for every kernel here
constexpr float kAlphaMax = 0.99f;   // opacity clamp
constexpr float kTMin = 1e-4f;       // transmittance stop
constexpr float kLog2e = 1.4426950408889634f;
// log2(1/255): the 1/255 alpha cut taken on log2(alpha)
constexpr float kCutLog2 = -7.994353436858858f;

struct Grid {
  int W, H, TX, TY, G, GX, GY;
  int64_t nbins;
};

inline Grid make_grid(int W, int H, int G) {
  Grid g;
  g.W = W;
  g.H = H;
  g.TX = (W + kTile - 1) / kTile;
  g.TY = (H + kTile - 1) / kTile;
  g.G = G;
  g.GX = (g.TX + G - 1) / G;
  g.GY = (g.TY + G - 1) / G;
  g.nbins = (int64_t)g.GX * g.GY;
  return g;
}

inline int bits_for(uint64_t v) {  // bits needed to represent values 0..v-1 (at least 1)
  int b = 1;
  while (b < 64 && (1ull << b) < v) ++b;
  return b;
}

// ---- preprocess + scans ------------------------------------------------------
hipError_t launch_preprocess(const gs_scene &s, const gs_camera &c, const Grid &g, const gs_projected &o,
                             hipStream_t st);
size_t scan_tmp_bytes(int64_t n);
// out[0..n] = exclusive prefix sum of in[0..n) (out[n] = total)
hipError_t launch_scan(const uint32_t *in, uint64_t *out, int64_t n, void *tmp, hipStream_t st);
// as launch_scan, and order[0..*nvis) = indices i with in[i] > 0, in index order
hipError_t launch_scan_compact(const uint32_t *in, uint64_t *out, int64_t n, uint32_t *order, uint32_t *nvis,
                               void *tmp, hipStream_t st);
// out[0..n] = exclusive prefix sum of in[idx[i]]
hipError_t launch_scan_gather(const uint32_t *in, const uint32_t *idx, uint64_t *out, int64_t n, void *tmp,
                              hipStream_t st);

// ---- binning, sort, ranges -------------------------------------------------
size_t sort_tmp_bytes(uint64_t n);
// Stable sort of (keys, vals) on key bits [lo, hi); ping-pongs with (keys_alt, vals_alt) and
// reports in *in_alt whether the result ended in the alternate buffers.
hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n, int lo,
                      int hi, void *tmp, hipStream_t st, bool *in_alt);
hipError_t radix_sort32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt, uint64_t n, int lo,
                        int hi, void *tmp, hipStream_t st, bool *in_alt);
int radix_passes(int lo, int hi);
hipError_t launch_depth_keys(const uint32_t *order, const float4 *rgb, uint32_t nvis, uint32_t *keys,
                             hipStream_t st);
// entries of the visible Gaussians order[0..nvis) (depth order), Gaussian i's first entry at dpos[i]
hipError_t launch_binning(const uint32_t *order, const uint64_t *dpos, uint32_t nvis, uint64_t K,
                          const uint16_t *rect, const Grid &g, uint32_t *bin_keys, uint32_t *vals, hipStream_t st);
hipError_t launch_ranges(const uint32_t *bin_keys, const uint32_t *vals, uint64_t n, const uint16_t *rect,
                         const float *rgb, const Grid &g, uint32_t *ranges, uint16_t *masks, uint64_t *keys,
                         hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);

// ---- rasterizers -------------------------------------------------------------
struct RasterJob {
  const double2 *xy;
  const float4 *conic;
  const float4 *rgb;
  const uint32_t *vals;
  const uint16_t *masks;
  const uint32_t *ranges;
  float *image;
  float *aux;
  int W, H, TX, TY, GX, GY;
  int nbins;
  int bin0;  // first (job, bin) work item of this job in a batched launch
};

struct RasterParams {
  int G, prec, splits;
  float bg[3];
  uint32_t aux_flags;
};

hipError_t launch_raster_fp32(const RasterJob &j, const RasterParams &p, hipStream_t st);
hipError_t launch_raster_mfma(const RasterJob &j, const RasterParams &p, hipStream_t st);
hipError_t launch_raster_batch(const RasterJob *table_dev, int n_jobs, int total_items, const RasterParams &p,
                               uint32_t *counter, hipStream_t st);

}  // namespace gsi
