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
constexpr float kLn2 = 0.6931471805599453f;
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

// ---- opacity-aware tile culling (GS_OPT_TIGHT) ---------------------------------
// A Gaussian with centre (mx, my), conic (a, b, c) and opacity o stays in a tile while the
// ellipse q(p) = (p - mu')^T conic (p - mu') <= Q, Q = 2 ln(255 o) + kTightMargin, meets the
// rectangle spanned by the tile's pixel centres.  Per tile row the ellipse's part inside the
// row's band of pixel-centre rows is convex, so the tiles it meets are one contiguous span:
// its x-extent runs from the left boundary at the band height nearest the ellipse's leftmost
// point to the right boundary at the height nearest its rightmost point.
//
// The preprocess counts entries and the binning places them with these functions, from the
// same stored values, so both agree exactly; contraction into FMAs is off inside them, so
// that agreement does not depend on how each kernel is compiled.  The arithmetic is FP32 in
// coordinates relative to the footprint's top-left tile (|values| of a few hundred pixels at
// most), with the hardware square root and reciprocal (a few ulp, one instruction each), which
// keeps the error in q near 1e-4 or below.
constexpr double kTightMargin = 0.01;

__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

struct TightEllipse {
  float mxr, myr;          // centre relative to (16 x0, 16 y0)
  float a, b, c, det, Q, inv_a;
  float ymax, ys;          // half-height of the ellipse; height of its leftmost point
  int x0, x1, y0;          // footprint columns [x0, x1], first row y0
  bool empty;
};

__device__ __forceinline__ TightEllipse tight_ellipse(double mx, double my, float a, float b, float c, float opacity,
                                                      int x0, int x1, int y0) {
#pragma clang fp contract(off)
  TightEllipse e;
  e.mxr = (float)(mx - 16.0 * x0);
  e.myr = (float)(my - 16.0 * y0);
  e.a = a;
  e.b = b;
  e.c = c;
  e.det = a * c - b * b;
  e.Q = (float)(2.0 * log(255.0 * (double)opacity) + kTightMargin);
  e.x0 = x0;
  e.x1 = x1;
  e.y0 = y0;
  e.empty = !(e.Q >= 0.0f) || !(e.det > 0.0f) || !(a > 0.0f) || !(c > 0.0f);
  const float inv_det = e.empty ? 0.0f : hw_rcp(e.det);
  e.inv_a = e.empty ? 0.0f : hw_rcp(a);
  e.ymax = e.empty ? 0.0f : hw_sqrt(e.Q * a * inv_det);
  e.ys = e.empty ? 0.0f : b * hw_sqrt(e.Q * hw_rcp(c) * inv_det);
  return e;
}

// Tiles [*lo, *hi] of tile row ty that the ellipse meets (*lo > *hi when none).
__device__ __forceinline__ void tight_row_span(const TightEllipse &e, int ty, int *lo, int *hi) {
#pragma clang fp contract(off)
  *lo = e.x0;
  *hi = e.x0 - 1;
  if (e.empty) return;
  const float top = (float)((ty - e.y0) * kTile) + 0.5f - e.myr;   // first pixel-centre row of the band
  const float dy0 = fmaxf(top, -e.ymax), dy1 = fminf(top + (float)(kTile - 1), e.ymax);
  if (dy0 > dy1) return;
  const float dl = fminf(fmaxf(e.ys, dy0), dy1), dr = fminf(fmaxf(-e.ys, dy0), dy1);
  const float aQ = e.a * e.Q;
  const float xl = e.mxr + (-e.b * dl - hw_sqrt(fmaxf(aQ - e.det * dl * dl, 0.0f))) * e.inv_a;
  const float xr = e.mxr + (-e.b * dr + hw_sqrt(fmaxf(aQ - e.det * dr * dr, 0.0f))) * e.inv_a;
  // tile x0 + k meets [xl, xr] (relative) when 16 k + 0.5 <= xr and 16 k + 15.5 >= xl
  const float kl = fmaxf(ceilf((xl - (kTile - 0.5f)) * (1.0f / kTile)), 0.0f);
  const float kh = fminf(floorf((xr - 0.5f) * (1.0f / kTile)), (float)(e.x1 - e.x0));
  if (kl <= kh) {
    *lo = e.x0 + (int)kl;
    *hi = e.x0 + (int)kh;
  }
}

// Opacity-aware culling with GxG groups (G <= 8).  Group row gy holds tile rows
// [gy G, gy G + G) of the footprint; a group is kept while the span of one of those rows
// reaches one of its G tile columns, i.e. lies partly in [gx G, gx G + G).  A row's span
// [lo, hi] does so for the group columns [lo / G, hi / G]; the kept columns of a group row are
// the union of those ranges over its rows (not always one interval: a thin, slanted ellipse
// can pass the one-pixel gap between two rows' pixel-centre bands far to the side).
struct TightGroupRow {
  int lo[8], hi[8];   // group columns reached from each tile row (lo > hi: none)
  int cmin, cmax;     // their hull (cmin > cmax: none)
  bool chain;         // the reached rows are consecutive and each range meets or touches the
                      // previous one, so the union is the hull (the usual case)
};

__device__ __forceinline__ TightGroupRow tight_group_row(const TightEllipse &e, int G, int gy, int y1) {
  TightGroupRow r;
  r.cmin = 1 << 30;
  r.cmax = -1;
  r.chain = true;
  int plo = 0, phi = -1;     // the previous tile row's range
  bool seen = false, ended = false;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    r.lo[i] = 0;
    r.hi[i] = -1;
    const int ty = gy * G + i;
    if (i < G && ty >= e.y0 && ty <= y1) {
      int lo, hi;
      tight_row_span(e, ty, &lo, &hi);
      if (lo <= hi) {
        r.lo[i] = lo / G;
        r.hi[i] = hi / G;
        r.cmin = min(r.cmin, r.lo[i]);
        r.cmax = max(r.cmax, r.hi[i]);
        if (ended || (seen && (r.lo[i] > phi + 1 || r.hi[i] < plo - 1))) r.chain = false;
        seen = true;
        plo = r.lo[i];
        phi = r.hi[i];
      } else if (seen) {
        ended = true;
      }
    }
  }
  return r;
}

__device__ __forceinline__ bool tight_group_has(const TightGroupRow &r, int c) {
  bool any = false;
#pragma unroll
  for (int i = 0; i < 8; ++i) any |= (r.lo[i] <= c) & (c <= r.hi[i]);
  return any;
}

__device__ __forceinline__ uint32_t tight_group_count(const TightGroupRow &r) {
  if (r.cmin > r.cmax) return 0u;
  if (r.chain) return (uint32_t)(r.cmax - r.cmin + 1);
  uint32_t n = 0;
  for (int c = r.cmin; c <= r.cmax; ++c) n += tight_group_has(r, c) ? 1u : 0u;
  return n;
}

// Group column of the row's kept group number `nth` (nth < tight_group_count(r)).
__device__ __forceinline__ int tight_group_nth(const TightGroupRow &r, uint32_t nth) {
  if (r.chain) return r.cmin + (int)nth;
  for (int c = r.cmin; c <= r.cmax; ++c) {
    if (!tight_group_has(r, c)) continue;
    if (nth == 0) return c;
    --nth;
  }
  return r.cmax;   // (not reached)
}

// Membership mask of group (gx, gy) under the culling: bit (ty % G) G + (tx % G) for each
// member tile the ellipse meets.
__device__ __forceinline__ uint64_t tight_group_mask(const TightEllipse &e, int G, int gx, int gy, int y1) {
  uint64_t m = 0;
  for (int ly = 0; ly < G; ++ly) {
    const int ty = gy * G + ly;
    if (ty < e.y0 || ty > y1) continue;
    int lo, hi;
    tight_row_span(e, ty, &lo, &hi);
    lo = max(lo, gx * G);
    hi = min(hi, gx * G + G - 1);
    if (lo <= hi) m |= (((1ull << (hi - lo + 1)) - 1ull) << (lo - gx * G)) << (ly * G);
  }
  return m;
}

// ---- preprocess + scans ------------------------------------------------------
// scan_tmp (scan_tmp_bytes(n) bytes, may be null): when scan_presummed(n), the preprocess also
// leaves there the tile sums of the count scan, and launch_scan_compact(.., presummed = true)
// then skips its reduce pass
bool scan_presummed(int64_t n);
hipError_t launch_preprocess(const gs_scene &s, const gs_camera &c, const Grid &g, const gs_projected &o,
                             bool tight, void *scan_tmp, hipStream_t st);
// Scans (reduce-then-scan); tmp holds scan_tmp_bytes(n) bytes.
size_t scan_tmp_bytes(int64_t n);
// out[0..n] = exclusive prefix sum of in[0..n) (out[n] = total); order[0..*nvis) = indices i
// with in[i] > 0, in index order
hipError_t launch_scan_compact(const uint32_t *in, uint64_t *out, int64_t n, uint32_t *order, uint32_t *nvis,
                               void *tmp, bool presummed, hipStream_t st);
// out[0..m] = exclusive prefix sum of in[idx[i]] for i < m = *n_dev (m <= n_max)
hipError_t launch_scan_gather(const uint32_t *in, const uint32_t *idx, uint64_t *out, int64_t n_max,
                              const uint32_t *n_dev, void *tmp, hipStream_t st);
// entries per block of the binning's block firsts (the first Gaussian of each block of entries)
constexpr uint64_t kFirstsBlock = 1024;

// ---- binning, sort, ranges -------------------------------------------------
// scratch of a radix sort over at most n keys (per-tile digit counts and digit totals)
size_t radix_tmp_bytes(uint64_t n);
// scratch of the depth sort of n_max keys (sort_depth; counts, totals and the last pass's weights)
size_t depth_sort_tmp_bytes(uint64_t n_max);
// Stable sort of (keys, vals) on key bits [lo, hi); ping-pongs with (keys_alt, vals_alt) and
// reports in *in_alt whether the result ended in the alternate buffers.
hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n, int lo,
                      int hi, void *tmp, hipStream_t st, bool *in_alt);
// keys[i] = depth bits of order[i] for i < *nvis (n_max >= *nvis), counts = {*K, *nvis} (the
// entry and visible counts side by side, for one copy to the host), the low 32 bits of counts[2]
// = *K if *K <= capacity else 0 (the entry count the device-count bin sort takes), and in tmp
// the first depth pass's per-tile digit counts for the sort_depth call that follows (same n_max
// and tmp).
hipError_t launch_depth_keys(const uint32_t *order, const float4 *rgb, const uint32_t *nvis, uint64_t n_max,
                             uint32_t *keys, const uint64_t *K, uint64_t *counts, uint64_t *host_counts,
                             uint64_t capacity, void *tmp, hipStream_t st);
// Sorts the visible list order[0..*nvis) stably by the depth keys in keys (four passes over
// bits [0, 31): depths are positive), using keys_alt, vals_alt and vals_b (n_max each) as
// scratch; the sorted depth keys end in keys.  The last pass also writes dpos[i] = the
// entries of the Gaussians before the i-th in depth order (the exclusive scan of count[order[i]],
// dpos[*nvis] = all entries) and first[b] = the i whose entries hold entry b * kFirstsBlock, for
// b < nfirst.  n_max > 1 (otherwise nothing is done).  Reads the visible count on the device,
// so it can be enqueued before the host knows it.
hipError_t sort_depth(uint32_t *order, const uint32_t *nvis, uint64_t n_max, uint32_t *keys, uint32_t *keys_alt,
                      uint32_t *vals_alt, uint32_t *vals_b, void *tmp, hipStream_t st, const uint32_t *count,
                      uint64_t *dpos, uint32_t *first, uint64_t nfirst);
// Entries of the V depth-ordered visible Gaussians (the i-th one's first entry at dpos[i];
// dkeys[i] its depth bits) as (bin key, rank in depth order) pairs in (bkey, bval), a stable
// sort on the bin bits ping-ponging with (bkey_alt, bval_alt) whose last pass writes the final
// Gaussian indices to vals and the 64-bit keys to keys, then the bin ranges (cleared first) and,
// for group > 1, the membership masks.  With tight (opacity-aware culling) entries follow the
// culled spans of tight_row_span.  vals and keys must not alias the four work arrays.
// block_first (or nullptr): the first Gaussian of every 1,024-entry block (sort_depth).
// V_dev and K_dev (both or neither): the visible and entry counts read on the device, V and K
// then upper bounds of them (grids sized for K; the surplus workgroups return at once).
hipError_t bin_and_sort(const uint32_t *order, const uint32_t *dkeys, const uint64_t *dpos, const uint32_t *block_first,
                        uint32_t V, uint64_t K, const uint32_t *V_dev, const uint32_t *K_dev,
                        const uint16_t *rect, const double *xy, const float *conic, bool tight, const Grid &g,
                        uint32_t *bkey, uint32_t *bval, uint32_t *bkey_alt, uint32_t *bval_alt, uint32_t *ranges,
                        void *masks, uint32_t *vals, uint64_t *keys, void *tmp, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);

// ---- XCD-aware work order ---------------------------------------------------------------
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b to XCD b % 8), and each XCD
// has its own L2.  Work whose neighbours share data is therefore given to the XCDs in
// contiguous pieces rather than one unit per XCD in turn.
constexpr int kXcds = 8;

// Sort tile of workgroup b when the ntiles tiles of a sort are split into 8 contiguous ranges
// of per = ceil(ntiles / 8), XCD x walking [x per, (x + 1) per) in order: the runs that
// neighbouring tiles scatter side by side into each digit's output then share one L2.  ntiles
// may be known only on the device (a sort of a device-counted length); the grid is
// xcd_sort_grid(t) workgroups for any t >= ntiles, and a workgroup with no tile gets ~0u.
inline unsigned xcd_sort_grid(uint64_t tiles) {
  const uint64_t per = (tiles + kXcds - 1) / kXcds;
  return (unsigned)((per ? per : 1) * kXcds);
}
__device__ __forceinline__ uint32_t xcd_sort_tile(uint32_t b, uint64_t ntiles) {
  const uint32_t per = (uint32_t)((ntiles + kXcds - 1) / kXcds), k = b / kXcds;
  if (k >= per) return ~0u;
  const uint32_t t = (b % kXcds) * per + k;
  return t < ntiles ? t : ~0u;
}

// Bin of workgroup b of a single-image raster launch of xcd_raster_grid(GX, GY) workgroups:
// blocks of kXcdBlock x kXcdBlock neighbouring bins, XCD x taking blocks x, x + 8, x + 16, ...
// and each block's bins in turn, so that neighbouring bins (which share most of their
// Gaussians) read them through one L2 while every XCD still draws blocks from the whole frame.
// -1 for a workgroup past the frame's bins.
constexpr int kXcdBlock = 4;
inline unsigned xcd_raster_grid(int GX, int GY) {
  const int nb = ((GX + kXcdBlock - 1) / kXcdBlock) * ((GY + kXcdBlock - 1) / kXcdBlock);
  return (unsigned)(((nb + kXcds - 1) / kXcds) * kXcds * kXcdBlock * kXcdBlock);
}
__device__ __forceinline__ int xcd_raster_bin(int b, int GX, int GY) {
  constexpr int kPer = kXcdBlock * kXcdBlock;
  const int x = b % kXcds, k = b / kXcds;
  const int block = x + kXcds * (k / kPer), within = k % kPer;
  const int nbx = (GX + kXcdBlock - 1) / kXcdBlock;
  const int gx = (block % nbx) * kXcdBlock + within % kXcdBlock;
  const int gy = (block / nbx) * kXcdBlock + within / kXcdBlock;
  return (gx < GX && gy < GY) ? gy * GX + gx : -1;
}

// ---- rasterizers -------------------------------------------------------------
struct RasterJob {
  const double2 *xy;
  const float4 *conic;
  const float4 *rgb;
  const uint32_t *vals;
  const void *masks;       // uint16_t per entry for G = 2, 4; uint64_t for G = 8
  const uint32_t *ranges;
  float *image;
  float *aux;
  int W, H, TX, TY, GX, GY;
  int nbins;
  int parts;  // workgroups per bin: each takes G^2 / parts of the group's member tiles (row-major)
  int items;  // nbins * parts work items (one workgroup each)
  int bin0;   // first work item of this job in a batched launch
};

struct RasterParams {
  int G, prec, splits;
  float bg[3];
  uint32_t aux_flags;
  bool all_rows;               // every quadrant runs every row (no quadrant culling)
  bool tile_rows;              // grouped MFMA rasterizers: each member tile builds its own rows
};

hipError_t launch_raster_fp32(const RasterJob &j, const RasterParams &p, hipStream_t st);
hipError_t launch_raster_mfma(const RasterJob &j, const RasterParams &p, hipStream_t st);
// Jobs of one batched launch, passed by value as a kernel argument (copied at launch).
constexpr int kMaxBatch = 32;
struct BatchTable {
  int n_jobs, total;
  RasterJob jobs[kMaxBatch];   // jobs[j].bin0: first (job, bin) item of job j, ascending
};
// Persistent batched launches: `grid` workgroups take items [0, table.total) from the counters
// (zeroed before).  The items form kBatchSeqs interleaved sequences of kBatchRun-item runs
// (sequence c: runs c, c + 8, c + 16, ...), each drained one item per claim by the workgroups b
// with b % kBatchSeqs == c through its own counter, kBatchCounterStride words from the next.
// With one counter for every workgroup the claims queued on one address: 140 µs for the 8,160
// bins of a 1080p frame against 78 µs for the single-image launch (100 µs now).  As workgroup b
// runs on XCD b mod 8, a sequence's runs of neighbouring bins (a job's bins are row-major) also
// read their shared Gaussians through one L2.  (Claims of four items were slower, 179 µs: the
// workgroups that start last then hold four items each.)  Every sequence with items has
// workgroups (grid >= 8, or grid = total < 8 with every item in run 0), so every item is taken
// exactly once.
constexpr int kBatchSeqs = 8;
constexpr int kBatchRun = 16;
constexpr int kBatchCounterStride = GS_BATCH_COUNTER_BYTES / 4 / kBatchSeqs;
static_assert(kBatchCounterStride >= 16, "counters of the batched launch share a 64-byte line");

// Item of claim k of sequence c (increasing in k).
__device__ __forceinline__ int64_t batch_item(uint32_t k, int c) {
  return ((int64_t)(k / kBatchRun) * kBatchSeqs + c) * kBatchRun + (int64_t)(k % kBatchRun);
}

// The work loop of a persistent batched rasterizer: item(i) renders work item i.  The next claim
// is issued before the current item is rendered, so its round trip overlaps it; the barriers
// around each hand-over also keep an item's staging out of LDS still read for the one before.
template <typename F>
__device__ __forceinline__ void batch_items(uint32_t *counters, int total, int *s_item, F &&item) {
  const int seq = (int)(blockIdx.x % kBatchSeqs);
  uint32_t *ctr = counters + seq * kBatchCounterStride;
  if (threadIdx.x == 0) {
    const int64_t i = batch_item(atomicAdd(ctr, 1u), seq);
    *s_item = i < total ? (int)i : total;
  }
  __syncthreads();
  int it = *s_item;
  __syncthreads();
  while (it < total) {
    uint32_t nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(ctr, 1u);
    item(it);
    if (threadIdx.x == 0) {
      const int64_t i = batch_item(nxt, seq);
      *s_item = i < total ? (int)i : total;
    }
    __syncthreads();
    it = *s_item;
    __syncthreads();
  }
}

hipError_t launch_raster_fp32_batch(const BatchTable &table, int grid, const RasterParams &p, uint32_t *counter,
                                    hipStream_t st);
hipError_t launch_raster_mfma_batch(const BatchTable &table, int grid, const RasterParams &p, uint32_t *counter,
                                    hipStream_t st);

}  // namespace gsi
