// Plain FP32 rasterizer (paper, Background: tile-based rasterization, eq. power_d, eq. power).
//
// One 256-lane workgroup per bin (a tile, or a GxG tile group); each lane owns one pixel
// position and, for a group, that position in every member tile.  The bin's depth-sorted
// list is streamed through LDS in chunks of 256 entries.  Per (entry, pixel):
//   d = x - mu'                       (eq. power_d)
//   log2(alpha_raw) = log2(o) + log2(e) * (-1/2 d^T conic d)   (eq. power)
//   skip when alpha_raw < 1/255, alpha = min(0.99, alpha_raw)
//   T' = T (1 - alpha); stop (without blending) when T' < 1e-4; else C += alpha T c, T = T'.
// The pixel's offset to the centre is formed from a group-relative FP32 copy of the FP64
// centre, so |d| stays small and exact.  Lanes map to 8x8 quadrants per wave so that a
// splat that misses a quadrant is skipped by the whole wave.
#include "gs_internal.hpp"

namespace gsi {
namespace {


struct Fp32Shared {
  float4 a[kBlock];  // (u, v, -a/2 log2e, -b log2e)
  float4 b[kBlock];  // (-c/2 log2e, log2 o, r, g)
  float4 c[kBlock];  // (b, mask bits, -, -)
};

// Renders bin `bin` of job J (one workgroup; this rasterizer takes one work item per bin).
// Shared by the single-image and batched kernels.
template <int G, bool AUX>
__device__ __forceinline__ void raster_bin_fp32(const RasterJob &J, const RasterParams &P, int bin, Fp32Shared &sm) {
  constexpr int NT = G * G;
  const int gx = bin % J.GX, gy = bin / J.GX;
  const int ox = gx * G * kTile, oy = gy * G * kTile;
  const uint32_t start = J.ranges[2 * bin], end = J.ranges[2 * bin + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int px = (w & 1) * 8 + (lane & 7), py = (w >> 1) * 8 + (lane >> 3);

  float T[NT], C0[NT], C1[NT], C2[NT], Ws[NT], cut[NT];
  uint32_t nstop[NT], nseen[NT], nblend[NT], nlast[NT];
  float X[NT], Y[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int lx = (k % G) * kTile + px, ly = (k / G) * kTile + py;
    X[k] = lx + 0.5f;
    Y[k] = ly + 0.5f;
    const bool inside = (ox + lx < J.W) && (oy + ly < J.H);
    T[k] = 1.0f; C0[k] = C1[k] = C2[k] = 0.0f; Ws[k] = 0.0f;
    cut[k] = inside ? kCutLog2 : INFINITY;
    nstop[k] = 0; nseen[k] = 0; nblend[k] = 0; nlast[k] = 0;
  }

  for (uint32_t cs = start; cs < end; cs += kBlock) {
    const int cnt = (int)min((uint32_t)kBlock, end - cs);
    __syncthreads();
    if (t < cnt) {
      const uint32_t e = cs + t;
      const uint32_t g = J.vals[e];
      const double2 m = J.xy[g];
      const float4 co = J.conic[g];
      const float4 cl = J.rgb[g];
      const uint32_t mk = (G > 1) ? (uint32_t) static_cast<const uint16_t *>(J.masks)[e] : 1u;
      sm.a[t] = make_float4((float)(m.x - ox), (float)(m.y - oy), -0.5f * kLog2e * co.x, -kLog2e * co.y);
      sm.b[t] = make_float4(-0.5f * kLog2e * co.z, __log2f(co.w), cl.x, cl.y);
      sm.c[t] = make_float4(cl.z, __uint_as_float(mk), 0.0f, 0.0f);
    }
    bool alive = false;
#pragma unroll
    for (int k = 0; k < NT; ++k) alive |= cut[k] != INFINITY;
    if (!__syncthreads_or(alive)) break;
    for (int j = 0; j < cnt; ++j) {
      if ((j & 31) == 0) {
        // a wave whose pixels have all stopped leaves the chunk early
        bool any = false;
#pragma unroll
        for (int k = 0; k < NT; ++k) any |= cut[k] != INFINITY;
        if (__ballot(any) == 0) break;
      }
      const float4 A = sm.a[j];
      const float4 B = sm.b[j];
      const float4 Cc = sm.c[j];
      const uint32_t mk = __float_as_uint(Cc.y);
#pragma unroll
      for (int k = 0; k < NT; ++k) {
        if (G > 1 && !((mk >> k) & 1u)) continue;
        if (AUX) nseen[k]++;
        const float dx = X[k] - A.x, dy = Y[k] - A.y;
        const float D = fmaf(dx, fmaf(A.z, dx, A.w * dy), fmaf(B.x * dy, dy, B.y));
        if (D >= cut[k]) {
          // branch-free body: T' = T (1 - alpha) as one FMA; a stop (T' < 1e-4) blends
          // nothing, keeps T and disables the pixel
          const float al = fminf(kAlphaMax, __builtin_amdgcn_exp2f(D));
          const float Tn = fmaf(-T[k], al, T[k]);
          const bool ok = Tn >= kTMin;
          const float wgt = ok ? al * T[k] : 0.0f;
          C0[k] = fmaf(wgt, B.z, C0[k]);
          C1[k] = fmaf(wgt, B.w, C1[k]);
          C2[k] = fmaf(wgt, Cc.x, C2[k]);
          T[k] = ok ? Tn : T[k];
          cut[k] = ok ? cut[k] : INFINITY;
          if (AUX) {
            Ws[k] += wgt;
            nblend[k] += ok ? 1u : 0u;
            nstop[k] = ok ? nstop[k] : nseen[k];
            nlast[k] = ok ? nseen[k] : nlast[k];
          }
        }
      }
    }
  }

  const int64_t HW = (int64_t)J.W * J.H;
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const int xx = ox + (k % G) * kTile + px, yy = oy + (k / G) * kTile + py;
    if (xx >= J.W || yy >= J.H) continue;
    const int64_t pix = (int64_t)yy * J.W + xx;
    J.image[pix] = C0[k] + T[k] * P.bg[0];
    J.image[HW + pix] = C1[k] + T[k] * P.bg[1];
    J.image[2 * HW + pix] = C2[k] + T[k] * P.bg[2];
    if (AUX) {
      int plane = 0;
      if (P.aux_flags & GS_AUX_TFINAL) J.aux[(plane++) * HW + pix] = T[k];
      if (P.aux_flags & GS_AUX_WSUM) J.aux[(plane++) * HW + pix] = Ws[k];
      if (P.aux_flags & GS_AUX_NEVAL) {
        const bool stopped = (cut[k] == INFINITY);
        J.aux[(plane++) * HW + pix] = (float)(stopped ? nstop[k] : nseen[k]);
      }
      if (P.aux_flags & GS_AUX_NBLEND) J.aux[(plane++) * HW + pix] = (float)nblend[k];
      if (P.aux_flags & GS_AUX_LAST) J.aux[(plane++) * HW + pix] = (float)nlast[k];
    }
  }
}

// One workgroup per bin, in the XCD-aware order of the MFMA rasterizer.
template <int G, bool AUX>
__global__ __launch_bounds__(kBlock) void k_raster_fp32(RasterJob J, RasterParams P) {
  __shared__ Fp32Shared sm;
  const int item = xcd_raster_bin((int)blockIdx.x, J.GX, J.GY);
  if (item < 0) return;
  raster_bin_fp32<G, AUX>(J, P, item, sm);
}

// Persistent batched rasterizer (see the MFMA variant).
template <int G, bool AUX>
__global__ __launch_bounds__(kBlock) void k_raster_fp32_batch(const BatchTable tb,
                                                              RasterParams P, uint32_t *counter) {
  __shared__ Fp32Shared sm;
  __shared__ int s_item;
  batch_items(counter, tb.total, &s_item, [&](int item) {
    int lo = 0, hi = tb.n_jobs;   // last job with bin0 <= item
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tb.jobs[mid].bin0 <= item) lo = mid; else hi = mid;
    }
    const RasterJob J = tb.jobs[lo];
    raster_bin_fp32<G, AUX>(J, P, item - J.bin0, sm);
  });
}

struct BatchArgs {
  const BatchTable *table;
  int grid;
  uint32_t *counter;
};

template <int G, bool AUX>
hipError_t launch_g(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  if (b) {
    hipLaunchKernelGGL((k_raster_fp32_batch<G, AUX>), dim3((unsigned)b->grid), dim3(kBlock), 0, st, *b->table, p,
                       b->counter);
  } else {
    hipLaunchKernelGGL((k_raster_fp32<G, AUX>), dim3(xcd_raster_grid(j.GX, j.GY)), dim3(kBlock), 0, st, j, p);
  }
  return hipGetLastError();
}

hipError_t dispatch(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  const bool aux = p.aux_flags != 0;
  switch (p.G) {
    case 1: return aux ? launch_g<1, true>(j, p, b, st) : launch_g<1, false>(j, p, b, st);
    case 2: return aux ? launch_g<2, true>(j, p, b, st) : launch_g<2, false>(j, p, b, st);
    case 4: return aux ? launch_g<4, true>(j, p, b, st) : launch_g<4, false>(j, p, b, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_raster_fp32(const RasterJob &j, const RasterParams &p, hipStream_t st) {
  if (j.items == 0) return hipSuccess;
  return dispatch(j, p, nullptr, st);
}

hipError_t launch_raster_fp32_batch(const BatchTable &table, int grid, const RasterParams &p, uint32_t *counter,
                                    hipStream_t st) {
  if (table.total == 0) return hipSuccess;
  BatchArgs b{&table, grid, counter};
  RasterJob dummy{};
  return dispatch(dummy, p, &b, st);
}

}  // namespace gsi
