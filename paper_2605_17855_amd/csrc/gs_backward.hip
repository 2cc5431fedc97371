// Backward pass of the FP32 compositing: the derivative of the forward recurrence of the
// plain rasterizer (paper, Background: eq. power_d, eq. power, the 1/255 cut, the 0.99
// clamp, the 1e-4 stop) on the branch the forward takes.
//
// One 256-lane workgroup per 16x16 tile, one pixel per lane, 8x8 quadrants per wave as in
// the forward.  Two passes over the tile's depth-sorted list, each staged through LDS in
// chunks of 256 entries:
//  1. the forward recurrence again, in the forward rasterizer's FP32 arithmetic (the same
//     operations in the same order, so every cut, clamp and stop is decided the same way),
//     for the pixel's final transmittance T_end and the end of its blended prefix;
//  2. the list back to front.  T_i = T_{i+1} / (1 - alpha_i) (a 1-ulp hardware reciprocal)
//     recovers the transmittance in front of each blended Gaussian and S, the colour the
//     later Gaussians add, grows by c_i alpha_i T_i.  A pair's nine gradient terms are
//     summed over the wave (a reduce-scatter with lane swaps, then DPP row sums) and nine
//     lanes add them to the Gaussian's gradients, one hardware FP32 atomic add each (the
//     buffers are ordinary device memory).
#include "gs_backward.hpp"
#include "gs_mfma.hpp"

namespace gsi {
namespace {

struct BwdShared {
  float4 a[kBlock];   // (u, v, -a/2 log2e, -b log2e): centre relative to the tile, power rows
  float4 b[kBlock];   // (-c/2 log2e, log2 o, r, g)
  float4 c[kBlock];   // (b colour, conic a, conic b, conic c)
  float2 d[kBlock];   // (1 / opacity, Gaussian index bits)
  uint32_t last;      // end of the longest blended prefix of the tile's pixels
};

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of each row (every lane of the row gets it): quad_perm [1,0,3,2] and
// [2,3,0,1], then the half-row and row mirrors.
__device__ __forceinline__ float row_sum(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return v;
}

// Reduce-scatter steps of two registers at once.  swap32_add: lanes 0..31 get a[i] + a[i+32],
// lanes 32..63 get b[i-32] + b[i].  swap16_add (rows of 16 lanes): row 0 gets a's rows 0 + 1,
// row 1 b's rows 0 + 1, row 2 a's rows 2 + 3, row 3 b's rows 2 + 3.
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wave sums of the nine gradient terms v[0..8], added to the Gaussian's gradients by nine lanes
// in one hardware FP32 atomic.  After the two swap steps the rows of x0 hold the partial sums
// of terms (0, 2, 1, 3), those of x1 terms (4, 6, 5, 7) and every row of x2 term 8; a row sum
// completes each.  Term f goes to rgb[3g + f] (f < 3), opacity[g] (3), conic[3g + f - 4]
// (4..6), xy[2g + f - 7] (7, 8).
__device__ __forceinline__ void add_terms(const BackwardJob &J, const float (&v)[9], uint32_t g, int lane) {
  const float x0 = row_sum(swap16_add(swap32_add(v[0], v[1]), swap32_add(v[2], v[3])));
  const float x1 = row_sum(swap16_add(swap32_add(v[4], v[5]), swap32_add(v[6], v[7])));
  const float w8 = swap32_add(v[8], v[8]);
  const float x2 = row_sum(swap16_add(w8, w8));
  const int row = lane >> 4, c = lane & 15;
  if (c < 2 || (c == 2 && row == 0)) {
    const int rf = row == 1 ? 2 : row == 2 ? 1 : row;
    const int f = c == 0 ? rf : c == 1 ? 4 + rf : 8;
    const float val = c == 0 ? x0 : c == 1 ? x1 : x2;
    const size_t G = g;
    float *dst = f < 3 ? J.g_rgb + 3 * G + f
               : f == 3 ? J.g_op + G
               : f < 7 ? J.g_conic + 3 * G + (f - 4)
               : J.g_xy + 2 * G + (f - 7);
    unsafeAtomicAdd(dst, val);
  }
}

__device__ __forceinline__ void stage(const BackwardJob &J, BwdShared &sm, uint32_t cs, int cnt, int ox, int oy) {
  const int t = threadIdx.x;
  if (t < cnt) {
    const uint32_t g = J.vals[cs + t];
    const double2 m = J.xy[g];
    const float4 co = J.conic[g];
    const float4 cl = J.rgb[g];
    sm.a[t] = make_float4((float)(m.x - ox), (float)(m.y - oy), -0.5f * kLog2e * co.x, -kLog2e * co.y);
    sm.b[t] = make_float4(-0.5f * kLog2e * co.z, __log2f(co.w), cl.x, cl.y);
    sm.c[t] = make_float4(cl.z, co.x, co.y, co.z);
    sm.d[t] = make_float2(1.0f / co.w, __uint_as_float(g));
  }
}

__global__ __launch_bounds__(kBlock) void k_raster_backward(BackwardJob J) {
  __shared__ BwdShared sm;
  const int tile = blockIdx.x;
  const int ox = (tile % J.TX) * kTile, oy = (tile / J.TX) * kTile;
  const uint32_t start = J.ranges[2 * tile], end = J.ranges[2 * tile + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int px = (w & 1) * 8 + (lane & 7), py = (w >> 1) * 8 + (lane >> 3);
  const float X = px + 0.5f, Y = py + 0.5f;
  const bool inside = (ox + px < J.W) && (oy + py < J.H);

  // pass 1: the forward recurrence
  float T = 1.0f;
  float cut = inside ? kCutLog2 : INFINITY;
  uint32_t last = start;
  if (t == 0) sm.last = start;
  for (uint32_t cs = start; cs < end; cs += kBlock) {
    const int cnt = (int)min((uint32_t)kBlock, end - cs);
    __syncthreads();
    stage(J, sm, cs, cnt, ox, oy);
    if (!__syncthreads_or(cut != INFINITY)) break;
    for (int j = 0; j < cnt; ++j) {
      const float4 A = sm.a[j];
      const float4 B = sm.b[j];
      const float dx = X - A.x, dy = Y - A.y;
      const float D = fmaf(dx, fmaf(A.z, dx, A.w * dy), fmaf(B.x * dy, dy, B.y));
      if (D >= cut) {
        const float al = fminf(kAlphaMax, __builtin_amdgcn_exp2f(D));
        const float Tn = fmaf(-T, al, T);
        if (Tn >= kTMin) {
          T = Tn;
          last = cs + (uint32_t)j + 1u;
        } else {
          cut = INFINITY;
        }
      }
    }
  }
  __syncthreads();
  atomicMax(&sm.last, last);
  __syncthreads();
  const uint32_t tile_last = sm.last;

  // pass 2: back to front
  const int64_t HW = (int64_t)J.W * J.H;
  const int64_t pix = (int64_t)(oy + py) * J.W + (ox + px);
  const float gp0 = inside ? J.dimage[pix] : 0.0f;
  const float gp1 = inside ? J.dimage[HW + pix] : 0.0f;
  const float gp2 = inside ? J.dimage[2 * HW + pix] : 0.0f;
  const float bT0 = J.bg[0] * T, bT1 = J.bg[1] * T, bT2 = J.bg[2] * T;
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
  for (uint32_t ce = tile_last; ce > start;) {
    const int cnt = (int)min((uint32_t)kBlock, ce - start);
    const uint32_t cs = ce - (uint32_t)cnt;
    __syncthreads();
    stage(J, sm, cs, cnt, ox, oy);
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const float4 A = sm.a[j];
      const float4 B = sm.b[j];
      const float dx = X - A.x, dy = Y - A.y;
      const float D = fmaf(dx, fmaf(A.z, dx, A.w * dy), fmaf(B.x * dy, dy, B.y));
      const bool act = (cs + (uint32_t)j < last) && (D >= kCutLog2);
      if (__ballot(act) == 0) continue;
      float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      if (act) {
        const float4 Cc = sm.c[j];
        const float rop = sm.d[j].x;
        const float raw = __builtin_amdgcn_exp2f(D);
        const float al = fminf(kAlphaMax, raw);
        const float inv = __builtin_amdgcn_rcpf(1.0f - al);   // 1 - alpha >= 0.01
        const float Ti = T * inv;
        const float wgt = al * Ti;
        v[0] = gp0 * wgt;
        v[1] = gp1 * wgt;
        v[2] = gp2 * wgt;
        const float dLda = gp0 * (B.z * Ti - (S0 + bT0) * inv) + gp1 * (B.w * Ti - (S1 + bT1) * inv) +
                           gp2 * (Cc.x * Ti - (S2 + bT2) * inv);
        const float dLdp = raw < kAlphaMax ? dLda * al : 0.0f;
        v[3] = dLdp * rop;
        v[4] = -0.5f * dx * dx * dLdp;
        v[5] = -dx * dy * dLdp;
        v[6] = -0.5f * dy * dy * dLdp;
        v[7] = (Cc.y * dx + Cc.z * dy) * dLdp;
        v[8] = (Cc.z * dx + Cc.w * dy) * dLdp;
        S0 = fmaf(B.z, wgt, S0);
        S1 = fmaf(B.w, wgt, S1);
        S2 = fmaf(Cc.x, wgt, S2);
        T = Ti;
      }
      add_terms(J, v, __float_as_uint(sm.d[j].y), lane);
    }
    ce = cs;
  }
}

// ---- backward of the MFMA forward ------------------------------------------------------
// The same derivative as above, for the image the tensorized forward writes: the power of each
// (Gaussian, pixel) pair comes from the forward's own MFMA contraction (the Gaussian-side row and
// the pixel-side operand built by the same functions, so D = log2(alpha_raw) is bit-identical to
// the forward's and every cut, clamp and stop is decided the same way), and the forward's final
// transmittance and blended-prefix end (GS_AUX_TFINAL, GS_AUX_LAST) replace the replay pass.
//
// One workgroup per tile, chunks of 256 entries from the tile's longest blended prefix back to
// its first entry.  Each wave takes only the rows whose alpha can reach the cut in its 8x8
// quadrant (quadrant culling, as in the forward), as 32-row MFMA blocks; after the lane swap a
// lane holds the 32 rows' D for its pixel and walks them back to front.  A row is active for a
// pixel when it lies before the pixel's blended-prefix end and D reaches the cut (the forward
// blended exactly those).  The per-pair gradient terms and their wave sums and atomics are those
// of the FP32 backward, with d = pixel centre - centre formed in the tile frame.
template <int S>
struct BwdMfmaShared {
  static constexpr int RS = (S == 3) ? 32 : 16;
  __align__(16) uint16_t A[kBlock * RS];   // Gaussian-side rows
  float4 p0[kBlock];   // (u, v, conic a, conic b): centre in the tile frame
  float4 p1[kBlock];   // (conic c, 1 / opacity, r, g)
  float2 p2[kBlock];   // (b, Gaussian index bits)
  uint8_t qm[kBlock];  // quadrant masks
  uint8_t wl[4][kBlock];
  uint32_t last;
};

template <int PREC, int S>
__global__ __launch_bounds__(kBlock) void k_raster_backward_mfma(BackwardJob J, int all_rows) {
  using N = mfma::Narrow<PREC>;
  constexpr int RS = BwdMfmaShared<S>::RS;
  __shared__ BwdMfmaShared<S> sm;
  const int tile = blockIdx.x;
  const int ox = (tile % J.TX) * kTile, oy = (tile / J.TX) * kTile;
  const uint32_t start = J.ranges[2 * tile], len = J.ranges[2 * tile + 1] - start;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int px = (w & 1) * 8 + (lane & 7), py = (w >> 1) * 8 + (lane >> 3);
  const float xi = (float)(px - 8), yi = (float)(py - 8);   // pixel centre in the tile frame
  const bool inside = (ox + px < J.W) && (oy + py < J.H);
  mfma::short8 B0, B1, B20, B21;
  mfma::make_pixel_operand<PREC>(B0, B1, B20, B21);

  const int64_t HW = (int64_t)J.W * J.H;
  const int64_t pix = (int64_t)(oy + py) * J.W + (ox + px);
  float T = inside ? J.t_final[pix] : 1.0f;
  // (a blended-prefix end beyond the tile's list cannot come from the forward; clamped so that no
  // entry outside the tile is read)
  const uint32_t last = inside ? min((uint32_t)J.last[pix], len) : 0u;
  if (t == 0) sm.last = 0;
  __syncthreads();
  atomicMax(&sm.last, last);
  __syncthreads();
  const uint32_t tile_last = sm.last;

  const float gp0 = inside ? J.dimage[pix] : 0.0f;
  const float gp1 = inside ? J.dimage[HW + pix] : 0.0f;
  const float gp2 = inside ? J.dimage[2 * HW + pix] : 0.0f;
  const float bT0 = J.bg[0] * T, bT1 = J.bg[1] * T, bT2 = J.bg[2] * T;
  float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
  mfma::short8 pad = {}, zero = {};
  if (lane < 32) pad[5] = (short)N::enc(-1000.0f);

  for (uint32_t ce = tile_last; ce > 0;) {
    const int cnt = (int)min((uint32_t)kBlock, ce);
    const uint32_t cs = ce - (uint32_t)cnt;   // positions in the tile's list
    __syncthreads();
    if (t < cnt) {
      const uint32_t g = J.vals[start + cs + t];
      const double2 m = J.xy[g];
      const float4 co = J.conic[g];
      const float4 cl = J.rgb[g];
      const float u = (float)(m.x - ((double)ox + 8.5)), v = (float)(m.y - ((double)oy + 8.5));
      const float l2o = mfma::log2_opacity(co.w);
      mfma::build_row<PREC, S>(&sm.A[t * RS], u, v, co.x, co.y, co.z, l2o);
      sm.p0[t] = make_float4(u, v, co.x, co.y);
      sm.p1[t] = make_float4(co.z, 1.0f / co.w, cl.x, cl.y);
      sm.p2[t] = make_float2(cl.z, __uint_as_float(g));
      sm.qm[t] = all_rows ? (uint8_t)0xF : (uint8_t)mfma::quad_mask(u, v, co.x, co.y, co.z, l2o);
    }
    __syncthreads();
    const int n = mfma::wave_list(sm.qm, cnt, sm.wl[w]);
    for (int blk = ((n + 31) >> 5) - 1; blk >= 0; --blk) {
      const int slot = 32 * blk + (lane & 31);
      const bool real = slot < n;
      const int rr = real ? (int)sm.wl[w][slot] : 0;
      const uint16_t *rp = sm.A + (size_t)rr * RS + 8 * (lane >> 5);
      const mfma::short8 a = real ? *reinterpret_cast<const mfma::short8 *>(rp) : pad;
      mfma::float16v z = {};
      mfma::float16v d0 = N::mma(a, B0, z);
      mfma::float16v d1 = N::mma(a, B1, z);
      if (S == 3) {
        const mfma::short8 a2 = real ? *reinterpret_cast<const mfma::short8 *>(rp + 16) : zero;
        d0 = N::mma(a2, B20, d0);
        d1 = N::mma(a2, B21, d1);
      }
      float D[32];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        auto pr = __builtin_amdgcn_permlane32_swap(__float_as_uint(d0[j]), __float_as_uint(d1[j]), false, false);
        D[8 * (j >> 2) + (j & 3)] = __uint_as_float(pr[0]);
        D[8 * (j >> 2) + 4 + (j & 3)] = __uint_as_float(pr[1]);
      }
#pragma unroll
      for (int m = 31; m >= 0; --m) {
        const int sl = 32 * blk + m;
        if (sl >= n) continue;                      // (uniform)
        const int ri = sm.wl[w][sl];
        const bool act = (cs + (uint32_t)ri < last) && (D[m] >= kCutLog2);
        if (__ballot(act) == 0) continue;
        float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (act) {
          const float4 P0 = sm.p0[ri];
          const float4 P1 = sm.p1[ri];
          const float bcol = sm.p2[ri].x;
          const float dx = xi - P0.x, dy = yi - P0.y;
          const float raw = __builtin_amdgcn_exp2f(D[m]);
          const float al = fminf(kAlphaMax, raw);
          const float inv = __builtin_amdgcn_rcpf(1.0f - al);   // 1 - alpha >= 0.01
          const float Ti = T * inv;
          const float wgt = al * Ti;
          v[0] = gp0 * wgt;
          v[1] = gp1 * wgt;
          v[2] = gp2 * wgt;
          const float dLda = gp0 * (P1.z * Ti - (S0 + bT0) * inv) + gp1 * (P1.w * Ti - (S1 + bT1) * inv) +
                             gp2 * (bcol * Ti - (S2 + bT2) * inv);
          const float dLdp = raw < kAlphaMax ? dLda * al : 0.0f;
          v[3] = dLdp * P1.y;
          v[4] = -0.5f * dx * dx * dLdp;
          v[5] = -dx * dy * dLdp;
          v[6] = -0.5f * dy * dy * dLdp;
          v[7] = (P0.z * dx + P0.w * dy) * dLdp;
          v[8] = (P0.w * dx + P1.x * dy) * dLdp;
          S0 = fmaf(P1.z, wgt, S0);
          S1 = fmaf(P1.w, wgt, S1);
          S2 = fmaf(bcol, wgt, S2);
          T = Ti;
        }
        add_terms(J, v, __float_as_uint(sm.p2[ri].y), lane);
      }
    }
    ce = cs;
  }
}

template <int PREC>
hipError_t launch_bwd_mfma_p(const BackwardJob &j, int splits, int all_rows, unsigned tiles, hipStream_t st) {
  switch (splits) {
    case 1: hipLaunchKernelGGL((k_raster_backward_mfma<PREC, 1>), dim3(tiles), dim3(kBlock), 0, st, j, all_rows); break;
    case 2: hipLaunchKernelGGL((k_raster_backward_mfma<PREC, 2>), dim3(tiles), dim3(kBlock), 0, st, j, all_rows); break;
    case 3:
      if (PREC == GS_PREC_FP16_MFMA) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_raster_backward_mfma<PREC, 3>), dim3(tiles), dim3(kBlock), 0, st, j, all_rows);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_backward_mfma(const BackwardJob &j, int prec, int splits, bool all_rows, hipStream_t st) {
  const int tiles = j.TX * j.TY;
  if (tiles == 0) return hipSuccess;
  if (prec == GS_PREC_FP16_MFMA) return launch_bwd_mfma_p<GS_PREC_FP16_MFMA>(j, splits, all_rows ? 1 : 0, tiles, st);
  if (prec == GS_PREC_BF16_MFMA) return launch_bwd_mfma_p<GS_PREC_BF16_MFMA>(j, splits, all_rows ? 1 : 0, tiles, st);
  return hipErrorInvalidValue;
}

hipError_t launch_raster_backward(const BackwardJob &j, hipStream_t st) {
  const int tiles = j.TX * j.TY;
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_backward, dim3((unsigned)tiles), dim3(kBlock), 0, st, j);
  return hipGetLastError();
}

}  // namespace gsi
