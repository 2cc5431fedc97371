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
//  2. the list back to front.  T_i = T_{i+1} / (1 - alpha_i) recovers the transmittance in
//     front of each blended Gaussian and S, the colour the later Gaussians add, grows by
//     c_i alpha_i T_i.  A pair's nine gradient terms are summed over the wave with
//     DPP and lane swaps, and nine lanes add them to the Gaussian's gradients, one hardware FP32
//     atomic add each (the buffers are ordinary device memory).
#include "gs_backward.hpp"

namespace gsi {
namespace {

struct BwdShared {
  float4 a[kBlock];   // (u, v, -a/2 log2e, -b log2e): centre relative to the tile, power rows
  float4 b[kBlock];   // (-c/2 log2e, log2 o, r, g)
  float4 c[kBlock];   // (b colour, conic a, conic b, conic c)
  float2 d[kBlock];   // (opacity, Gaussian index bits)
  uint32_t last;      // end of the longest blended prefix of the tile's pixels
};

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes, the same bits in every lane (each step adds a lane's value to its
// partner's, symmetric in the two).  Within 16-lane rows by DPP: quad_perm [1,0,3,2] and
// [2,3,0,1], then the half-row and row mirrors; across rows by the lane-swap instructions:
// rows 0 <-> 1 and 2 <-> 3, then the two halves of the wave.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
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
    sm.d[t] = make_float2(co.w, __uint_as_float(g));
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
        const float op = sm.d[j].x;
        const float raw = __builtin_amdgcn_exp2f(D);
        const float al = fminf(kAlphaMax, raw);
        const float inv = 1.0f / (1.0f - al);
        const float Ti = T * inv;
        const float wgt = al * Ti;
        v[0] = gp0 * wgt;
        v[1] = gp1 * wgt;
        v[2] = gp2 * wgt;
        const float dLda = gp0 * (B.z * Ti - (S0 + bT0) * inv) + gp1 * (B.w * Ti - (S1 + bT1) * inv) +
                           gp2 * (Cc.x * Ti - (S2 + bT2) * inv);
        const float dLdp = raw < kAlphaMax ? dLda * al : 0.0f;
        v[3] = dLdp / op;
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
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = wave_sum(v[k]);
      // every lane holds the nine sums: lanes 0..8 add one each, in one vector atomic
      if (lane < 9) {
        const size_t g = __float_as_uint(sm.d[j].y);
        float val = v[0];
#pragma unroll
        for (int k = 1; k < 9; ++k) val = (lane == k) ? v[k] : val;
        float *dst = lane < 3 ? J.g_rgb + 3 * g + lane
                   : lane == 3 ? J.g_op + g
                   : lane < 7 ? J.g_conic + 3 * g + (lane - 4)
                   : J.g_xy + 2 * g + (lane - 7);
        unsafeAtomicAdd(dst, val);
      }
    }
    ce = cs;
  }
}

}  // namespace

hipError_t launch_raster_backward(const BackwardJob &j, hipStream_t st) {
  const int tiles = j.TX * j.TY;
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_backward, dim3((unsigned)tiles), dim3(kBlock), 0, st, j);
  return hipGetLastError();
}

}  // namespace gsi
