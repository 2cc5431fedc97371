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

}  // namespace

hipError_t launch_raster_backward(const BackwardJob &j, hipStream_t st) {
  const int tiles = j.TX * j.TY;
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_backward, dim3((unsigned)tiles), dim3(kBlock), 0, st, j);
  return hipGetLastError();
}

}  // namespace gsi
