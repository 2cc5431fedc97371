// Shared pieces of the tensorized power (paper: "Tensorizing the Power Computation",
// "Padding the Inner Dimension", "Warp-Level WMMA Mapping") used by the MFMA rasterizer and the
// MFMA backward pass: the 16-bit operand encoders, the Gaussian-side row builder, the pixel-side
// operand, quadrant culling and the per-wave row lists.  Both kernels build a Gaussian's row
// and the pixel operand with these same functions, so their MFMA results agree bit for bit.
#pragma once

#include "gs_internal.hpp"

namespace gsi {
namespace mfma {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short short8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));


template <int PREC>
struct Narrow;

// The encoders take their argument as a materialised FP32 value (the empty asm pins it to a
// register): otherwise the compiler may fuse the FP32 multiply that produced it with the
// conversion into one mixed-precision FMA, which rounds once instead of twice, and may do so
// in one kernel and not in another, so the same Gaussian's row would differ between the
// ungrouped, grouped and batched rasterizers.
__device__ __forceinline__ float as_fp32(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <>
struct Narrow<GS_PREC_FP16_MFMA> {
  static constexpr float kScale = 2048.0f;            // 2^11
  __device__ static __forceinline__ uint16_t enc(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)as_fp32(x));
  }
  __device__ static __forceinline__ float dec(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
  __device__ static __forceinline__ float16v mma(short8 a, short8 b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(half8, a), __builtin_bit_cast(half8, b), c, 0,
                                                  0, 0);
  }
};

template <>
struct Narrow<GS_PREC_BF16_MFMA> {
  static constexpr float kScale = 256.0f;             // 2^8
  __device__ static __forceinline__ uint16_t enc(float x) { return __builtin_bit_cast(uint16_t, (__bf16)as_fp32(x)); }
  __device__ static __forceinline__ float dec(uint16_t h) { return (float)__builtin_bit_cast(__bf16, h); }
  __device__ static __forceinline__ float16v mma(short8 a, short8 b, float16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  }
};

// LDS row of one Gaussian: RS 16-bit slots.  Slot (h, i) of MFMA 0 is row[8h + i]; MFMA 1
// (splits == 3) uses row[16 + 8h + i].
//   splits 1: [k0..k5, 0, 0 | 0 x 8]
//   splits 2: [k0..k5, l0, l1 | l2..l5, 0 x 4]
//   splits 3: the splits-2 row, then [m0..m5, 0, 0 | 0 x 8]
//
// log2 of a Gaussian's opacity, the form the row and the quadrant test take it in (one
// transcendental instruction; opacities are normal numbers in (0, 1]).
__device__ __forceinline__ float log2_opacity(float o) { return __builtin_amdgcn_logf(o); }

// Contraction is off here: with it, the compiler may fuse the product that forms k[i] with
// the subtraction that forms the residual (one rounding instead of two), and whether it does
// depends on the surrounding code, so the same Gaussian's row could differ between the
// ungrouped, grouped and batched kernels.  Every operation below rounds as written.
// l2o = log2_opacity(o); the constant slot is log2(o) - (log2 e / 2) q.
template <int PREC, int S>
__device__ __forceinline__ void build_row(uint16_t *row, float u, float v, float a, float b, float c, float l2o) {
#pragma clang fp contract(off)
  using N = Narrow<PREC>;
  const float p3 = fmaf(a, u, b * v), p4 = fmaf(b, u, c * v);
  const float q = fmaf(u, p3, v * p4);
  float k[6] = {-0.5f * kLog2e * a, -kLog2e * b, -0.5f * kLog2e * c, kLog2e * p3, kLog2e * p4,
                fmaf(-0.5f * kLog2e, q, l2o)};
  uint16_t hi[6], lo[6], lo2[6] = {};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    hi[i] = N::enc(k[i]);
    float r = (k[i] - N::dec(hi[i])) * N::kScale;
    lo[i] = N::enc(r);
    if constexpr (S == 3) {   // (the encoders' register pin would keep an unused third piece alive)
      r = (r - N::dec(lo[i])) * N::kScale;
      lo2[i] = N::enc(r);
    }
  }
  short8 v0, v1;
#pragma unroll
  for (int i = 0; i < 6; ++i) v0[i] = (short)hi[i];
  v0[6] = S >= 2 ? (short)lo[0] : 0;
  v0[7] = S >= 2 ? (short)lo[1] : 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) v1[i] = S >= 2 ? (short)lo[2 + i] : 0;
#pragma unroll
  for (int i = 4; i < 8; ++i) v1[i] = 0;
  *reinterpret_cast<short8 *>(row) = v0;
  *reinterpret_cast<short8 *>(row + 8) = v1;
  if (S == 3) {
    short8 v2, v3;
#pragma unroll
    for (int i = 0; i < 6; ++i) v2[i] = (short)lo2[i];
    v2[6] = v2[7] = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) v3[i] = 0;
    *reinterpret_cast<short8 *>(row + 16) = v2;
    *reinterpret_cast<short8 *>(row + 24) = v3;
  }
}

// Quadrant culling.  Wave w blends the pixels of quadrant (w & 1, w >> 1) only, so a row that
// cannot pass the 1/255 alpha cut at any pixel centre of that quadrant is left out of the
// wave's MFMA blocks.  Bit qx + 2 qy of the mask is set unless the minimum of the conic's
// quadratic form q(d) = a dx^2 + 2 b dx dy + c dy^2 over the quadrant's pixel centres exceeds
// 2 ln(255 o) + kQuadMargin (alpha >= 1/255 reads q <= 2 ln(255 o)).  The margin in q, 0.72
// in log2(alpha), is far above the rounding of this test and of the split 16-bit power, so a
// left-out row is one whose D stays below the cut at every pixel of the quadrant: the blended
// result is the one every row would give.
//
// A rectangle that does not hold the centre has its minimum on an edge that faces the
// centre.  Along the facing horizontal edge y = ey the minimum is at dx = -b dy / a clamped
// into the edge, and q = a (dx + b dy / a)^2 + (det / a) dy^2 holds only non-negative terms;
// likewise along the facing vertical edge.  Clamping the centre into the rectangle picks the
// facing edges; a centre inside gives q = 0.
constexpr float kQuadMargin = 1.0f;
constexpr float kQuadQ0 = 11.0825270f + kQuadMargin;   // 2 ln 255 + margin

__device__ __forceinline__ uint32_t quad_mask(float u, float v, float a, float b, float c, float l2o) {
#pragma clang fp contract(off)
  const float Q = fmaf(2.0f * kLn2, l2o, kQuadQ0);   // 2 ln(o) + 2 ln 255 + margin
  if (!(Q > 0.0f)) return 0u;               // o < 1/255 e^{-margin/2}: never reaches the cut
  const float det = (float)((double)a * c - (double)b * b);
  if (!(a > 0.0f && c > 0.0f && det > 0.0f)) return 0xFu;
  const float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
  const float ba = b * ia, bc = b * ic, ga = det * ia, gc = det * ic;
  uint32_t mask = 0;
#pragma unroll
  for (int qy = 0; qy < 2; ++qy) {
#pragma unroll
    for (int qx = 0; qx < 2; ++qx) {
      const float xl = (float)(8 * qx - 8), xh = (float)(8 * qx - 1);
      const float yl = (float)(8 * qy - 8), yh = (float)(8 * qy - 1);
      // facing horizontal edge
      const float dy = fminf(fmaxf(v, yl), yh) - v;
      const float th = -ba * dy;
      const float sh = fminf(fmaxf(th, xl - u), xh - u) - th;
      const float qh = fmaf(a * sh, sh, ga * dy * dy);
      // facing vertical edge
      const float dx = fminf(fmaxf(u, xl), xh) - u;
      const float tv = -bc * dx;
      const float sv = fminf(fmaxf(tv, yl - v), yh - v) - tv;
      const float qv = fmaf(c * sv, sv, gc * dx * dx);
      if (fminf(qh, qv) <= Q) mask |= 1u << (qx + 2 * qy);
    }
  }
  return mask;
}

// Compacts, in order, the rows [0, nrows) whose quadrant mask holds this wave's bit into the
// wave's own list; returns its length (uniform).  IDX holds a row index (uint8_t up to 256 rows).
template <typename IDX>
__device__ __forceinline__ int wave_list(const uint8_t *qm, int nrows, IDX *wl) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int n = 0;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    const int r = r0 + lane;
    const bool in = r < nrows && ((qm[r] >> w) & 1u);
    const uint64_t b = __ballot(in);
    if (in) wl[n + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = (IDX)r;
    n += __popcll(b);
  }
  // the list is written and read by lanes of this wave only
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return n;
}

// Compacts, in order, the rows [0, nrows) whose 16-bit mask has bit `bit` into the wave's own
// list; returns its length (uniform).  (The grouped rasterizer keeps one quadrant bit per
// member tile and wave in each row's mask.)
template <typename IDX>
__device__ __forceinline__ int wave_list_bit(const uint16_t *qm, int nrows, int bit, IDX *wl) {
  const int lane = threadIdx.x & 63;
  int n = 0;
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    const int r = r0 + lane;
    const bool in = r < nrows && ((qm[r] >> bit) & 1u);
    const uint64_t b = __ballot(in);
    if (in) wl[n + __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = (IDX)r;
    n += __popcll(b);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  return n;
}

// Pixel-side operand: phi of this lane's panel pixel (n = lane % 32) in both panels, in a frame
// whose origin lies (xo, yo) pixels before the tile's own (the tile frame for xo = yo = 0; the
// frame of a tile group for the grouped rasterizer).  The entries are integers, exact in the
// 16-bit formats while |x|, |y| <= 32 (FP16) or <= 16 (BF16).
template <int PREC>
__device__ __forceinline__ void make_pixel_operand(short8 &B0, short8 &B1, short8 &B20, short8 &B21, int xo = 0,
                                                   int yo = 0) {
  const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3;   // the wave's quadrant
  const int qx0 = (w & 1) * 8, qy0 = (w >> 1) * 8;
  {
    using N = Narrow<PREC>;
    const int n = lane & 31, h = lane >> 5;
    const float inv = 1.0f / N::kScale, inv2 = inv * inv;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float x = (float)(qx0 + (n & 7) - 8 + xo), y = (float)(qy0 + (n >> 3) + 4 * p - 8 + yo);
      const float phi[6] = {x * x, x * y, y * y, x, y, 1.0f};
      short8 b, b2;
      if (h == 0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) b[i] = (short)N::enc(phi[i]);
        b[6] = (short)N::enc(phi[0] * inv);
        b[7] = (short)N::enc(phi[1] * inv);
#pragma unroll
        for (int i = 0; i < 6; ++i) b2[i] = (short)N::enc(phi[i] * inv2);
        b2[6] = b2[7] = 0;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (short)N::enc(phi[2 + i] * inv);
#pragma unroll
        for (int i = 4; i < 8; ++i) b[i] = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) b2[i] = 0;
      }
      if (p == 0) { B0 = b; B20 = b2; } else { B1 = b; B21 = b2; }
    }
  }

}

}  // namespace mfma
}  // namespace gsi
