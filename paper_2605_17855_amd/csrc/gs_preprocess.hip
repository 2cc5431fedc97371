// Frustum culling and feature computation (one lane per Gaussian, SoA loads), and the
// exclusive scan of per-Gaussian bin counts.
//
// Per Gaussian (paper, Background: "frustum culling", "feature computation"):
//   camera-space centre t = R mu + t_cam (FP64), cull t_z <= znear;
//   covariance Sigma = M diag(s)^2 M^T from the normalised quaternion M and s = exp(log_scale);
//   first-order projection Sigma' = J R Sigma R^T J^T + 0.3 I with the Jacobian J of the
//   pinhole map taken at the centre, its lateral coordinate clamped to 1.3x the half
//   field of view (FP32), conic = Sigma'^-1 (FP32);
//   projected centre mu' = (fx t_x/t_z + cx, fy t_y/t_z + cy) in FP64 (the centre feeds
//   d = x - mu' of eq. power_d at absolute pixel coordinates, where FP32 would leave
//   ~1e-4 px of rounding at 1080p);
//   footprint half-width r = 3 sqrt(lambda_max(Sigma')), tile rectangle of the square
//   [mu' - r, mu' + r], culled when it misses the grid;
//   colour = real SH (degree <= 3) at the unit direction from the camera centre, + 0.5,
//   clamped below at 0; depth = t_z.
#include "gs_internal.hpp"

namespace gsi {
namespace {

struct PreArgs {
  int64_t n;
  const float *mean, *log_scale, *quat, *opacity, *sh;
  double R[9], t[3];
  float Rf[9];
  double fx, fy, cx, cy, znear;
  float fxf, fyf, limx, limy;
  float campos[3];
  int TX, TY, G;
  int tight;   // opacity-aware tile culling (group 1)
  double2 *xy;
  float4 *conic;
  float4 *rgb;
  ushort4 *rect;
  uint32_t *count;
  uint64_t *bsum;   // if set: per-workgroup sums of the counts and of the visible flags, the
  uint32_t *bvis;   // tile sums of the count scan (256-value tiles)
};

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// exclusive scan over the workgroup; *total = sum over the workgroup
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *sh4, T *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T incl = wave_inclusive_scan<T>(v);
  if (lane == 63) sh4[w] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const T x = sh4[k];
    before += k < w ? x : (T)0;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Real orthonormal spherical harmonics with the Condon-Shortley phase, index l*l + l + m,
// for a unit direction (x, y, z).  Constants are sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
// times sqrt(2) for m != 0, folded with the polynomial factors of P_l^|m|:
//   l=0: 1/(2 sqrt(pi))
//   l=1: sqrt(3/(4 pi))
//   l=2: sqrt(15/(4 pi)), sqrt(5/(16 pi)), sqrt(15/(16 pi))
//   l=3: sqrt(35/(32 pi)), sqrt(105/(4 pi)), sqrt(21/(32 pi)), sqrt(7/(16 pi)), sqrt(105/(16 pi))
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *b) {
  b[0] = 0.28209479177387814f;
  if (DEG < 1) return;
  const float c1 = 0.4886025119029199f;
  b[1] = -c1 * y;
  b[2] = c1 * z;
  b[3] = -c1 * x;
  if (DEG < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, yz = y * z, xz = x * z;
  b[4] = 1.0925484305920792f * xy;
  b[5] = -1.0925484305920792f * yz;
  b[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
  b[7] = -1.0925484305920792f * xz;
  b[8] = 0.5462742152960396f * (xx - yy);
  if (DEG < 3) return;
  b[9] = -0.5900435899266435f * y * (3.0f * xx - yy);
  b[10] = 2.890611442640554f * xy * z;
  b[11] = -0.4570457994644658f * y * (5.0f * zz - 1.0f);
  b[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
  b[13] = -0.4570457994644658f * x * (5.0f * zz - 1.0f);
  b[14] = 1.445305721320277f * z * (xx - yy);
  b[15] = -0.5900435899266435f * x * (xx - 3.0f * yy);
}

// The SH degree is a template argument so that every coefficient load of a lane is issued
// before the first multiply-add uses one (a runtime-bounded loop would wait on each load in
// turn).  The per-Gaussian parameters are loaded before the near-plane test for the same
// reason: one round trip to memory instead of two.
template <int DEG>
__device__ __forceinline__ uint32_t preprocess_one(const PreArgs &a, int64_t g) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const int64_t n = a.n;
  uint32_t cnt = 0;
  ushort4 rc = make_ushort4(0, 0, 0, 0);

  const double px = a.mean[g], py = a.mean[n + g], pz = a.mean[2 * n + g];
  const float ls0 = a.log_scale[g], ls1 = a.log_scale[n + g], ls2 = a.log_scale[2 * n + g];
  float qw = a.quat[g], qx = a.quat[n + g], qy = a.quat[2 * n + g], qz = a.quat[3 * n + g];
  const float opac = a.opacity[g];
  const double tx = fma(a.R[0], px, fma(a.R[1], py, fma(a.R[2], pz, a.t[0])));
  const double ty = fma(a.R[3], px, fma(a.R[4], py, fma(a.R[5], pz, a.t[1])));
  const double tz = fma(a.R[6], px, fma(a.R[7], py, fma(a.R[8], pz, a.t[2])));

  if (tz > a.znear) {
    // scales and rotation
    const float s0 = expf(ls0), s1 = expf(ls1), s2 = expf(ls2);
    const float qi = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qi; qx *= qi; qy *= qi; qz *= qi;
    const float M[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    // Jacobian rows at the clamped lateral position
    const float tzf = (float)tz;
    const float ux = fminf(fmaxf((float)(tx / tz), -a.limx), a.limx);
    const float uy = fminf(fmaxf((float)(ty / tz), -a.limy), a.limy);
    const float izf = 1.0f / tzf;
    const float j00 = a.fxf * izf, j02 = -a.fxf * ux * izf;
    const float j11 = a.fyf * izf, j12 = -a.fyf * uy * izf;
    // T = J R (2x3), P = T M diag(s), Sigma' = P P^T + 0.3 I
    float T0[3], T1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T0[k] = j00 * a.Rf[k] + j02 * a.Rf[6 + k];
      T1[k] = j11 * a.Rf[3 + k] + j12 * a.Rf[6 + k];
    }
    const float sc[3] = {s0, s1, s2};
    float P0[3], P1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      P0[k] = (T0[0] * M[k] + T0[1] * M[3 + k] + T0[2] * M[6 + k]) * sc[k];
      P1[k] = (T1[0] * M[k] + T1[1] * M[3 + k] + T1[2] * M[6 + k]) * sc[k];
    }
    // Sigma' = P P^T + 0.3 I.  det(P P^T) = |P0 x P1|^2 (Cauchy-Binet), so every term of
    // det(Sigma') is non-negative and FP32 keeps full relative precision for thin splats.
    const float pxx = P0[0] * P0[0] + P0[1] * P0[1] + P0[2] * P0[2];
    const float pyy = P1[0] * P1[0] + P1[1] * P1[1] + P1[2] * P1[2];
    const float sxy = P0[0] * P1[0] + P0[1] * P1[1] + P0[2] * P1[2];
    const float cr0 = P0[1] * P1[2] - P0[2] * P1[1];
    const float cr1 = P0[2] * P1[0] - P0[0] * P1[2];
    const float cr2 = P0[0] * P1[1] - P0[1] * P1[0];
    const float sxx = pxx + 0.3f, syy = pyy + 0.3f;
    const float det = (cr0 * cr0 + cr1 * cr1 + cr2 * cr2) + 0.3f * (pxx + pyy) + 0.09f;
    if (det > 0.0f) {
      const float idet = 1.0f / det;
      const float ca = syy * idet, cb = -sxy * idet, cc = sxx * idet;
      const double mx = a.fx * tx / tz + a.cx;
      const double my = a.fy * ty / tz + a.cy;
      const float mid = 0.5f * (sxx + syy), hd = 0.5f * (sxx - syy);
      const float lmax = mid + sqrtf(hd * hd + sxy * sxy);
      const double r = 3.0 * (double)sqrtf(lmax);
      const double fx0 = floor((mx - r) * (1.0 / kTile)), fx1 = floor((mx + r) * (1.0 / kTile));
      const double fy0 = floor((my - r) * (1.0 / kTile)), fy1 = floor((my + r) * (1.0 / kTile));
      const int x0 = (int)fmax(fx0, 0.0), x1 = (int)fmin(fx1, (double)(a.TX - 1));
      const int y0 = (int)fmax(fy0, 0.0), y1 = (int)fmin(fy1, (double)(a.TY - 1));
      if (x0 <= x1 && y0 <= y1) {
        const int G = a.G;
        cnt = (uint32_t)((x1 / G - x0 / G + 1) * (y1 / G - y0 / G + 1));
        if (a.tight) {
          // entries of the tiles (groups) the alpha-cut ellipse meets; the binning walks the
          // same spans
          const TightEllipse el = tight_ellipse(mx, my, ca, cb, cc, opac, x0, x1, y0);
          cnt = 0;
          if (G == 1) {
            for (int ty = y0; ty <= y1; ++ty) {
              int lo, hi;
              tight_row_span(el, ty, &lo, &hi);
              cnt += (uint32_t)(hi - lo + 1);
            }
          } else {
            for (int gy = y0 / G; gy <= y1 / G; ++gy) cnt += tight_group_count(tight_group_row(el, G, gy, y1));
          }
        }
        rc = make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)(x1 + 1),
                          (unsigned short)(y1 + 1));
        // colour
        float dx = (float)px - a.campos[0], dy = (float)py - a.campos[1], dz = (float)pz - a.campos[2];
        const float di = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= di; dy *= di; dz *= di;
        // the Gaussian's coefficients are contiguous: only visible Gaussians fetch their lines
        float coef[NB * 3];
        const float *shg = a.sh + (int64_t)g * (NB * 3);
        if constexpr ((NB * 3) % 4 == 0) {
#pragma unroll
          for (int k = 0; k < NB * 3; k += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(shg + k);
            coef[k] = v.x; coef[k + 1] = v.y; coef[k + 2] = v.z; coef[k + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int k = 0; k < NB * 3; ++k) coef[k] = shg[k];
        }
        float b[16];
        sh_basis<DEG>(dx, dy, dz, b);
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          float acc = 0.0f;
#pragma unroll
          for (int k = 0; k < NB; ++k) acc = fmaf(coef[k * 3 + ch], b[k], acc);
          col[ch] = fmaxf(acc + 0.5f, 0.0f);
        }
        a.xy[g] = make_double2(mx, my);
        a.conic[g] = make_float4(ca, cb, cc, opac);
        a.rgb[g] = make_float4(col[0], col[1], col[2], tzf);
      }
    }
  }
  a.count[g] = cnt;
  a.rect[g] = rc;
  return cnt;
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_preprocess(PreArgs a) {
  __shared__ uint64_t sh[4];
  __shared__ uint32_t shv[4];
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t cnt = g < a.n ? preprocess_one<DEG>(a, g) : 0u;
  if (a.bsum) {   // the count scan's tile sums, so that it needs no reduce pass
    uint64_t tot;
    uint32_t totv;
    block_exclusive_scan<uint64_t>(cnt, sh, &tot);
    block_exclusive_scan<uint32_t>(cnt > 0 ? 1u : 0u, shv, &totv);
    if (threadIdx.x == 0) {
      a.bsum[blockIdx.x] = tot;
      a.bvis[blockIdx.x] = totv;
    }
  }
}

// ---- exclusive scan: u32 counts -> u64 offsets (n + 1 entries) ------------------
// Reduce-then-scan with no inter-workgroup waits: per-tile sums, then a down-sweep in which
// each workgroup adds up the sums of the tiles before its own (read from L2) and rescans its
// tile from that offset; the last tile also writes the grand totals.  Above kDirectTiles
// tiles that adding up would grow quadratically, so one workgroup first scans the tile sums
// in place (three launches).  Block scans use wave shuffles (one LDS exchange of the four
// wave totals).
// Optionally the values are gathered through an index list (v[i] = in[idx[i]]), the indices
// with v[i] > 0 are compacted in index order (the visible list), and n is read from device
// memory (the grid covers an upper bound).
// Items per thread: 4 for scans of up to 2^20 values (1,024-value tiles, so that small scans
// still spread over every CU), 16 above that.
constexpr int64_t kSmallScan = 1ll << 20;
template <int ITEMS>
constexpr int64_t scan_tile() { return (int64_t)kBlock * ITEMS; }

template <bool GATHER, int kScanItems>
__device__ __forceinline__ void load_items(const uint32_t *in, const uint32_t *idx, int64_t base, int64_t n,
                                           uint32_t *v) {
  if (!GATHER && base + kScanItems <= n && ((base & 3) == 0)) {
    const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
    for (int q = 0; q < kScanItems / 4; ++q) {
      const uint4 x = p[q];
      v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? (GATHER ? in[idx[base + i]] : in[base + i]) : 0u;
}

template <bool GATHER, bool COMPACT, int kScanItems>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *in, const uint32_t *idx, int64_t n_host,
                                                        const uint32_t *n_dev, uint64_t *bsum, uint32_t *bvis) {
  constexpr int64_t kScanTile = scan_tile<kScanItems>();
  __shared__ uint64_t sh[4];
  __shared__ uint32_t shv[4];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  load_items<GATHER, kScanItems>(in, idx, base, n, v);
  uint64_t s = 0;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    s += v[i];
    c += v[i] > 0;
  }
  uint64_t tot;
  block_exclusive_scan<uint64_t>(s, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
  if (COMPACT) {
    uint32_t totv;
    block_exclusive_scan<uint32_t>(c, shv, &totv);
    if (threadIdx.x == 0) bvis[blockIdx.x] = totv;
  }
}

constexpr int64_t kDirectTiles = 4096;

// one workgroup: exclusive scan of the tile sums in place
template <bool COMPACT>
__global__ __launch_bounds__(kBlock) void k_scan_top(uint64_t *bsum, uint32_t *bvis, int64_t nb) {
  __shared__ uint64_t sh[4];
  __shared__ uint32_t shv[4];
  uint64_t carry = 0;
  uint32_t carryv = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kBlock) {
    const int64_t i = b0 + threadIdx.x;
    uint64_t tot;
    const uint64_t ex = block_exclusive_scan<uint64_t>(i < nb ? bsum[i] : 0, sh, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
    if (COMPACT) {
      uint32_t totv;
      const uint32_t exv = block_exclusive_scan<uint32_t>(i < nb ? bvis[i] : 0u, shv, &totv);
      if (i < nb) bvis[i] = carryv + exv;
      carryv += totv;
    }
  }
}

// PREFIXED: bsum/bvis already hold each tile's exclusive offset (k_scan_top ran); otherwise
// they hold sums of `spt` consecutive groups per tile (spt = 1: the reduce pass's tile sums;
// more: the preprocess's 256-value sums)
template <bool GATHER, bool COMPACT, int kScanItems, bool PREFIXED>
__global__ __launch_bounds__(kBlock) void k_scan_down(const uint32_t *in, const uint32_t *idx, int64_t n_host,
                                                      const uint32_t *n_dev, const uint64_t *bsum,
                                                      const uint32_t *bvis, uint64_t *out, uint32_t *order,
                                                      uint32_t *nvis, int spt) {
  constexpr int64_t kScanTile = scan_tile<kScanItems>();
  __shared__ uint64_t sh[4];
  __shared__ uint32_t shv[4];
  const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
  if ((int64_t)blockIdx.x * kScanTile >= n) {
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) {   // empty scan: the totals are zero
      out[0] = 0;
      if (COMPACT) *nvis = 0;
    }
    return;
  }
  // offset of this tile: the sums of the tiles before it
  uint64_t pre_all = 0;
  uint32_t prev_all = 0;
  if (PREFIXED) {
    pre_all = bsum[blockIdx.x];
    if (COMPACT) prev_all = bvis[blockIdx.x];
  } else {
    uint64_t pre = 0;
    uint32_t prev = 0;
    for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x * spt; j += kBlock) {
      pre += bsum[j];
      if (COMPACT) prev += bvis[j];
    }
    block_exclusive_scan<uint64_t>(pre, sh, &pre_all);
    if (COMPACT) block_exclusive_scan<uint32_t>(prev, shv, &prev_all);
  }
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  load_items<GATHER, kScanItems>(in, idx, base, n, v);
  uint64_t s = 0;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    s += v[i];
    c += v[i] > 0;
  }
  uint64_t tot;
  uint64_t run = pre_all + block_exclusive_scan<uint64_t>(s, sh, &tot);
  uint32_t runv = 0, totv = 0;
  if (COMPACT) runv = prev_all + block_exclusive_scan<uint32_t>(c, shv, &totv);
  if (threadIdx.x == 0 && (int64_t)(blockIdx.x + 1) * kScanTile >= n) {   // the last tile: grand totals
    out[n] = pre_all + tot;
    if (COMPACT) *nvis = prev_all + totv;
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) {
      out[base + i] = run;
      if (COMPACT && v[i] > 0) order[runv++] = (uint32_t)(base + i);
    }
    run += v[i];
  }
}

template <bool GATHER, bool COMPACT, int ITEMS>
hipError_t scan_impl_t(const uint32_t *in, const uint32_t *idx, uint64_t *out, int64_t n, const uint32_t *n_dev,
                       uint32_t *order, uint32_t *nvis, void *tmp, bool presummed, hipStream_t st) {
  const int64_t nb = (n + scan_tile<ITEMS>() - 1) / scan_tile<ITEMS>();
  uint64_t *bsum = static_cast<uint64_t *>(tmp);
  if (presummed) {
    // the preprocess left one sum per 256 values (scan_presummed(n) holds)
    const int64_t n256 = (n + kBlock - 1) / kBlock;
    uint32_t *bv = reinterpret_cast<uint32_t *>(bsum + (n256 > 0 ? n256 : 1));
    hipLaunchKernelGGL((k_scan_down<GATHER, COMPACT, ITEMS, false>), dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kBlock),
                       0, st, in, idx, n, n_dev, bsum, bv, out, order, nvis, (int)(scan_tile<ITEMS>() / kBlock));
    return hipGetLastError();
  }
  uint32_t *bvis = reinterpret_cast<uint32_t *>(bsum + (nb > 0 ? nb : 1));
  if (nb > 0)
    hipLaunchKernelGGL((k_scan_reduce<GATHER, COMPACT, ITEMS>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, idx, n,
                       n_dev, bsum, bvis);
  if (nb > kDirectTiles) {
    hipLaunchKernelGGL((k_scan_top<COMPACT>), dim3(1), dim3(kBlock), 0, st, bsum, bvis, nb);
    hipLaunchKernelGGL((k_scan_down<GATHER, COMPACT, ITEMS, true>), dim3((unsigned)nb), dim3(kBlock), 0, st, in, idx,
                       n, n_dev, bsum, bvis, out, order, nvis, 1);
  } else {
    hipLaunchKernelGGL((k_scan_down<GATHER, COMPACT, ITEMS, false>), dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kBlock),
                       0, st, in, idx, n, n_dev, bsum, bvis, out, order, nvis, 1);
  }
  return hipGetLastError();
}

template <bool GATHER, bool COMPACT>
hipError_t scan_impl(const uint32_t *in, const uint32_t *idx, uint64_t *out, int64_t n, const uint32_t *n_dev,
                     uint32_t *order, uint32_t *nvis, void *tmp, hipStream_t st, bool presummed = false) {
  if (n <= kSmallScan)
    return scan_impl_t<GATHER, COMPACT, 4>(in, idx, out, n, n_dev, order, nvis, tmp, presummed, st);
  return scan_impl_t<GATHER, COMPACT, 16>(in, idx, out, n, n_dev, order, nvis, tmp, presummed, st);
}

}  // namespace

bool scan_presummed(int64_t n) { return n > 0 && n <= kSmallScan; }

hipError_t launch_preprocess(const gs_scene &s, const gs_camera &c, const Grid &g, const gs_projected &o,
                             bool tight, void *scan_tmp, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  PreArgs a;
  a.n = s.n;
  a.mean = s.mean;
  a.log_scale = s.log_scale;
  a.quat = s.quat;
  a.opacity = s.opacity;
  a.sh = s.sh;
  for (int i = 0; i < 9; ++i) {
    a.R[i] = c.R[i];
    a.Rf[i] = c.R[i];
  }
  for (int i = 0; i < 3; ++i) a.t[i] = c.t[i];
  a.fx = c.fx; a.fy = c.fy; a.cx = c.cx; a.cy = c.cy; a.znear = c.znear;
  a.fxf = c.fx; a.fyf = c.fy;
  a.limx = (float)(1.3 * (0.5 * c.width) / (double)c.fx);
  a.limy = (float)(1.3 * (0.5 * c.height) / (double)c.fy);
  // camera centre -R^T t
  for (int i = 0; i < 3; ++i)
    a.campos[i] = (float)(-((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]));
  a.TX = g.TX; a.TY = g.TY; a.G = g.G;
  a.tight = tight ? 1 : 0;
  a.xy = reinterpret_cast<double2 *>(o.xy);
  a.conic = reinterpret_cast<float4 *>(o.conic);
  a.rgb = reinterpret_cast<float4 *>(o.rgb);
  a.rect = reinterpret_cast<ushort4 *>(o.rect);
  a.count = o.count;
  const unsigned blocks = (unsigned)((s.n + kBlock - 1) / kBlock);
  a.bsum = nullptr;
  a.bvis = nullptr;
  if (scan_tmp && scan_presummed(s.n)) {   // layout read by scan_impl_t (presummed)
    a.bsum = static_cast<uint64_t *>(scan_tmp);
    a.bvis = reinterpret_cast<uint32_t *>(a.bsum + blocks);
  }
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess<0>, dim3(blocks), dim3(kBlock), 0, st, a); break;
    case 1: hipLaunchKernelGGL(k_preprocess<1>, dim3(blocks), dim3(kBlock), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_preprocess<2>, dim3(blocks), dim3(kBlock), 0, st, a); break;
    case 3: hipLaunchKernelGGL(k_preprocess<3>, dim3(blocks), dim3(kBlock), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t scan_tmp_bytes(int64_t n) {
  // the most tile sums of any scan of at most n values
  const int64_t small = n < kSmallScan ? n : kSmallScan;
  int64_t nb = (small + scan_tile<4>() - 1) / scan_tile<4>();
  const int64_t nb_large = (n + scan_tile<16>() - 1) / scan_tile<16>();
  if (nb_large > nb) nb = nb_large;
  const int64_t n256 = (small + kBlock - 1) / kBlock;   // the preprocess's sums (scan_presummed)
  if (n256 > nb) nb = n256;
  return (size_t)((nb > 0 ? nb : 1) * (sizeof(uint64_t) + sizeof(uint32_t)) + 16);
}

hipError_t launch_scan_compact(const uint32_t *in, uint64_t *out, int64_t n, uint32_t *order, uint32_t *nvis,
                               void *tmp, bool presummed, hipStream_t st) {
  return scan_impl<false, true>(in, nullptr, out, n, nullptr, order, nvis, tmp, st, presummed && scan_presummed(n));
}

hipError_t launch_scan_gather(const uint32_t *in, const uint32_t *idx, uint64_t *out, int64_t n_max,
                              const uint32_t *n_dev, void *tmp, hipStream_t st) {
  return scan_impl<true, false>(in, idx, out, n_max, n_dev, nullptr, nullptr, tmp, st);
}

}  // namespace gsi
