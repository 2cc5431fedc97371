// Duplicated entries, LSD radix sort of 64-bit (bin | depth) keys, bin ranges and masks.
//
// Background ("Gaussian sorting"): every Gaussian emits one entry per overlapped tile and
// the entries of a tile are ordered by depth with a radix sort.  With cross-tile grouping
// (Grouped Rasterization, Algorithm 1) the entry is per overlapped group of GxG tiles and
// carries a tile-membership bit mask; entries are ordered by (group, depth).
//
// Key = (bin << 32) | bits(float depth): depths are positive, so their IEEE bits order as
// unsigned integers.  Entries are emitted Gaussian-major and the LSD passes are stable, so
// equal keys keep Gaussian-index order: the result equals a stable sort on (bin, depth, index).
#include "gs_internal.hpp"

namespace gsi {
namespace {

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_binning(int64_t n, const uint32_t *count, const uint64_t *offset,
                                                    const ushort4 *rect, const float4 *rgb, int G, int GX,
                                                    uint64_t capacity, uint64_t *keys, uint32_t *vals) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  const uint32_t c = count[g];
  if (c == 0) return;
  uint64_t o = offset[g];
  if (o + c > capacity) return;  // the host reports GS_ERR_CAPACITY
  const uint64_t dbits = __float_as_uint(rgb[g].w);
  const ushort4 r = rect[g];
  const int gx0 = r.x / G, gx1 = (r.z - 1) / G, gy0 = r.y / G, gy1 = (r.w - 1) / G;
  for (int gy = gy0; gy <= gy1; ++gy)
    for (int gx = gx0; gx <= gx1; ++gx) {
      keys[o] = ((uint64_t)(gy * GX + gx) << 32) | dbits;
      vals[o] = (uint32_t)g;
      ++o;
    }
}

// ---- radix sort --------------------------------------------------------------
// Workgroup tile: 4 waves x 8 rounds x 64 lanes = 2048 keys.  Wave w owns the contiguous
// sub-tile [w*512, (w+1)*512) and walks it in rounds of 64 consecutive keys, so
// (wave, round, lane) order is input order and per-digit ranks are stable.
constexpr int kRounds = 8;
constexpr int kWaveTile = kRounds * 64;
constexpr int kSortTile = 4 * kWaveTile;
constexpr int kDigits = 256;

__global__ __launch_bounds__(kBlock) void k_radix_count(const uint64_t *keys, uint64_t n, int shift, uint32_t dmask,
                                                        uint32_t nblocks, uint32_t *counts, uint32_t *ghist) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  static_assert(kSortTile % kBlock == 0, "tile is a whole number of workgroup strides");
#pragma unroll
  for (int r = 0; r < kSortTile / kBlock; ++r) {
    uint64_t i = base + (uint64_t)r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & dmask], 1u);
  }
  __syncthreads();
  const uint32_t v = h[threadIdx.x];
  counts[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = v;
  if (v) atomicAdd(&ghist[threadIdx.x], v);
}

// one workgroup per digit: offsets[d][b] = (keys with smaller digit) + (digit-d keys in blocks < b)
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t *counts, uint32_t nblocks,
                                                             const uint32_t *ghist) {
  __shared__ uint32_t sh[kBlock];
  __shared__ uint32_t sbase;
  const int d = blockIdx.x;
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int k = 0; k < d; ++k) b += ghist[k];
    sbase = b;
  }
  __syncthreads();
  uint32_t *row = counts + (uint64_t)d * nblocks;
  const uint32_t per = (nblocks + kBlock - 1) / kBlock;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nblocks) s += row[b0 + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    uint32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = sbase + sh[threadIdx.x] - s;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nblocks) {
      uint32_t c = row[b0 + i];
      row[b0 + i] = run;
      run += c;
    }
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                          uint32_t *vout, uint64_t n, int shift, uint32_t dmask,
                                                          uint32_t nblocks, const uint32_t *offsets) {
  __shared__ uint32_t wcnt[4][kDigits];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) wcnt[k][threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)w * kWaveTile;
  uint64_t key[kRounds];
  uint32_t val[kRounds], pos[kRounds], dig[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane;
    const bool valid = i < n;
    key[r] = valid ? kin[i] : 0ull;
    val[r] = valid ? vin[i] : 0u;
    const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
    dig[r] = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t old = wcnt[w][d];
    pos[r] = old + rank;
    // all lanes of the wave have read wcnt before the group's first lane updates it
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    const uint32_t c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d];
    const uint32_t g = offsets[(uint64_t)d * nblocks + blockIdx.x];
    __syncthreads();
    wcnt[0][d] = g;
    wcnt[1][d] = g + c0;
    wcnt[2][d] = g + c0 + c1;
    wcnt[3][d] = g + c0 + c1 + c2;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane;
    if (i < n) {
      const uint32_t dst = wcnt[w][dig[r]] + pos[r];
      kout[dst] = key[r];
      vout[dst] = val[r];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ranges(const uint64_t *keys, const uint32_t *vals, uint64_t n,
                                                   const ushort4 *rect, int G, int GX, uint32_t *ranges,
                                                   uint16_t *masks) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t bin = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != bin) ranges[2 * (uint64_t)bin] = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != bin) ranges[2 * (uint64_t)bin + 1] = (uint32_t)(i + 1);
  if (G > 1 && masks) {
    const ushort4 r = rect[vals[i]];
    const int gx = (int)(bin % (uint32_t)GX), gy = (int)(bin / (uint32_t)GX);
    uint32_t m = 0;
    for (int ly = 0; ly < G; ++ly)
      for (int lx = 0; lx < G; ++lx) {
        const int tx = gx * G + lx, ty = gy * G + ly;
        if (tx >= r.x && tx < r.z && ty >= r.y && ty < r.w) m |= 1u << (ly * G + lx);
      }
    masks[i] = (uint16_t)m;
  }
}

inline unsigned grid_for(uint64_t n) {
  uint64_t b = (n + kBlock - 1) / kBlock;
  return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t b = (n + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)b), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_binning(const gs_projected &p, int64_t n, const Grid &g, uint64_t capacity, uint64_t *keys,
                          uint32_t *vals, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_binning, dim3(grid_for((uint64_t)n)), dim3(kBlock), 0, st, n, p.count, p.offset,
                     reinterpret_cast<const ushort4 *>(p.rect), reinterpret_cast<const float4 *>(p.rgb), g.G,
                     g.GX, capacity, keys, vals);
  return hipGetLastError();
}

int radix_passes(int lo, int hi) { return hi > lo ? (hi - lo + 7) / 8 : 0; }

size_t sort_tmp_bytes(uint64_t n) {
  const uint64_t nblocks = (n + kSortTile - 1) / kSortTile;
  // digit counts (256 x nblocks) + one 256-bin global histogram per pass (at most 8 passes)
  return (size_t)(kDigits * (nblocks ? nblocks : 1) + 8 * kDigits) * sizeof(uint32_t);
}

hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n, int lo,
                      int hi, void *tmp, hipStream_t st, bool *in_alt) {
  *in_alt = false;
  if (n <= 1 || hi <= lo) return hipSuccess;
  const uint32_t nblocks = (uint32_t)((n + kSortTile - 1) / kSortTile);
  uint32_t *counts = static_cast<uint32_t *>(tmp);
  uint32_t *ghist = counts + (uint64_t)kDigits * nblocks;
  const int passes = radix_passes(lo, hi);
  hipError_t e = launch_fill_u32(ghist, (uint64_t)passes * kDigits, 0u, st);
  if (e != hipSuccess) return e;
  uint64_t *kin = keys, *kout = keys_alt;
  uint32_t *vin = vals, *vout = vals_alt;
  for (int p = 0; p < passes; ++p) {
    const int shift = lo + 8 * p;
    const int bits = (hi - shift) < 8 ? (hi - shift) : 8;
    const uint32_t dmask = (1u << bits) - 1u;
    uint32_t *gh = ghist + p * kDigits;
    hipLaunchKernelGGL(k_radix_count, dim3(nblocks), dim3(kBlock), 0, st, kin, n, shift, dmask, nblocks, counts, gh);
    hipLaunchKernelGGL(k_radix_digit_scan, dim3(kDigits), dim3(kBlock), 0, st, counts, nblocks, gh);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kBlock), 0, st, kin, vin, kout, vout, n, shift, dmask,
                       nblocks, counts);
    std::swap(kin, kout);
    std::swap(vin, vout);
    *in_alt = !*in_alt;
  }
  return hipGetLastError();
}

hipError_t launch_ranges(const uint64_t *keys, const uint32_t *vals, uint64_t n, const uint16_t *rect, const Grid &g,
                         uint32_t *ranges, uint16_t *masks, hipStream_t st) {
  hipError_t e = launch_fill_u32(ranges, (uint64_t)g.nbins * 2, 0u, st);
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(n)), dim3(kBlock), 0, st, keys, vals, n,
                     reinterpret_cast<const ushort4 *>(rect), g.G, g.GX, ranges, masks);
  return hipGetLastError();
}

}  // namespace gsi
