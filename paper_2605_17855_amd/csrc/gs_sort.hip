// Duplicated entries, LSD radix sort of 64-bit (bin | depth) keys, bin ranges and masks.
//
// Background ("Gaussian sorting"): every Gaussian emits one entry per overlapped tile and
// the entries of a tile are ordered by depth with a radix sort.  With cross-tile grouping
// (Grouped Rasterization, Algorithm 1) the entry is per overlapped group of GxG tiles and
// carries a tile-membership bit mask; entries are ordered by (group, depth).
//
// Key = (bin << 32) | bits(float depth): depths are positive, so their IEEE bits order as
// unsigned integers.  An LSD radix sort takes the low (depth) digits first.  Those digits
// are a property of the Gaussian, not of the entry, so their passes run on the visible
// Gaussians before duplication (V elements instead of K entries): the visible list is
// sorted stably by depth bits, entries are emitted in that order (one thread per entry,
// load-balanced over Gaussians of any footprint), and the remaining passes sort the
// entries stably on the bin digits.  The result is exactly the stable sort of the 64-bit
// keys of Gaussian-major emission, i.e. the order (bin, depth bits, Gaussian index).
//
// Each pass is three kernels without inter-workgroup waits: per-tile digit counts, one
// workgroup per digit scanning its row of tile counts (and writing the row total), and a
// stable scatter that derives the digit bases from the row totals and writes each digit's
// run through LDS so that lanes store consecutive addresses.  The depth sort takes the 31
// bits of a positive depth in four passes (8, 8, 8 and 7 bits); its last pass also counts,
// per tile and digit, the entries of the keys' Gaussians, so that its scatter writes each
// Gaussian's first entry in depth order (the offset scan the binning needs) next to the
// sorted keys.  (Three passes of up to 11 bits were measured slower: a 2,048-digit pass
// costs nearly two 256-digit ones.)
#include "gs_internal.hpp"

namespace gsi {
namespace {

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (; i < n; i += stride) p[i] = v;
}

// ---- radix sort --------------------------------------------------------------
// Workgroup tile: 4 waves x R rounds x 64 lanes.  Wave w owns the contiguous sub-tile
// [w*64R, (w+1)*64R) and walks it in rounds of 64 consecutive keys, so (wave, round, lane)
// order is input order and per-digit ranks are stable.  Sorts of up to 2^20 keys use R = 4
// (1,024-key tiles: the ~200K visible Gaussians of a 1M scene still give ~200 workgroups, and
// the per-pass digit scans stay short; 512-key tiles were 1.3 % slower end to end), larger
// ones R = 8 (2,048 keys).
constexpr int kDigits = 256;                   // digits of at most 8 bits
// A sort of more than kSmallSort keys on exactly 9 bits (the bins of 4x4 groups at 1080p, 8x8
// at 2160p) takes them in one pass of 512 digits: one pass over the entries instead of two
// (5 + 4 bits), its per-tile counts still 1 byte per key with 2,048-key tiles.
constexpr int kWideDigits = 512;
constexpr int kWideBits = 9;
constexpr int kDepthBits = 31;                 // a positive float's sign bit is zero
constexpr int kSmallR = 4;                      // sorts up to kSmallSort keys: 1,024-key tiles
constexpr int kLargeR = 8;                      // larger sorts: 2,048-key tiles
constexpr uint64_t kSmallSort = 1ull << 20;
template <int R>
struct SortTile {
  static constexpr int kRounds = R;
  static constexpr int kWaveTile = R * 64;
  static constexpr int kTile = 4 * kWaveTile;
};

// lanes of the wave holding the same digit as this lane (among lanes with valid keys)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int nbits) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Exclusive scan of v over the 256 threads of the workgroup (wave shuffles, one LDS
// exchange of the four wave totals); *total = the sum.  sh4 holds 4 values.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan_t(T v, T *sh4, T *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
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
__device__ __forceinline__ uint32_t block_exclusive_scan_u32(uint32_t v, uint32_t *sh4, uint32_t *total) {
  return block_exclusive_scan_t<uint32_t>(v, sh4, total);
}

// Per-tile digit counts: counts[d * tiles + tile].  Keys are loaded up front (8 in flight
// per lane) and counted with one LDS atomic each.
// n is *n_dev when n_dev is given (the grid then covers an upper bound and the surplus
// workgroups return at once), else n_host.
__device__ __forceinline__ uint64_t count_of(uint64_t n_host, const uint32_t *n_dev) {
  return n_dev ? (uint64_t)*n_dev : n_host;
}

// Weights of the depth sort's last pass: the entry count of each key's Gaussian
// (count[vals[i]]), summed per tile and digit into wcounts[d * tiles + tile] by the count
// kernel, scanned over the tiles of each digit into wprefix (64-bit) with the digit totals in
// wtotals.
struct DigitWeights {
  const uint32_t *vals;
  const uint32_t *count;
  uint32_t *wcounts;
  uint64_t *wprefix;
  uint64_t *wtotals;
};

template <typename KT, int R, int DIG, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_radix_count(const KT *keys, uint64_t n_host, const uint32_t *n_dev,
                                                        int shift, int nbits, uint32_t tiles_max, uint32_t *counts,
                                                        DigitWeights wt) {
  constexpr int kRounds = SortTile<R>::kRounds, kWaveTile = SortTile<R>::kWaveTile, kSortTile = SortTile<R>::kTile;
  __shared__ uint32_t h[DIG];
  __shared__ uint32_t hw[WEIGHTED ? DIG : 1];
  const uint64_t n = count_of(n_host, n_dev);
  const uint32_t tile = xcd_sort_tile(blockIdx.x, (n + kSortTile - 1) / kSortTile);
  if (tile == ~0u) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ndig = 1 << nbits;
  for (int d = t; d < ndig; d += kBlock) {
    h[d] = 0;
    if (WEIGHTED) hw[d] = 0;
  }
  const uint32_t dmask = (1u << nbits) - 1u;
  const uint64_t base = (uint64_t)tile * kSortTile + (uint64_t)w * kWaveTile;
  KT key[kRounds];
  uint32_t c[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane;
    key[r] = i < n ? keys[i] : (KT)0;
    c[r] = WEIGHTED && i < n ? wt.vals[i] : 0u;
  }
  if (WEIGHTED) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) c[r] = base + (uint64_t)r * 64 + lane < n ? wt.count[c[r]] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = base + (uint64_t)r * 64 + lane < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
    if (valid) {
      atomicAdd(&h[d], 1u);   // (cheaper than grouping equal digits per wave first)
      if (WEIGHTED) atomicAdd(&hw[d], c[r]);
    }
  }
  __syncthreads();
  for (int d = t; d < ndig; d += kBlock) {
    counts[(uint64_t)d * tiles_max + tile] = h[d];
    if (WEIGHTED) wt.wcounts[(uint64_t)d * tiles_max + tile] = hw[d];
  }
}

// One workgroup per digit d: counts[d][*] becomes the exclusive prefix over tiles (within the
// digit) and totals[d] the digit's total.
// With weights (wt.wcounts), the digit's row of weights likewise into wt.wprefix and wt.wtotals.
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t *counts, uint32_t tiles_max,
                                                             uint32_t *totals, uint64_t n_host, const uint32_t *n_dev,
                                                             uint32_t tile_size, DigitWeights wt) {
  __shared__ uint32_t sh[4];
  __shared__ uint64_t sh8[4];
  const int d = blockIdx.x, t = threadIdx.x;
  uint32_t *row = counts + (uint64_t)d * tiles_max;
  // tiles holding keys (the count kernel wrote no counts for the others)
  const uint64_t n = count_of(n_host, n_dev);
  const uint32_t tiles = (uint32_t)((n + tile_size - 1) / tile_size);
  const uint32_t per = (tiles + kBlock - 1) / kBlock;
  const uint32_t b0 = t * per;
  uint32_t s = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < tiles) s += row[b0 + i];
  uint32_t tot;
  uint32_t run = block_exclusive_scan_u32(s, sh, &tot);
  if (t == 0) totals[d] = tot;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < tiles) {
      const uint32_t c = row[b0 + i];
      row[b0 + i] = run;
      run += c;
    }
  if (wt.wcounts) {
    const uint32_t *wrow = wt.wcounts + (uint64_t)d * tiles_max;
    uint64_t *prow = wt.wprefix + (uint64_t)d * tiles_max;
    uint64_t ws = 0;
    for (uint32_t i = 0; i < per; ++i)
      if (b0 + i < tiles) ws += wrow[b0 + i];
    uint64_t wtot;
    uint64_t wrun = block_exclusive_scan_t<uint64_t>(ws, sh8, &wtot);
    if (t == 0) wt.wtotals[d] = wtot;
    for (uint32_t i = 0; i < per; ++i)
      if (b0 + i < tiles) {
        prow[b0 + i] = wrun;
        wrun += wrow[b0 + i];
      }
  }
}

// Stable scatter of one tile: ranks from per-wave digit counters; the tile's start for digit
// d is (keys with a smaller digit) + offsets[d][tile]; keys are placed in LDS in tile-local
// digit order and then stored so that consecutive lanes write consecutive addresses.
// Final placement of the bin sort's last pass (fin != nullptr): the value of each key is the
// rank of its Gaussian in depth order; instead of the rank the pass writes the Gaussian index
// order[rank] to vals and the 64-bit key (bin << 32) | dkeys[rank] to keys (the two V-sized
// arrays stay in cache), next to the sorted bin keys.
struct FinalOut {
  const uint32_t *order;   // visible Gaussians in depth order
  const uint32_t *dkeys;   // their depth bits
  uint32_t *vals;          // Gaussian index of each sorted entry
  uint64_t *keys;          // 64-bit key of each sorted entry
  uint32_t bin_mask;       // the bin bits of a sort key (above them: the member-tile rectangle)
};

// First entries of the depth sort's last pass (WEIGHTED): dpos[p] = the entries of the
// Gaussians before the p-th in depth order, i.e. the exclusive scan of their entry counts
// (dpos[n] = all entries), and first[b] = p for every block b of kFirstsBlock entries whose
// first entry is one of the p-th Gaussian's (b < nfirst).  The key's place among the entries
// is the digit's weight base (the weights of smaller digits, then of this digit in earlier
// tiles) plus the weights of the keys before it in its tile's run of the digit.
struct FirstEntries {
  uint64_t *dpos;
  uint32_t *first;
  uint64_t nfirst;
};

template <typename KT, int R, int DIG, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const KT *kin, const uint32_t *vin, KT *kout, uint32_t *vout,
                                                          uint64_t n_host, const uint32_t *n_dev, int shift, int nbits,
                                                          uint32_t tiles_max, const uint32_t *offsets,
                                                          const uint32_t *totals, FinalOut fin, DigitWeights wt,
                                                          FirstEntries fe) {
  constexpr int kRounds = SortTile<R>::kRounds, kWaveTile = SortTile<R>::kWaveTile, kSortTile = SortTile<R>::kTile;
  constexpr int M = DIG / kBlock;   // digits per thread in the digit-level scans
  static_assert(DIG % kBlock == 0, "digits in whole multiples of the workgroup");
  __shared__ uint32_t wcnt[4][DIG];
  __shared__ uint32_t bstart[DIG];
  __shared__ uint32_t gbase[DIG];
  __shared__ uint32_t sh4[4];
  __shared__ uint64_t sh8[4];
  __shared__ KT s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  __shared__ uint64_t gw[WEIGHTED ? DIG : 1];          // weight base of each digit in this tile
  __shared__ uint32_t s_w[WEIGHTED ? kSortTile : 1];   // key weights in tile-local sorted order
  __shared__ uint32_t s_wx[WEIGHTED ? kSortTile : 1];  // their exclusive scan
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const uint64_t n = count_of(n_host, n_dev);
  if (WEIGHTED && n == 0 && blockIdx.x == 0 && t == 0) fe.dpos[0] = 0;   // no keys: no entries
  const uint32_t tile = xcd_sort_tile(blockIdx.x, (n + kSortTile - 1) / kSortTile);
  if (tile == ~0u) return;
  const uint64_t tile0 = (uint64_t)tile * kSortTile;
  const int ndig = 1 << nbits;
  const uint32_t dmask = (1u << nbits) - 1u;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t base = tile0 + (uint64_t)w * kWaveTile;
  KT key[kRounds];
  uint32_t val[kRounds], pos[kRounds], dig[kRounds], kw[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane;
    key[r] = i < n ? kin[i] : (KT)0;
    val[r] = i < n ? vin[i] : 0u;
  }
  if (WEIGHTED) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) kw[r] = base + (uint64_t)r * 64 + lane < n ? wt.count[val[r]] : 0u;
  }
  // this thread's digits t*M .. t*M + M - 1: their totals, this tile's offsets within them and,
  // weighted, the same two of the weights
  uint32_t tot_d[M], off_d[M];
  uint64_t wtot_d[WEIGHTED ? M : 1], woff_d[WEIGHTED ? M : 1];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int d = t * M + j;
    tot_d[j] = d < ndig ? totals[d] : 0u;
    off_d[j] = d < ndig ? offsets[(uint64_t)d * tiles_max + tile] : 0u;
    if (WEIGHTED) {
      wtot_d[j] = d < ndig ? wt.wtotals[d] : 0ull;
      woff_d[j] = d < ndig ? wt.wprefix[(uint64_t)d * tiles_max + tile] : 0ull;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int d = t; d < ndig; d += kBlock) wcnt[k][d] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = base + (uint64_t)r * 64 + lane < n;
    const uint32_t d = (uint32_t)(key[r] >> shift) & dmask;
    dig[r] = d;
    const uint64_t peers = match_digit(d, valid, nbits);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t old = wcnt[w][d];
    pos[r] = old + rank;
    // every lane of the wave has read the counter before the group's first lane updates it,
    // and the update is visible to the whole wave before the next round reads (the counters
    // are written and read by lanes of this wave only; the fences order the LDS accesses
    // across the barrier for the compiler as well as the hardware)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid && rank == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  // per digit: tile-local start (scan over digits of the tile's counts) and global start
  // (scan over digits of the totals, plus this tile's offset within the digit)
  uint32_t c[M][4], loc = 0, gsum = 0;
  uint64_t wsum = 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int d = t * M + j;
#pragma unroll
    for (int k = 0; k < 4; ++k) c[j][k] = d < ndig ? wcnt[k][d] : 0u;
    loc += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    gsum += tot_d[j];
    if (WEIGHTED) wsum += wtot_d[j];
  }
  uint32_t all;
  uint32_t bs = block_exclusive_scan_u32(loc, sh4, &all);
  uint32_t gb = block_exclusive_scan_u32(gsum, sh4, &all);
  uint64_t wall = 0, wb = 0;
  if (WEIGHTED) wb = block_exclusive_scan_t<uint64_t>(wsum, sh8, &wall);
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int d = t * M + j;
    if (d < ndig) {
      bstart[d] = bs;
      gbase[d] = gb + off_d[j];
      wcnt[0][d] = bs;
      wcnt[1][d] = bs + c[j][0];
      wcnt[2][d] = bs + c[j][0] + c[j][1];
      wcnt[3][d] = bs + c[j][0] + c[j][1] + c[j][2];
      if (WEIGHTED) gw[d] = wb + woff_d[j];
    }
    bs += c[j][0] + c[j][1] + c[j][2] + c[j][3];
    gb += tot_d[j];
    if (WEIGHTED) wb += wtot_d[j];
  }
  if (WEIGHTED && tile == 0 && t == 0) fe.dpos[n] = wall;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane;
    if (i < n) {
      const uint32_t lp = wcnt[w][dig[r]] + pos[r];
      s_key[lp] = key[r];
      s_val[lp] = val[r];
      if (WEIGHTED) s_w[lp] = kw[r];
    }
  }
  __syncthreads();
  const uint32_t nvalid = (uint32_t)((n - tile0) < (uint64_t)kSortTile ? (n - tile0) : (uint64_t)kSortTile);
  if (WEIGHTED) {
    // exclusive scan of the weights in tile-local sorted order (R consecutive keys per thread;
    // 32 bits hold a tile's sum unless the frame has 2^32 entries, which the caller rejects)
    uint32_t x[kRounds], ssum = 0;
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      const uint32_t i = (uint32_t)t * kRounds + q;
      x[q] = i < nvalid ? s_w[i] : 0u;
      ssum += x[q];
    }
    uint32_t tall;
    uint32_t ex = block_exclusive_scan_u32(ssum, sh4, &tall);
#pragma unroll
    for (int q = 0; q < kRounds; ++q) {
      s_wx[t * kRounds + q] = ex;
      ex += x[q];
    }
    __syncthreads();
    for (uint32_t i = t; i < nvalid; i += kBlock) {
      const KT k = s_key[i];
      const uint32_t d = (uint32_t)(k >> shift) & dmask;
      const uint32_t p = gbase[d] + (i - bstart[d]);
      kout[p] = k;
      vout[p] = s_val[i];
      const uint64_t o = gw[d] + (s_wx[i] - s_wx[bstart[d]]);
      fe.dpos[p] = o;
      const uint64_t end = o + s_w[i];
      for (uint64_t bk = (o + kFirstsBlock - 1) / kFirstsBlock; bk * kFirstsBlock < end && bk < fe.nfirst; ++bk)
        fe.first[bk] = p;
    }
    return;
  }
  if (fin.vals) {
    // all gathers of the thread first, then the stores (several round trips in flight)
    uint32_t gi[kRounds], dk[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t i = (uint32_t)t + (uint32_t)r * kBlock;
      const uint32_t v = i < nvalid ? s_val[i] : 0u;
      gi[r] = i < nvalid ? fin.order[v] : 0u;
      dk[r] = i < nvalid ? fin.dkeys[v] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint32_t i = (uint32_t)t + (uint32_t)r * kBlock;
      if (i >= nvalid) break;
      const KT k = s_key[i];
      const uint32_t d = (uint32_t)(k >> shift) & dmask;
      const uint32_t p = gbase[d] + (i - bstart[d]);
      kout[p] = k;
      fin.vals[p] = gi[r];
      fin.keys[p] = ((uint64_t)((uint32_t)k & fin.bin_mask) << 32) | dk[r];
    }
    return;
  }
  for (uint32_t i = t; i < nvalid; i += kBlock) {
    const KT k = s_key[i];
    const uint32_t d = (uint32_t)(k >> shift) & dmask;
    kout[gbase[d] + (i - bstart[d])] = k;
    vout[gbase[d] + (i - bstart[d])] = s_val[i];
  }
}

// Depth keys of the visible Gaussians (key[i] = bits(depth of order[i]), i < *nvis), the entry
// and visible counts, and the first depth pass's per-tile digit counts (one workgroup per sort
// tile of R x 256 keys; counts[d * tiles + tile] for the digit bits [0, nbits0)).
template <int R>
__global__ __launch_bounds__(kBlock) void k_depth_keys(const uint32_t *order, const float4 *rgb, const uint32_t *nvis,
                                                       uint32_t *keys, const uint64_t *K, uint64_t *counts,
                                                       uint64_t *host_counts, uint64_t capacity, int nbits0,
                                                       uint32_t *dcounts, uint32_t tiles) {
  constexpr int kSortTile = SortTile<R>::kTile;
  __shared__ uint32_t h[kDigits];
  const uint32_t V = *nvis;
  if (blockIdx.x == 0 && threadIdx.x == 0) {   // the entry and visible counts, side by side
    const uint64_t k = *K;
    counts[0] = k;
    counts[1] = V;
    // the entry count of a bin sort that reads it on the device: 0 (nothing binned) on overflow
    reinterpret_cast<uint32_t *>(counts + 2)[0] = k <= capacity ? (uint32_t)k : 0u;
    if (host_counts) {     // the caller's pinned host memory, polled by the host
      host_counts[0] = k;
      host_counts[1] = V;
    }
  }
  // the tile order of the sort's own passes over the V keys
  const uint32_t tile = xcd_sort_tile(blockIdx.x, ((uint64_t)V + kSortTile - 1) / kSortTile);
  if (tile == ~0u) return;
  const uint64_t tile0 = (uint64_t)tile * kSortTile;
  const int ndig = 1 << nbits0;
  for (int d = threadIdx.x; d < ndig; d += kBlock) h[d] = 0;
  __syncthreads();
  const uint32_t dmask = (1u << nbits0) - 1u;
  uint32_t g[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = tile0 + (uint64_t)r * kBlock + threadIdx.x;
    g[r] = i < V ? order[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = tile0 + (uint64_t)r * kBlock + threadIdx.x;
    if (i < V) {
      const uint32_t k = __float_as_uint(rgb[g[r]].w);
      keys[i] = k;
      atomicAdd(&h[k & dmask], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < ndig; d += kBlock) dcounts[(uint64_t)d * tiles + tile] = h[d];
}

// ---- binning: one thread per entry -------------------------------------------
// dpos[i] = first entry of the i-th visible Gaussian in depth order (exclusive scan of its
// bin count; dpos[V] = K).  Every visible Gaussian owns at least one entry, so a workgroup's
// ITEMS consecutive entries span at most ITEMS consecutive Gaussians: the offset scan's block
// firsts (or a wave-wide search) give the first, the workgroup stages their offsets in LDS,
// and each entry finds its Gaussian by binary search there.

// Last Gaussian (local index) of the staged offsets s_pos[0..span] whose first entry is <= e
// (span <= ITEMS, s_pos[0] <= e < s_pos[span]), in a fixed number of steps: no data-dependent
// loop, so the searches of a thread's several entries interleave.
template <int ITEMS>
__device__ __forceinline__ uint32_t local_gaussian_fixed(const uint64_t *s_pos, uint32_t span, uint64_t e) {
  uint32_t lo = 0;
#pragma unroll
  for (uint32_t step = ITEMS / 2; step > 0; step >>= 1) {
    const uint32_t c = lo + step;
    const bool take = c <= span && s_pos[c <= span ? c : span] <= e;
    lo = take ? c : lo;
  }
  return lo;
}

// The bin ranges start empty (the ranges kernel writes the non-empty ones after the sort):
// every workgroup of the binning grid clears its grid-stride share.
__device__ __forceinline__ void clear_ranges(uint32_t *ranges, uint64_t nranges) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nranges; i += (uint64_t)gridDim.x * kBlock)
    ranges[i] = 0u;
}

// Member tiles of a group entry without culling: the rectangle of the footprint's tiles inside
// group (gx, gy), [x0, x1) x [y0, y1) in member-tile units.  The binning packs it (x0, x1 - 1,
// y0, y1 - 1 at 3 bits each) above the bin bits of the entry's sort key, which the bin passes
// carry along without sorting on them, so the ranges kernel expands it into the mask without
// gathering the Gaussian's rect again.
constexpr int kRectDescBits = 12;
__device__ __forceinline__ uint32_t rect_desc(ushort4 rc, int G, int gx, int gy) {
  const int x0 = max((int)rc.x - gx * G, 0), x1 = min((int)rc.z - gx * G, G);
  const int y0 = max((int)rc.y - gy * G, 0), y1 = min((int)rc.w - gy * G, G);
  return (uint32_t)x0 | (uint32_t)(x1 - 1) << 3 | (uint32_t)y0 << 6 | (uint32_t)(y1 - 1) << 9;
}
__device__ __forceinline__ uint64_t rect_desc_mask(uint32_t desc, int G) {
  const int x0 = desc & 7, x1 = (int)((desc >> 3) & 7) + 1, y0 = (desc >> 6) & 7, y1 = (int)((desc >> 9) & 7) + 1;
  const uint64_t row = ((1ull << (x1 - x0)) - 1ull) << x0;   // x1 - x0 <= G <= 8
  uint64_t m = 0;
  for (int ly = y0; ly < y1; ++ly) m |= row << (ly * G);
  return m;
}

// Stages the first-entry offsets of the Gaussians that own entries [e0, e0 + ITEMS) into
// s_pos[0..span] (s_pos[l] = dpos[first + l]) and, with s_g, their indices s_g[l] = order[first + l].
template <int ITEMS>
__device__ __forceinline__ void stage_block_gaussians(const uint64_t *dpos, const uint32_t *block_first, uint32_t nvis,
                                                      uint64_t e0, uint64_t *s_pos, uint32_t *s_first,
                                                      uint32_t *first, uint32_t *span,
                                                      const uint32_t *order = nullptr, uint32_t *s_g = nullptr) {
  const int t = threadIdx.x, lane = t & 63;
  if (block_first) {
    // recorded by the offset scan (e0 is a multiple of its 1,024-entry blocks)
    if (t == 0) *s_first = block_first[e0 / kFirstsBlock];
  } else if (t < 64) {
    // 64-ary search for the last Gaussian i with dpos[i] <= e0, over [lo, hi)
    uint32_t lo = 0, hi = nvis;
    while (hi - lo > 1) {
      const uint32_t step = (hi - lo + 63) / 64;
      const uint32_t probe = lo + (uint32_t)lane * step;
      const bool le = probe < hi && dpos[probe] <= e0;
      const uint64_t m = __ballot(le);
      // dpos increases, so the lanes with le set are 0..j; lane j's probe is the new lower bound
      const int j = 63 - __clzll(m);
      const uint32_t nlo = lo + (uint32_t)j * step;
      hi = (nlo + step < hi) ? nlo + step : hi;
      lo = nlo;
    }
    if (lane == 0) *s_first = lo;
  }
  __syncthreads();
  *first = *s_first;
  *span = (nvis - *first) < (uint32_t)ITEMS ? (nvis - *first) : (uint32_t)ITEMS;
  for (uint32_t i = t; i <= *span; i += kBlock) {
    s_pos[i] = dpos[*first + i];
    if (s_g && i < *span) s_g[i] = order[*first + i];
  }
  __syncthreads();
}

// The first radix pass's per-tile digit counts, taken where the keys are written (the binning
// workgroup covers exactly one sort tile, in the sort's XCD-aware tile order):
// counts[d * tiles + tile] for the digit bits [0, nbits0).
struct FirstCounts {
  uint32_t *counts;   // nullptr: no sort follows
  int nbits0;
  uint32_t tiles;
};

// One workgroup per sort tile of entries.  Each thread first finds the Gaussians of all its
// entries (LDS searches, interleaved), then gathers their rects (one round trip for all of
// them), then writes: the entry's Gaussian comes from the staged block, not from a gather per
// entry.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_binning(const uint32_t *order, const uint64_t *dpos,
                                                    const uint32_t *block_first, uint32_t nvis_host,
                                                    uint64_t K_host, const uint32_t *nvis_dev, const uint32_t *K_dev,
                                                    const ushort4 *rect, int G, int GX, int desc_shift,
                                                    uint32_t *bin_keys, uint32_t *vals, uint32_t *ranges,
                                                    uint64_t nranges, FirstCounts fc) {
  constexpr int NI = ITEMS / kBlock;
  __shared__ uint64_t s_pos[ITEMS + 1];
  __shared__ uint32_t s_g[ITEMS];
  __shared__ uint32_t s_first;
  __shared__ uint32_t h[kWideDigits];
  const uint32_t nvis = (uint32_t)count_of(nvis_host, nvis_dev);
  const uint64_t K = count_of(K_host, K_dev);
  const uint32_t tile = xcd_sort_tile(blockIdx.x, (K + ITEMS - 1) / ITEMS);
  const uint64_t e0 = (uint64_t)tile * ITEMS;
  clear_ranges(ranges, nranges);
  if (tile == ~0u) return;
  for (int d = threadIdx.x; d < kWideDigits; d += kBlock) h[d] = 0;
  uint32_t first, span;
  stage_block_gaussians<ITEMS>(dpos, block_first, nvis, e0, s_pos, &s_first, &first, &span, order, s_g);
  const uint32_t dmask = (1u << fc.nbits0) - 1u;
  uint32_t l[NI];
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    l[it] = e < K ? local_gaussian_fixed<ITEMS>(s_pos, span, e) : 0u;
  }
  ushort4 r[NI];
#pragma unroll
  for (int it = 0; it < NI; ++it) r[it] = rect[s_g[l[it]]];   // (l < span: a staged Gaussian)
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    if (e < K) {
      const uint32_t j = (uint32_t)(e - s_pos[l[it]]);
      const int gx0 = r[it].x / G, gx1 = (r[it].z - 1) / G, gy0 = r[it].y / G;
      const int wdt = gx1 - gx0 + 1;
      const int gy = gy0 + (int)(j / (uint32_t)wdt), gx = gx0 + (int)(j % (uint32_t)wdt);
      const uint32_t bin = (uint32_t)(gy * GX + gx);
      // (desc_shift > 0: group bins without culling, the member-tile rectangle above the bin bits)
      bin_keys[e] = desc_shift ? bin | rect_desc(r[it], G, gx, gy) << desc_shift : bin;
      vals[e] = first + l[it];   // the Gaussian's rank in depth order; the last sort pass turns it into its index
      if (fc.counts) atomicAdd(&h[bin & dmask], 1u);
    }
  }
  if (fc.counts) {
    __syncthreads();
    for (int d = threadIdx.x; d < (1 << fc.nbits0); d += kBlock) fc.counts[(uint64_t)d * fc.tiles + tile] = h[d];
  }
}

// Binning under opacity-aware culling: a Gaussian's entries follow its tile rows (group
// rows), each a span from tight_row_span (a union of group-column ranges); entry j walks the
// rows until its own.  (Measured on the 1M-Gaussian 1080p frame, this beat an LDS table of
// row spans built per workgroup: the span of a row is a few instructions, the table's
// dependent loads and prefix pass are not.)
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_binning_tight(const uint32_t *order, const uint64_t *dpos,
                                                          const uint32_t *block_first, uint32_t nvis_host,
                                                          uint64_t K_host, const uint32_t *nvis_dev,
                                                          const uint32_t *K_dev, const ushort4 *rect,
                                                          const double2 *xy, const float4 *conic, int TX, int G,
                                                          int GX, uint32_t *bin_keys, uint32_t *vals,
                                                          uint32_t *ranges, uint64_t nranges, FirstCounts fc) {
  __shared__ uint64_t s_pos[ITEMS + 1];
  __shared__ uint32_t s_g[ITEMS];
  __shared__ uint32_t s_first;
  __shared__ uint32_t h[kWideDigits];
  const uint32_t nvis = (uint32_t)count_of(nvis_host, nvis_dev);
  const uint64_t K = count_of(K_host, K_dev);
  const uint32_t tile = xcd_sort_tile(blockIdx.x, (K + ITEMS - 1) / ITEMS);
  const uint64_t e0 = (uint64_t)tile * ITEMS;
  const int lane = threadIdx.x & 63;
  clear_ranges(ranges, nranges);
  if (tile == ~0u) return;
  for (int d = threadIdx.x; d < kWideDigits; d += kBlock) h[d] = 0;
  uint32_t first, span;
  stage_block_gaussians<ITEMS>(dpos, block_first, nvis, e0, s_pos, &s_first, &first, &span, order, s_g);
  const uint32_t dmask = (1u << fc.nbits0) - 1u;
#pragma unroll
  for (int it = 0; it < ITEMS / kBlock; ++it) {
    const uint64_t e = e0 + (uint64_t)it * kBlock + threadIdx.x;
    const bool valid = e < K;
    if (__ballot(valid) == 0) continue;
    uint32_t rank = 0, g = 0, left = 0;
    if (valid) {
      const uint32_t l = local_gaussian_fixed<ITEMS>(s_pos, span, e);
      rank = first + l;
      g = s_g[l];
      left = (uint32_t)(e - s_pos[l]);
    }
    uint32_t bin = 0;   // (the walks always end early for counts from the preprocess)
    bool placed = false;
    // A wave whose entries all belong to one Gaussian (the large ones, where walking the rows
    // per entry costs most) shares the walk: lane k takes tile (group) row k, a wave prefix
    // sum of the row counts gives each row's first entry, and each lane finds its row by
    // bisection over those sums.  Same spans as the preprocess counted.
    const uint32_t g0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)g);
    if (__ballot(valid && g != g0) == 0) {
      const ushort4 r = rect[g0];
      const int row0 = r.y / G;
      const int R = (r.w - 1) / G - row0 + 1;   // tile rows (G = 1) or group rows
      if (R <= 64) {
        const double2 m = xy[g0];
        const float4 co = conic[g0];
        const TightEllipse el = tight_ellipse(m.x, m.y, co.x, co.y, co.z, co.w, r.x, r.z - 1, r.y);
        int lo = 0, hi = -1;
        uint32_t cnt = 0;
        if (lane < R) {
          if (G == 1) {
            tight_row_span(el, r.y + lane, &lo, &hi);
            cnt = (uint32_t)(hi - lo + 1);
          } else {
            cnt = tight_group_count(tight_group_row(el, G, row0 + lane, r.w - 1));
          }
        }
        uint32_t incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t u = __shfl_up(incl, off, 64);
          if (lane >= off) incl += u;
        }
        int pos = 0;   // rows whose entries all precede this lane's entry
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const uint32_t v = __shfl(incl, pos + step - 1, 64);
          if (v <= left) pos += step;
        }
        const uint32_t ip = __shfl(incl, pos, 64), cp = __shfl(cnt, pos, 64);
        const uint32_t within = left - (ip - cp);
        if (G == 1) {
          const int lop = __shfl(lo, pos, 64);
          bin = (uint32_t)((r.y + pos) * TX + lop) + within;
        } else if (valid) {
          const TightGroupRow row = tight_group_row(el, G, row0 + pos, r.w - 1);
          bin = (uint32_t)((row0 + pos) * GX + tight_group_nth(row, within));
        }
        placed = true;
      }
    }
    if (valid && !placed) {
      const ushort4 r = rect[g];
      const double2 m = xy[g];
      const float4 co = conic[g];
      const TightEllipse el = tight_ellipse(m.x, m.y, co.x, co.y, co.z, co.w, r.x, r.z - 1, r.y);
      if (G == 1) {
        for (int ty = r.y; ty < r.w; ++ty) {
          int lo, hi;
          tight_row_span(el, ty, &lo, &hi);
          const uint32_t cnt = (uint32_t)(hi - lo + 1);
          if (left < cnt) {
            bin = (uint32_t)(ty * TX + lo) + left;
            break;
          }
          left -= cnt;
        }
      } else {
        for (int gy = r.y / G; gy <= (r.w - 1) / G; ++gy) {
          const TightGroupRow row = tight_group_row(el, G, gy, r.w - 1);
          const uint32_t cnt = tight_group_count(row);
          if (left < cnt) {
            bin = (uint32_t)(gy * GX + tight_group_nth(row, left));
            break;
          }
          left -= cnt;
        }
      }
    }
    if (valid) {
      bin_keys[e] = bin;
      vals[e] = rank;   // the Gaussian's rank in depth order; the last sort pass turns it into its index
      if (fc.counts) atomicAdd(&h[bin & dmask], 1u);
    }
  }
  if (fc.counts) {
    __syncthreads();
    for (int d = threadIdx.x; d < (1 << fc.nbits0); d += kBlock) fc.counts[(uint64_t)d * fc.tiles + tile] = h[d];
  }
}

// Bin ranges (cleared beforehand), tile-membership masks and the 64-bit keys.  Entry i holds
// its Gaussian's rank r in the depth-sorted visible list; the Gaussian index order[r] and the
// depth bits dkeys[r] come from those two V-sized arrays (cache-resident), not from the
// per-Gaussian records.  A workgroup takes kRangeItems x 256 consecutive entries, thread t
// the entries t, t + 256, ... (coalesced), and issues all their loads before the dependent
// gathers, so several round trips are in flight at once.
constexpr int kRangeItems = 4;

__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t *bin_keys, const uint32_t *ranks, uint64_t n_host,
                                                   const uint32_t *n_dev, const uint32_t *order, const uint32_t *dkeys,
                                                   const ushort4 *rect, const double2 *xy, const float4 *conic,
                                                   int tight, int G, int GX, int desc_shift, uint32_t *vals,
                                                   uint32_t *ranges, void *masks, uint64_t *keys) {
  const uint64_t n = count_of(n_host, n_dev);
  const uint32_t bmask = desc_shift ? (1u << desc_shift) - 1u : ~0u;
  const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRangeItems + threadIdx.x;
  uint32_t bin[kRangeItems], prev[kRangeItems], next[kRangeItems], r[kRangeItems];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    const bool in = i < n;
    bin[j] = in ? bin_keys[i] : 0u;
    prev[j] = (in && i > 0) ? bin_keys[i - 1] & bmask : 0xFFFFFFFFu;
    next[j] = (in && i + 1 < n) ? bin_keys[i + 1] & bmask : 0xFFFFFFFFu;
    r[j] = in ? ranks[i] : 0u;
  }
  uint32_t g[kRangeItems], d[kRangeItems];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const bool in = base + (uint64_t)j * kBlock < n;
    g[j] = in ? order[r[j]] : 0u;
    d[j] = in ? dkeys[r[j]] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    if (i >= n) break;
    const uint32_t b = bin[j] & bmask;
    if (prev[j] != b) ranges[2 * (uint64_t)b] = (uint32_t)i;
    if (next[j] != b) ranges[2 * (uint64_t)b + 1] = (uint32_t)(i + 1);
    keys[i] = ((uint64_t)b << 32) | d[j];
    vals[i] = g[j];
    if (G > 1 && masks) {
      const ushort4 rc = rect[g[j]];
      const int gx = (int)(b % (uint32_t)GX), gy = (int)(b / (uint32_t)GX);
      uint64_t m = 0;
      if (desc_shift) {
        m = rect_desc_mask(bin[j] >> desc_shift, G);
      } else if (tight) {
        // member tiles the alpha-cut ellipse meets
        const double2 mu = xy[g[j]];
        const float4 co = conic[g[j]];
        const TightEllipse el = tight_ellipse(mu.x, mu.y, co.x, co.y, co.z, co.w, rc.x, rc.z - 1, rc.y);
        m = tight_group_mask(el, G, gx, gy, rc.w - 1);
      } else {
        // member tiles inside the footprint: a rectangle of rows [y0, y1) and columns [x0, x1)
        const int x0 = max((int)rc.x - gx * G, 0), x1 = min((int)rc.z - gx * G, G);
        const int y0 = max((int)rc.y - gy * G, 0), y1 = min((int)rc.w - gy * G, G);
        const uint64_t row = ((1ull << (x1 - x0)) - 1ull) << x0;   // x1 - x0 <= G <= 8
        for (int ly = y0; ly < y1; ++ly) m |= row << (ly * G);
      }
      if (G == 8) static_cast<uint64_t *>(masks)[i] = m;
      else static_cast<uint16_t *>(masks)[i] = (uint16_t)m;
    }
  }
}

// Bin ranges and (MASKS: group > 1) membership masks once the last bin pass has placed the
// final Gaussian indices and 64-bit keys: only the sorted bin keys are read for the ranges.
template <bool MASKS>
__global__ __launch_bounds__(kBlock) void k_ranges_final(const uint32_t *bin_keys, uint64_t n_host,
                                                         const uint32_t *n_dev, const uint32_t *vals,
                                                         const ushort4 *rect, const double2 *xy, const float4 *conic,
                                                         int tight, int G, int GX, int desc_shift, uint32_t *ranges,
                                                         void *masks) {
  const uint64_t n = count_of(n_host, n_dev);
  const uint32_t bmask = desc_shift ? (1u << desc_shift) - 1u : ~0u;
  const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRangeItems + threadIdx.x;
  uint32_t bin[kRangeItems], prev[kRangeItems], next[kRangeItems];
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    const bool in = i < n;
    bin[j] = in ? bin_keys[i] : 0u;
    prev[j] = (in && i > 0) ? bin_keys[i - 1] & bmask : 0xFFFFFFFFu;
    next[j] = (in && i + 1 < n) ? bin_keys[i + 1] & bmask : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint64_t i = base + (uint64_t)j * kBlock;
    if (i >= n) break;
    const uint32_t b = bin[j] & bmask;
    if (prev[j] != b) ranges[2 * (uint64_t)b] = (uint32_t)i;
    if (next[j] != b) ranges[2 * (uint64_t)b + 1] = (uint32_t)(i + 1);
    if (MASKS && desc_shift) {
      const uint64_t m = rect_desc_mask(bin[j] >> desc_shift, G);
      if (G == 8) static_cast<uint64_t *>(masks)[i] = m;
      else static_cast<uint16_t *>(masks)[i] = (uint16_t)m;
    } else if (MASKS) {
      const uint32_t g = vals[i];
      const ushort4 rc = rect[g];
      const int gx = (int)(b % (uint32_t)GX), gy = (int)(b / (uint32_t)GX);
      uint64_t m = 0;
      if (tight) {
        const double2 mu = xy[g];
        const float4 co = conic[g];
        const TightEllipse el = tight_ellipse(mu.x, mu.y, co.x, co.y, co.z, co.w, rc.x, rc.z - 1, rc.y);
        m = tight_group_mask(el, G, gx, gy, rc.w - 1);
      } else {
        const int x0 = max((int)rc.x - gx * G, 0), x1 = min((int)rc.z - gx * G, G);
        const int y0 = max((int)rc.y - gy * G, 0), y1 = min((int)rc.w - gy * G, G);
        const uint64_t row = ((1ull << (x1 - x0)) - 1ull) << x0;
        for (int ly = y0; ly < y1; ++ly) m |= row << (ly * G);
      }
      if (G == 8) static_cast<uint64_t *>(masks)[i] = m;
      else static_cast<uint16_t *>(masks)[i] = (uint16_t)m;
    }
  }
}

inline unsigned grid_for(uint64_t n, uint64_t per = kBlock) {
  const uint64_t b = (n + per - 1) / per;
  return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)b), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

// tiles of a sort of n keys, and the most tiles of any sort of at most n keys
inline uint64_t sort_tiles(uint64_t n) {
  return n <= kSmallSort ? (n + SortTile<kSmallR>::kTile - 1) / SortTile<kSmallR>::kTile
                         : (n + SortTile<kLargeR>::kTile - 1) / SortTile<kLargeR>::kTile;
}

// Digit width of the passes over key bits [lo, hi): passes of (nearly) equal width, at most
// maxw bits each (13 bits -> 7 + 6 and 32 -> 4 x 8 with 8; 31 -> 11 + 11 + 9 with 11).
constexpr int pass_width(int lo, int hi, int maxw = 8) {
  return (hi - lo + (hi - lo + maxw - 1) / maxw - 1) / ((hi - lo + maxw - 1) / maxw);
}

// first_counted: the per-tile digit counts of the first pass are already in tmp (written where
// the keys were produced).  fin: the last pass places final Gaussian indices and 64-bit keys.
template <typename KT, int R, int DIG>
hipError_t radix_passes_r(KT *keys, uint32_t *vals, KT *keys_alt, uint32_t *vals_alt, uint64_t n,
                          const uint32_t *n_dev, int lo, int hi, void *tmp, hipStream_t st, bool *in_alt,
                          const FinalOut *fin, bool first_counted) {
  const uint32_t tiles = (uint32_t)((n + SortTile<R>::kTile - 1) / SortTile<R>::kTile);
  uint32_t *counts = static_cast<uint32_t *>(tmp);
  uint32_t *totals = counts + (uint64_t)DIG * tiles;
  KT *kin = keys, *kout = keys_alt;
  uint32_t *vin = vals, *vout = vals_alt;
  const int width = DIG == kWideDigits ? kWideBits : pass_width(lo, hi);
  const FinalOut none{nullptr, nullptr, nullptr, nullptr};
  const DigitWeights now{nullptr, nullptr, nullptr, nullptr, nullptr};
  const FirstEntries nofe{nullptr, nullptr, 0};
  for (int shift = lo; shift < hi; shift += width) {
    const int bits = (hi - shift) < width ? (hi - shift) : width;
    const bool last = shift + width >= hi;
    if (!(first_counted && shift == lo))
      hipLaunchKernelGGL((k_radix_count<KT, R, DIG, false>), dim3(xcd_sort_grid(tiles)), dim3(kBlock), 0, st, kin,
                         n, n_dev, shift, bits, tiles, counts, now);
    hipLaunchKernelGGL(k_radix_digit_scan, dim3(1u << bits), dim3(kBlock), 0, st, counts, tiles, totals, n, n_dev,
                       (uint32_t)SortTile<R>::kTile, now);
    hipLaunchKernelGGL((k_radix_scatter<KT, R, DIG, false>), dim3(xcd_sort_grid(tiles)), dim3(kBlock), 0, st, kin,
                       vin, kout, vout, n, n_dev, shift, bits, tiles, counts, totals, (last && fin) ? *fin : none,
                       now, nofe);
    std::swap(kin, kout);
    std::swap(vin, vout);
    *in_alt = !*in_alt;
  }
  return hipGetLastError();
}

// n: the number of keys, or (with n_dev) an upper bound of *n_dev.
template <typename KT>
hipError_t radix_passes_t(KT *keys, uint32_t *vals, KT *keys_alt, uint32_t *vals_alt, uint64_t n,
                          const uint32_t *n_dev, int lo, int hi, void *tmp, hipStream_t st, bool *in_alt,
                          const FinalOut *fin = nullptr, bool first_counted = false) {
  *in_alt = false;
  if (hi <= lo || n <= 1) return hipSuccess;
  if (n <= kSmallSort)
    return radix_passes_r<KT, kSmallR, kDigits>(keys, vals, keys_alt, vals_alt, n, n_dev, lo, hi, tmp, st, in_alt,
                                                fin, first_counted);
  if (hi - lo == kWideBits)
    return radix_passes_r<KT, kLargeR, kWideDigits>(keys, vals, keys_alt, vals_alt, n, n_dev, lo, hi, tmp, st,
                                                    in_alt, fin, first_counted);
  return radix_passes_r<KT, kLargeR, kDigits>(keys, vals, keys_alt, vals_alt, n, n_dev, lo, hi, tmp, st, in_alt,
                                              fin, first_counted);
}

hipError_t radix_sort(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt, uint64_t n, int lo,
                      int hi, void *tmp, hipStream_t st, bool *in_alt) {
  return radix_passes_t<uint64_t>(keys, vals, keys_alt, vals_alt, n, nullptr, lo, hi, tmp, st, in_alt);
}

// ---- depth sort -----------------------------------------------------------------------
// Four passes over the 31 bits of a positive depth (8, 8, 8 and 7 bits), the last one weighted.
constexpr int kDepthWidth = pass_width(0, kDepthBits);
constexpr int kDepthPasses = (kDepthBits + kDepthWidth - 1) / kDepthWidth;
constexpr int kDepthLastBits = kDepthBits - (kDepthPasses - 1) * kDepthWidth;
constexpr int kDepthLastDigits = 1 << kDepthLastBits;
static_assert(kDepthWidth == 8 && kDepthPasses == 4 && kDepthLastBits == 7, "depth passes of 8, 8, 8 and 7 bits");

// Scratch of the depth sort over tiles sort tiles (the same for every pass): per-tile digit
// counts and digit totals, and the last pass's weights per tile and digit with their 64-bit
// scans and totals.
struct DepthTmp {
  uint64_t *wprefix;
  uint64_t *wtotals;
  uint32_t *counts;
  uint32_t *totals;
  uint32_t *wcounts;
  size_t bytes;
};
inline DepthTmp depth_tmp(void *tmp, uint64_t tiles) {
  DepthTmp d;
  char *p = static_cast<char *>(tmp);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *q = p ? p + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  const uint64_t t = tiles ? tiles : 1;
  d.wprefix = reinterpret_cast<uint64_t *>(take(kDepthLastDigits * t * 8));
  d.wtotals = reinterpret_cast<uint64_t *>(take(kDepthLastDigits * 8));
  d.counts = reinterpret_cast<uint32_t *>(take(kDigits * t * 4));
  d.totals = reinterpret_cast<uint32_t *>(take(kDigits * 4));
  d.wcounts = reinterpret_cast<uint32_t *>(take(kDepthLastDigits * t * 4));
  d.bytes = off;
  return d;
}

// Keys ping-pong between keys and keys_alt; values run order -> vals_alt -> vals_b ->
// vals_alt -> order, so that the sorted list ends where it started.
template <int R>
hipError_t depth_passes(uint32_t *order, const uint32_t *nvis, uint64_t n_max, uint32_t *keys, uint32_t *keys_alt,
                        uint32_t *vals_alt, uint32_t *vals_b, void *tmp, hipStream_t st, const uint32_t *count,
                        uint64_t *dpos, uint32_t *first, uint64_t nfirst) {
  const uint32_t tiles = (uint32_t)sort_tiles(n_max);
  const DepthTmp d = depth_tmp(tmp, tiles);
  const unsigned grid = xcd_sort_grid(tiles);
  const uint32_t tile_keys = (uint32_t)SortTile<R>::kTile;
  const FinalOut none{nullptr, nullptr, nullptr, nullptr};
  const DigitWeights now{nullptr, nullptr, nullptr, nullptr, nullptr};
  const FirstEntries nofe{nullptr, nullptr, 0};
  uint32_t *kbuf[2] = {keys, keys_alt};
  uint32_t *vbuf[kDepthPasses + 1];
  vbuf[0] = vbuf[kDepthPasses] = order;
  for (int p = 1; p < kDepthPasses; ++p) vbuf[p] = (p & 1) ? vals_alt : vals_b;
  for (int p = 0; p < kDepthPasses; ++p) {
    const int shift = p * kDepthWidth;
    uint32_t *kin = kbuf[p & 1], *kout = kbuf[(p + 1) & 1];
    if (p + 1 < kDepthPasses) {
      if (p > 0)   // the first pass was counted by k_depth_keys
        hipLaunchKernelGGL((k_radix_count<uint32_t, R, kDigits, false>), dim3(grid), dim3(kBlock), 0, st, kin, n_max,
                           nvis, shift, kDepthWidth, tiles, d.counts, now);
      hipLaunchKernelGGL(k_radix_digit_scan, dim3(1u << kDepthWidth), dim3(kBlock), 0, st, d.counts, tiles, d.totals,
                         n_max, nvis, tile_keys, now);
      hipLaunchKernelGGL((k_radix_scatter<uint32_t, R, kDigits, false>), dim3(grid), dim3(kBlock), 0, st, kin,
                         vbuf[p], kout, vbuf[p + 1], n_max, nvis, shift, kDepthWidth, tiles, d.counts, d.totals, none,
                         now, nofe);
    } else {
      // weighted by the Gaussians' entry counts, with the first entries and block firsts
      const DigitWeights wt{vbuf[p], count, d.wcounts, d.wprefix, d.wtotals};
      hipLaunchKernelGGL((k_radix_count<uint32_t, R, kDigits, true>), dim3(grid), dim3(kBlock), 0, st, kin, n_max,
                         nvis, shift, kDepthLastBits, tiles, d.counts, wt);
      hipLaunchKernelGGL(k_radix_digit_scan, dim3(1u << kDepthLastBits), dim3(kBlock), 0, st, d.counts, tiles,
                         d.totals, n_max, nvis, tile_keys, wt);
      hipLaunchKernelGGL((k_radix_scatter<uint32_t, R, kDigits, true>), dim3(grid), dim3(kBlock), 0, st, kin, vbuf[p],
                         kout, vbuf[p + 1], n_max, nvis, shift, kDepthLastBits, tiles, d.counts, d.totals, none, wt,
                         FirstEntries{dpos, first, nfirst});
    }
  }
  return hipGetLastError();
}

size_t radix_tmp_bytes(uint64_t n) {
  // the most digit counts of any sort of at most n keys: 256 per 1,024-key tile up to
  // kSmallSort keys, 512 per 2,048-key tile above (the same 1 count per 4 keys), and the totals
  uint64_t counts = (uint64_t)kDigits * sort_tiles(n < kSmallSort ? n : kSmallSort);
  if (n > kSmallSort && (uint64_t)kWideDigits * sort_tiles(n) > counts) counts = (uint64_t)kWideDigits * sort_tiles(n);
  return ((size_t)(counts ? counts : kDigits) + kWideDigits) * sizeof(uint32_t);
}

size_t depth_sort_tmp_bytes(uint64_t n) { return depth_tmp(nullptr, sort_tiles(n ? n : 1)).bytes; }

hipError_t launch_depth_keys(const uint32_t *order, const float4 *rgb, const uint32_t *nvis, uint64_t n_max,
                             uint32_t *keys, const uint64_t *K, uint64_t *counts, uint64_t *host_counts,
                             uint64_t capacity, void *tmp, hipStream_t st) {
  // one workgroup per tile of the depth sort that follows (sort_depth, same n_max): its first
  // pass's digit counts are taken here
  const uint32_t tiles = (uint32_t)sort_tiles(n_max ? n_max : 1);
  uint32_t *dcounts = depth_tmp(tmp, tiles).counts;
  if (n_max <= kSmallSort)
    hipLaunchKernelGGL((k_depth_keys<kSmallR>), dim3(xcd_sort_grid(tiles)), dim3(kBlock), 0, st, order, rgb, nvis, keys,
                       K, counts, host_counts, capacity, kDepthWidth, dcounts, tiles);
  else
    hipLaunchKernelGGL((k_depth_keys<kLargeR>), dim3(xcd_sort_grid(tiles)), dim3(kBlock), 0, st, order, rgb, nvis, keys,
                       K, counts, host_counts, capacity, kDepthWidth, dcounts, tiles);
  return hipGetLastError();
}

hipError_t sort_depth(uint32_t *order, const uint32_t *nvis, uint64_t n_max, uint32_t *keys, uint32_t *keys_alt,
                      uint32_t *vals_alt, uint32_t *vals_b, void *tmp, hipStream_t st, const uint32_t *count,
                      uint64_t *dpos, uint32_t *first, uint64_t nfirst) {
  if (n_max <= 1) return hipSuccess;
  if (n_max <= kSmallSort)
    return depth_passes<kSmallR>(order, nvis, n_max, keys, keys_alt, vals_alt, vals_b, tmp, st, count, dpos, first,
                                 nfirst);
  return depth_passes<kLargeR>(order, nvis, n_max, keys, keys_alt, vals_alt, vals_b, tmp, st, count, dpos, first,
                               nfirst);
}

hipError_t bin_and_sort(const uint32_t *order, const uint32_t *dkeys, const uint64_t *dpos, const uint32_t *block_first,
                        uint32_t V, uint64_t K, const uint32_t *V_dev, const uint32_t *K_dev,
                        const uint16_t *rect, const double *xy, const float *conic, bool tight, const Grid &g,
                        uint32_t *bkey, uint32_t *bval, uint32_t *bkey_alt, uint32_t *bval_alt, uint32_t *ranges,
                        void *masks, uint32_t *vals, uint64_t *keys, void *tmp, hipStream_t st) {
  const uint64_t nranges = 2 * (uint64_t)g.nbins;
  if (K == 0) return launch_fill_u32(ranges, nranges, 0u, st);
  const ushort4 *r4 = reinterpret_cast<const ushort4 *>(rect);
  const double2 *m2 = reinterpret_cast<const double2 *>(xy);
  const float4 *c4 = reinterpret_cast<const float4 *>(conic);
  const int hi = bits_for((uint64_t)g.nbins);
  // group bins without culling carry their member-tile rectangle above the bin bits (they fit:
  // at most 2^18 groups); culled groups' masks are computed from the Gaussians' records again
  const int desc_shift = (g.G > 1 && !tight && masks && hi + kRectDescBits <= 32) ? hi : 0;
  // with a sort to follow (K > 1), the binning takes its first pass's digit counts; with the
  // counts on the device, K is the bound that sizes the grids and picks the tile size, as the
  // sort's own passes do
  const bool large = K > kSmallSort;
  const unsigned tiles = grid_for(K, large ? SortTile<kLargeR>::kTile : SortTile<kSmallR>::kTile);
  const int nbits0 = (large && hi == kWideBits) ? kWideBits : pass_width(0, hi);   // as radix_passes_t splits [0, hi)
  const FirstCounts fc{K > 1 ? static_cast<uint32_t *>(tmp) : nullptr, nbits0, tiles};
  const unsigned grid = xcd_sort_grid(tiles);   // the sort's tile order (k_radix_scatter)
  if (tight) {
    if (large)
      hipLaunchKernelGGL((k_binning_tight<SortTile<kLargeR>::kTile>), dim3(grid), dim3(kBlock), 0, st, order, dpos,
                         block_first, V, K, V_dev, K_dev, r4, m2, c4, g.TX, g.G, g.GX, bkey, bval, ranges, nranges, fc);
    else
      hipLaunchKernelGGL((k_binning_tight<SortTile<kSmallR>::kTile>), dim3(grid), dim3(kBlock), 0, st, order, dpos,
                         block_first, V, K, V_dev, K_dev, r4, m2, c4, g.TX, g.G, g.GX, bkey, bval, ranges, nranges, fc);
  } else {
    if (large)
      hipLaunchKernelGGL((k_binning<SortTile<kLargeR>::kTile>), dim3(grid), dim3(kBlock), 0, st, order, dpos,
                         block_first, V, K, V_dev, K_dev, r4, g.G, g.GX, desc_shift, bkey, bval, ranges, nranges,
                         fc);
    else
      hipLaunchKernelGGL((k_binning<SortTile<kSmallR>::kTile>), dim3(grid), dim3(kBlock), 0, st, order, dpos,
                         block_first, V, K, V_dev, K_dev, r4, g.G, g.GX, desc_shift, bkey, bval, ranges, nranges,
                         fc);
  }
  if (K <= 1) {
    // nothing to sort: the single entry's index, key and range directly
    hipLaunchKernelGGL(k_ranges, dim3(1), dim3(kBlock), 0, st, bkey, bval, K, K_dev, order, dkeys, r4, m2, c4,
                       tight ? 1 : 0, g.G, g.GX, desc_shift, vals, ranges, masks, keys);
    return hipGetLastError();
  }
  bool in_alt = false;
  const FinalOut fin{order, dkeys, vals, keys, desc_shift ? (1u << desc_shift) - 1u : ~0u};
  // the bin passes ping-pong between (bkey, bval) and (bkey_alt, bval_alt); the last one writes
  // the final indices and 64-bit keys, and its sorted bin keys land in kf
  hipError_t e = radix_passes_t<uint32_t>(bkey, bval, bkey_alt, bval_alt, K, K_dev, 0, hi, tmp, st, &in_alt, &fin,
                                          true);
  if (e != hipSuccess) return e;
  const uint32_t *kf = in_alt ? bkey_alt : bkey;
  const dim3 rgrid(grid_for(K, (uint64_t)kBlock * kRangeItems));
  if (g.G > 1 && masks)
    hipLaunchKernelGGL(k_ranges_final<true>, rgrid, dim3(kBlock), 0, st, kf, K, K_dev, vals, r4, m2, c4, tight ? 1 : 0,
                       g.G, g.GX, desc_shift, ranges, masks);
  else
    hipLaunchKernelGGL(k_ranges_final<false>, rgrid, dim3(kBlock), 0, st, kf, K, K_dev, vals, r4, m2, c4,
                       tight ? 1 : 0, g.G, g.GX, desc_shift, ranges, masks);
  return hipGetLastError();
}

}  // namespace gsi
