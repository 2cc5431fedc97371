// Tensorized rasterizer: the Gaussian-pixel power as a dense MFMA contraction
// (paper: "Tensorizing the Power Computation", "Padding the Inner Dimension",
// "Warp-Level WMMA Mapping"; cross-tile grouping: "Grouped Rasterization with Shared
// Gaussian", Algorithm 1), re-designed for gfx950 wave64 and v_mfma_f32_32x32x16_{f16,bf16}.
//
// Power as a product.  In a tile-local frame with origin at the tile centre (pixel centre
// minus tile origin minus 8.5, so x, y are integers in [-8, 7]), for a Gaussian with centre
// (u, v) in that frame, conic [[a,b],[b,c]] and opacity o:
//   log2(o exp(power)) = k . phi,  phi = [x^2, xy, y^2, x, y, 1]
//   k = log2(e) [-a/2, -b, -c/2, a u + b v, b u + c v, ln o - (a u^2 + 2 b u v + c v^2)/2]
// which is exact in real arithmetic.  The paper's printed pixel-side basis holds
// Gaussian-dependent offsets; this separable form keeps the pixel side (B) constant for
// every tile and every Gaussian, so it lives in registers for the whole kernel.  phi entries
// are small integers, exact in FP16 and BF16.  The Gaussian side (A) is split into
// `splits` FP16/BF16 pieces hi + lo 2^-s (+ lo2 2^-2s) that occupy spare K slots of the
// 16-wide inner dimension against scaled copies of phi, so the precision lost to the 16-bit
// operands is won back at no extra MFMA (zero-padding of unused slots is exact).
//
// Mapping.  One 256-lane workgroup per bin; wave w owns the 8x8 quadrant (w&1, w>>1) of each
// member tile, as two 8x4 panels of 32 pixels.  For a block of 32 Gaussians (rows), one
// MFMA per panel gives D[32 Gaussians][32 pixels] = log2(alpha_raw).  Lane l holds
// D[8(j/4) + 4(l/32) + j%4][l%32] in register j; one v_permlane32_swap per register pair
// (panel-0 value, panel-1 value) leaves lane l < 32 with all 32 rows of panel-0 pixel l and
// lane l >= 32 with all 32 rows of panel-1 pixel l-32.  Each lane then runs the exact
// sequential front-to-back recurrence over those rows in depth order (VALU: exp2, 1/255
// cut as a compare on D, clamp, FP32 transmittance product, stop test, colour FMA).
// Rows are staged for the whole tile; each wave then runs only the rows whose alpha can reach
// the cut somewhere in its quadrant (quadrant culling, below), gathered from LDS by index.
//
// Grouping.  2x2 groups build each entry's row once, in the frame of the group, for all
// their member tiles (below).  Larger groups (and 2x2 with per-tile rows) give each member
// tile a workgroup that walks the group's list: the entries whose mask bit is set are
// compacted in order (ballot + mbcnt) and their A rows built in that tile's frame, so each
// tile sees the same Gaussians in the same order with the same arithmetic as with G = 1 and
// those images are bit-identical to ungrouped ones.
#include <type_traits>

#include "gs_mfma.hpp"

namespace gsi {
namespace {

using namespace mfma;
struct TileState {
  float T, C0, C1, C2, W, cut;
  uint32_t nstop, nblend, last;   // last: 1 + list position of the last blended Gaussian
};

// Runs the rows wl[0, n) of buffer A/col (ascending indices) for one member tile.  Rows are
// gathered from LDS by index; the slots past n in the last block take a row whose D is -1000
// at every pixel, so they never pass the cut.  The block's 32 colours (and row indices) are
// copied to the wave's own buffer wc, so the blend reads them at fixed offsets.
// tpos (auxiliary outputs of the grouped kernel only): position of each staged row in the
// member tile's own list, within the chunk; without it the row index is that position.
// CH: rows per staged chunk (the stride of the colour planes); IDX: the row index type.
template <int PREC, int S, bool AUX, int CH = kBlock, typename IDX = uint8_t>
__device__ __forceinline__ void process_rows(const uint16_t *sA, const float *scol, const IDX *wl, int n,
                                             float4 *wc, short8 B0, short8 B1, short8 B20, short8 B21,
                                             TileState &st, uint32_t row_base, const IDX *tpos = nullptr) {
  using N = Narrow<PREC>;
  constexpr int RS = (S == 3) ? 32 : 16;
  const int lane = threadIdx.x & 63;
  const int nblk = (n + 31) >> 5;
  short8 pad = {}, zero = {};
  if (lane < 32) pad[5] = (short)N::enc(-1000.0f);
  for (int blk = 0; blk < nblk; ++blk) {
    // a wave whose 64 pixels have all stopped skips the rest of this tile's rows
    if (__ballot(st.cut != INFINITY) == 0) break;
    const int slot = 32 * blk + (lane & 31);
    const bool real = slot < n;
    const int ri = real ? (int)wl[slot] : 0;
    const uint16_t *rp = sA + (size_t)ri * RS + 8 * (lane >> 5);
    const short8 a = real ? *reinterpret_cast<const short8 *>(rp) : pad;
    const int rpos = (AUX && tpos) ? (int)tpos[ri] : ri;
    const float4 gc = make_float4(scol[ri], scol[CH + ri], scol[2 * CH + ri], __int_as_float(rpos));
    float16v z = {};
    float16v d0 = N::mma(a, B0, z);
    float16v d1 = N::mma(a, B1, z);
    if (S == 3) {
      const short8 a2 = real ? *reinterpret_cast<const short8 *>(rp + 16) : zero;
      d0 = N::mma(a2, B20, d0);
      d1 = N::mma(a2, B21, d1);
    }
    if (lane < 32) wc[lane] = gc;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float D[32];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      auto pr = __builtin_amdgcn_permlane32_swap(__float_as_uint(d0[j]), __float_as_uint(d1[j]), false, false);
      D[8 * (j >> 2) + (j & 3)] = __uint_as_float(pr[0]);
      D[8 * (j >> 2) + 4 + (j & 3)] = __uint_as_float(pr[1]);
    }
#pragma unroll
    for (int m = 0; m < 32; ++m) {
      if (D[m] >= st.cut) {
#pragma clang fp contract(off)
        // weight alpha T, then T' = T (1 - alpha) as one FMA written over T (no copy of T
        // outlives the row).  A stop (T' < 1e-4) blends nothing, puts back T' + alpha T (T to
        // within a unit in the last place, at T ~ 1e-4) and disables the pixel; it comes at most
        // once per pixel, so the blend without the stop's selects runs whenever no active lane
        // stops on this row.  Every operation rounds as written (no contraction), so all
        // rasterizer variants blend bit for bit alike.
        const float4 cl = wc[m];
        const float al = fminf(kAlphaMax, __builtin_amdgcn_exp2f(D[m]));
        float wgt = al * st.T;
        st.T = fmaf(-st.T, al, st.T);
        if (__builtin_expect(__ballot(!(st.T >= kTMin)) != 0, 0)) {
          const bool ok = st.T >= kTMin;
          st.T = ok ? st.T : st.T + wgt;
          wgt = ok ? wgt : 0.0f;
          st.cut = ok ? st.cut : INFINITY;
          if (AUX) st.nstop = ok ? st.nstop : row_base + (uint32_t)__float_as_int(cl.w) + 1;
          if (AUX) st.nblend += ok ? 0u : ~0u;
        }
        st.C0 = fmaf(wgt, cl.x, st.C0);
        st.C1 = fmaf(wgt, cl.y, st.C1);
        st.C2 = fmaf(wgt, cl.z, st.C2);
        if (AUX) {
          st.W += wgt;
          st.nblend += 1u;
          st.last = wgt > 0.0f ? row_base + (uint32_t)__float_as_int(cl.w) + 1 : st.last;
        }
      }
    }
  }
}

// LDS of the 1x1-tile rasterizer: one chunk of kBlock rows (the chunk barrier orders each
// build after the last read).
template <int S>
struct MfmaShared {
  static constexpr int RS = (S == 3) ? 32 : 16;
  __align__(16) uint16_t A[kBlock * RS];
  float col[3][kBlock];            // colour planes r, g, b of the staged rows
  uint32_t alive[2][4];
  uint8_t qm[kBlock];              // quadrant masks of the staged rows
  uint8_t wl[4][kBlock];           // each wave's row list (wave-private)
  float4 wc[4][32];                // each wave's colours of its current block (wave-private)
};

// LDS of one member tile of a group with per-tile rows: a buffer of CAP rows that fills over
// several steps through the group's list before it is blended (448 rows keep the layout under
// 26 KB: six workgroups per CU).
template <int S>
struct MfmaTileShared {
  static constexpr int RS = (S == 3) ? 32 : 16;
  static constexpr int CAP = (S == 3) ? kBlock : 448;
  __align__(16) uint16_t A[CAP * RS];
  float col[3][CAP];
  __align__(16) uint32_t wcnt[2][4];   // this tile's entries per wave in a step, by step parity
  uint32_t alive[4];
  uint8_t qm[CAP];
  uint16_t wl[4][CAP];
  float4 wc[4][32];
};

// ---- grouped tiles with the Gaussian-side rows built once per group -----------------------
// Grouped rasterization with a shared Gaussian (Algorithm 1): a chunk of the group's list is
// staged once, and each entry's Gaussian-side row is built once, in the frame of the whole
// group (origin at the group's centre), for every member tile.  The member tiles differ only in
// the pixel-side operand: phi of the tile's pixels in the group frame.  This is done for 2x2
// groups (|x|, |y| <= 16: phi exact in FP16 and BF16); larger frames keep the per-tile rows
// below, because the terms of the power grow with the frame's size squared while the FP32
// accumulation and the split operands keep a fixed relative precision (a 4x4 frame measured
// ~1e-3 of image error against 1x1 tiles' ~5e-6).  Each wave then walks, per member tile, the rows
// whose quadrant mask has its bit (the entry's membership bit folded in), with no workgroup
// barrier between member tiles.  In exact arithmetic this is the per-tile power; in FP16/BF16
// the split operands now multiply larger phi entries, so the grouped image matches the
// ungrouped one to the operands' rounding (held to the oracle's tolerance) instead of bit for bit.
template <int G, int PREC>
struct GroupFrame {
  static constexpr bool value = G == 2;
};

template <int S>
struct MfmaGroupShared {
  static constexpr int RS = (S == 3) ? 32 : 16;
  static constexpr int NTP = 2;        // member tiles per workgroup: one row of a 2x2 group
  // member tiles blended side by side: both (eight waves, one per tile and quadrant) when a row
  // is one or two pieces; with three pieces, the registers of eight waves would leave two
  // workgroups per CU, so four waves walk the two tiles one after the other
  static constexpr int PAR = S == 3 ? 1 : 2;
  static constexpr int NW = 4 * PAR;   // waves
  static constexpr int CH = 64 * NW;   // entries per staged chunk, one per thread
  __align__(16) uint16_t A[CH * RS];
  float col[3][CH];
  uint16_t qm[CH];                 // bit 4 j + q: quadrant q of the workgroup's member tile j
  uint16_t tpos[NTP][CH];          // auxiliary outputs: row position in member tile j's list
  uint32_t wcnt[NTP][NW];
  uint32_t alive[2][NW];
  uint16_t wl[NW][CH];
  float4 wc[NW][32];
};

template <int G, int PREC, int S, bool AUX>
__device__ __forceinline__ void raster_bin_mfma_group(const RasterJob &J, const RasterParams &P, int item,
                                                      MfmaGroupShared<S> &sm) {
  // two workgroups per 2x2 group (J.parts == 2), each taking one row of member tiles (twice the
  // workgroups of one per group: the CUs balance them far better); wave w blends quadrant
  // w & 3 of member tile w >> 2 (eight waves), or of both member tiles in turn (four waves).
  // Both workgroups stage the group's chunk; each builds only the rows of entries that reach
  // one of its own tiles
  using SH = MfmaGroupShared<S>;
  constexpr int NTP = SH::NTP, NW = SH::NW, CH = SH::CH, PAR = SH::PAR, RS = SH::RS;
  constexpr int TPW = NTP / PAR;   // member tiles per wave
  static_assert(NTP == 2 && (PAR == 1 || PAR == 2), "two member tiles per workgroup");
  const int bin = item / 2;
  const int k0 = (item % 2) * NTP;   // first member tile of the workgroup
  const int gx = bin % J.GX, gy = bin / J.GX;
  const int ox = gx * G * kTile, oy = gy * G * kTile;
  const uint32_t start = J.ranges[2 * bin], end = J.ranges[2 * bin + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int q = w & 3;                          // this wave's quadrant
  const int j0 = PAR == 2 ? (w >> 2) : 0;       // its first member tile (of the workgroup)
  const int px = (q & 1) * 8 + (lane & 7), py = (q >> 1) * 8 + (lane >> 3);
  const double fx0 = (double)ox + 8.0 * G + 0.5, fy0 = (double)oy + 8.0 * G + 0.5;   // group frame origin

  // the wave's member tiles' blending state, in registers (named, not an array: a copy indexed
  // by the tile loop's counter would place it in private memory)
  TileState st0, st1;
  uint32_t rows_done[TPW];
  uint32_t alive_w = 0;            // uniform per wave: its tiles whose pixels still blend (bit i)
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int k = k0 + j0 + i;
    const int tx0 = ox + (k % G) * kTile, ty0 = oy + (k / G) * kTile;
    const bool inside = (tx0 + px < J.W) && (ty0 + py < J.H);
    TileState &si = i == 0 ? st0 : st1;   // (i is a constant in the unrolled loop)
    si.T = 1.0f; si.C0 = si.C1 = si.C2 = 0.0f; si.W = 0.0f;
    si.cut = inside ? kCutLog2 : INFINITY;
    si.nstop = 0; si.nblend = 0; si.last = 0;
    rows_done[i] = 0;
    if (__ballot(inside) != 0) alive_w |= 1u << i;
  }
  // pixel-side operand of the wave's quadrant in the group frame: fixed for a wave with one
  // member tile, made per tile step otherwise
  short8 B0, B1, B20, B21;
  if (TPW == 1) {
    const int k = k0 + j0;
    make_pixel_operand<PREC>(B0, B1, B20, B21, (k % G) * kTile - 8 * G + 8, (k / G) * kTile - 8 * G + 8);
  }

  int it = 0;
  for (uint32_t cs = start; cs < end; cs += CH) {
    const int cnt = (int)min((uint32_t)CH, end - cs);
    if (it > 0) {
      // every wave is done with the previous chunk and has posted whether it still blends
      __syncthreads();
      uint32_t any = 0;
#pragma unroll
      for (int v = 0; v < NW; ++v) any |= sm.alive[(it - 1) & 1][v];
      if (!any) break;
    }
    uint32_t mk = 0;
    if (t < cnt) mk = (uint32_t) static_cast<const uint16_t *>(J.masks)[cs + t];
    if (t < cnt && ((mk >> k0) & ((1u << NTP) - 1u)) == 0u) sm.qm[t] = 0;   // no tile of this workgroup
    else if (t < cnt) {
      const uint32_t e = cs + t;
      const uint32_t g = J.vals[e];
      const double2 m = J.xy[g];
      const float4 co = J.conic[g];
      const float4 cl = J.rgb[g];
      const float u = (float)(m.x - fx0), v = (float)(m.y - fy0);
      const float l2o = log2_opacity(co.w);
      build_row<PREC, S>(&sm.A[t * RS], u, v, co.x, co.y, co.z, l2o);
      sm.col[0][t] = cl.x;
      sm.col[1][t] = cl.y;
      sm.col[2][t] = cl.z;
      uint32_t qmask = 0;
#pragma unroll
      for (int jj = 0; jj < NTP; ++jj) {
        const int kk = k0 + jj;
        if ((mk >> kk) & 1u) {
          // the quadrant test in member tile kk's own frame
          const float ut = u + (float)(8 * G - 8 - (kk % G) * kTile), vt = v + (float)(8 * G - 8 - (kk / G) * kTile);
          qmask |= (P.all_rows ? 0xFu : quad_mask(ut, vt, co.x, co.y, co.z, l2o)) << (4 * jj);
        }
      }
      sm.qm[t] = (uint16_t)qmask;
    }
    if (AUX) {   // each wave counts each member tile's entries among its 64
#pragma unroll
      for (int jj = 0; jj < NTP; ++jj) {
        const uint64_t bk = __ballot((mk >> (k0 + jj)) & 1u);
        if (lane == 0) sm.wcnt[jj][w] = (uint32_t)__popcll(bk);
      }
    }
    __syncthreads();
    if (AUX) {
      // each row's position in every member tile's list (entries of the chunk with its bit)
#pragma unroll
      for (int jj = 0; jj < NTP; ++jj) {
        const uint64_t bk = __ballot((mk >> (k0 + jj)) & 1u);
        uint32_t woff = 0;
        for (int v = 0; v < w; ++v) woff += sm.wcnt[jj][v];
        sm.tpos[jj][t] = (uint16_t)(woff + __builtin_amdgcn_mbcnt_hi((uint32_t)(bk >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bk, 0u)));
      }
      __syncthreads();
    }
    // one copy of the tile step: the member tile's state is moved into registers for it
#pragma unroll 1
    for (int i = 0; i < TPW; ++i) {
      if (!((alive_w >> i) & 1u)) continue;
      const int j = j0 + i, k = k0 + j;
      if (TPW > 1)
        make_pixel_operand<PREC>(B0, B1, B20, B21, (k % G) * kTile - 8 * G + 8, (k / G) * kTile - 8 * G + 8);
      const int nw = wave_list_bit(sm.qm, cnt, 4 * j + q, sm.wl[w]);
      TileState cur;
      if (i == 0) cur = st0; else cur = st1;
      process_rows<PREC, S, AUX, CH, uint16_t>(sm.A, &sm.col[0][0], sm.wl[w], nw, sm.wc[w], B0, B1, B20, B21, cur,
                                               i == 0 ? rows_done[0] : rows_done[TPW - 1],
                                               AUX ? sm.tpos[j] : nullptr);
      if (i == 0) st0 = cur; else st1 = cur;
      if (__ballot(cur.cut != INFINITY) == 0) alive_w &= ~(1u << i);
    }
    if (AUX) {
#pragma unroll
      for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int v = 0; v < NW; ++v) rows_done[i] += sm.wcnt[j0 + i][v];
    }
    if (lane == 0) sm.alive[it & 1][w] = alive_w != 0;
    ++it;
  }

  const int64_t HW = (int64_t)J.W * J.H;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int k = k0 + j0 + i;
    const int xx = ox + (k % G) * kTile + px, yy = oy + (k / G) * kTile + py;
    if (xx >= J.W || yy >= J.H) continue;
    const int64_t pix = (int64_t)yy * J.W + xx;
    const TileState &si = i == 0 ? st0 : st1;
    J.image[pix] = si.C0 + si.T * P.bg[0];
    J.image[HW + pix] = si.C1 + si.T * P.bg[1];
    J.image[2 * HW + pix] = si.C2 + si.T * P.bg[2];
    if (AUX) {
      int plane = 0;
      if (P.aux_flags & GS_AUX_TFINAL) J.aux[(plane++) * HW + pix] = si.T;
      if (P.aux_flags & GS_AUX_WSUM) J.aux[(plane++) * HW + pix] = si.W;
      if (P.aux_flags & GS_AUX_NEVAL) {
        const bool stopped = si.cut == INFINITY;
        J.aux[(plane++) * HW + pix] = (float)(stopped ? si.nstop : rows_done[i]);
      }
      if (P.aux_flags & GS_AUX_NBLEND) J.aux[(plane++) * HW + pix] = (float)si.nblend;
      if (P.aux_flags & GS_AUX_LAST) J.aux[(plane++) * HW + pix] = (float)si.last;
    }
  }
}

// Writes pixel (xx, yy) (nothing past the image): colour over the background by the final
// transmittance and the auxiliary planes.  rows_done: the entries of the tile's list consumed.
template <bool AUX>
__device__ __forceinline__ void write_tile(const RasterJob &J, const RasterParams &P, int xx, int yy,
                                           const TileState &sk, uint32_t rows_done) {
  if (xx >= J.W || yy >= J.H) return;
  const int64_t HW = (int64_t)J.W * J.H;
  const int64_t pix = (int64_t)yy * J.W + xx;
  J.image[pix] = sk.C0 + sk.T * P.bg[0];
  J.image[HW + pix] = sk.C1 + sk.T * P.bg[1];
  J.image[2 * HW + pix] = sk.C2 + sk.T * P.bg[2];
  if (AUX) {
    int plane = 0;
    if (P.aux_flags & GS_AUX_TFINAL) J.aux[(plane++) * HW + pix] = sk.T;
    if (P.aux_flags & GS_AUX_WSUM) J.aux[(plane++) * HW + pix] = sk.W;
    if (P.aux_flags & GS_AUX_NEVAL) {
      const bool stopped = sk.cut == INFINITY;
      J.aux[(plane++) * HW + pix] = (float)(stopped ? sk.nstop : rows_done);
    }
    if (P.aux_flags & GS_AUX_NBLEND) J.aux[(plane++) * HW + pix] = (float)sk.nblend;
    if (P.aux_flags & GS_AUX_LAST) J.aux[(plane++) * HW + pix] = (float)sk.last;
  }
}

// Renders bin `bin` of job J (one workgroup, 1x1 tiles): the tile's list chunk by chunk.
template <int PREC, int S, bool AUX>
__device__ __forceinline__ void raster_bin_mfma(const RasterJob &J, const RasterParams &P, int bin, MfmaShared<S> &sm,
                                                short8 B0, short8 B1, short8 B20, short8 B21) {
  constexpr int RS = MfmaShared<S>::RS;
  const int ox = (bin % J.GX) * kTile, oy = (bin / J.GX) * kTile;
  const uint32_t start = J.ranges[2 * bin], end = J.ranges[2 * bin + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int px = (w & 1) * 8 + (lane & 7), py = (w >> 1) * 8 + (lane >> 3);
  TileState st;
  st.T = 1.0f; st.C0 = st.C1 = st.C2 = 0.0f; st.W = 0.0f;
  st.cut = (ox + px < J.W) && (oy + py < J.H) ? kCutLog2 : INFINITY;
  st.nstop = 0; st.nblend = 0; st.last = 0;
  uint32_t rows_done = 0;   // uniform: entries consumed so far
  int it = 0;
  for (uint32_t cs = start; cs < end; cs += kBlock) {
    const int cnt = (int)min((uint32_t)kBlock, end - cs);
    if (it > 0) {
      // every wave is done with the previous chunk (single buffer) and has posted whether its
      // pixels are still blending
      __syncthreads();
      const uint32_t any = sm.alive[(it - 1) & 1][0] | sm.alive[(it - 1) & 1][1] | sm.alive[(it - 1) & 1][2] |
                           sm.alive[(it - 1) & 1][3];
      if (!any) break;
    }
    if (t < cnt) {
      const uint32_t e = cs + t;
      const uint32_t g = J.vals[e];
      const double2 m = J.xy[g];
      const float4 co = J.conic[g];
      const float4 cl = J.rgb[g];
      const float u = (float)(m.x - ((double)ox + 8.5)), v = (float)(m.y - ((double)oy + 8.5));
      const float l2o = log2_opacity(co.w);
      build_row<PREC, S>(&sm.A[t * RS], u, v, co.x, co.y, co.z, l2o);
      sm.col[0][t] = cl.x;
      sm.col[1][t] = cl.y;
      sm.col[2][t] = cl.z;
      sm.qm[t] = P.all_rows ? (uint8_t)0xF : (uint8_t)quad_mask(u, v, co.x, co.y, co.z, l2o);
    }
    __syncthreads();
    const int nw = wave_list(sm.qm, cnt, sm.wl[w]);
    process_rows<PREC, S, AUX>(sm.A, &sm.col[0][0], sm.wl[w], nw, sm.wc[w], B0, B1, B20, B21, st, rows_done);
    rows_done += cnt;
    const uint64_t bal = __ballot(st.cut != INFINITY);
    if (lane == 0) sm.alive[it & 1][w] = bal != 0;
    ++it;
  }
  write_tile<AUX>(J, P, ox + px, oy + py, st, rows_done);
}

// Renders member tile item % parts (row-major in the group) of group item / parts, for groups
// whose rows are built per member tile (one workgroup per member tile).  The workgroup walks
// the group's list in steps of kBlock entries; in each step the entries whose mask holds its
// tile (compacted in list order by ballot) have their rows built in the tile's own frame and
// appended to the row buffer.  The buffer is blended once it could not take another step, and
// at the end, so MFMA blocks fill up across steps (a 4x4 or 8x8 tile takes only a share of its
// group's entries) and a step costs one barrier.  The tile sees the rows of its 1x1 list in
// the same order with the same arithmetic, so the image is bit-identical to 1x1 tiles.
template <int G, int PREC, int S, bool AUX>
__device__ __forceinline__ void raster_member_tile(const RasterJob &J, const RasterParams &P, int item,
                                                   MfmaTileShared<S> &sm, short8 B0, short8 B1, short8 B20,
                                                   short8 B21) {
  constexpr int RS = MfmaTileShared<S>::RS, CAP = MfmaTileShared<S>::CAP;
  const int bin = item / J.parts, k = item % J.parts;
  const int tx0 = ((bin % J.GX) * G + k % G) * kTile, ty0 = ((bin / J.GX) * G + k / G) * kTile;
  if (tx0 >= J.W || ty0 >= J.H) return;   // a member tile past the image (uniform)
  const uint32_t start = J.ranges[2 * bin], end = J.ranges[2 * bin + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int px = (w & 1) * 8 + (lane & 7), py = (w >> 1) * 8 + (lane >> 3);
  // tile-frame origin in absolute pixels, exactly as the 1x1 path forms it
  const double fx0 = (double)tx0 + 8.5, fy0 = (double)ty0 + 8.5;
  TileState st;
  st.T = 1.0f; st.C0 = st.C1 = st.C2 = 0.0f; st.W = 0.0f;
  st.cut = (tx0 + px < J.W) && (ty0 + py < J.H) ? kCutLog2 : INFINITY;
  st.nstop = 0; st.nblend = 0; st.last = 0;
  uint32_t rows_done = 0;   // uniform: rows of this tile blended so far (list position of buffer row 0)
  int filled = 0;           // uniform: rows in the buffer
  int cp = 0;
  bool live = true;
  auto blend = [&]() {
    const int nw = wave_list(sm.qm, filled, sm.wl[w]);
    process_rows<PREC, S, AUX, CAP, uint16_t>(sm.A, &sm.col[0][0], sm.wl[w], nw, sm.wc[w], B0, B1, B20, B21, st,
                                              rows_done);
    rows_done += (uint32_t)filled;
    filled = 0;
  };
  for (uint32_t cs = start; cs < end; cs += kBlock) {
    if (filled > CAP - kBlock) {
      // the rows of the earlier steps are in place; then every wave is done reading them and
      // has posted whether its pixels are still blending
      __syncthreads();
      blend();
      const uint64_t ab = __ballot(st.cut != INFINITY);
      if (lane == 0) sm.alive[w] = ab != 0;
      __syncthreads();
      if (!(sm.alive[0] | sm.alive[1] | sm.alive[2] | sm.alive[3])) {
        live = false;
        break;
      }
    }
    const int cnt = (int)min((uint32_t)kBlock, end - cs);
    bool mine = false;
    double2 m = make_double2(0.0, 0.0);
    float4 co = make_float4(0.0f, 0.0f, 0.0f, 0.0f), cl = co;
    if (t < cnt) {
      const uint32_t e = cs + t;
      const uint64_t mk = G == 8 ? static_cast<const uint64_t *>(J.masks)[e]
                                 : (uint64_t) static_cast<const uint16_t *>(J.masks)[e];
      mine = (mk >> k) & 1u;
      if (mine) {
        const uint32_t g = J.vals[e];
        m = J.xy[g];
        co = J.conic[g];
        cl = J.rgb[g];
      }
    }
    const uint64_t bk = __ballot(mine);
    if (lane == 0) sm.wcnt[cp][w] = (uint32_t)__popcll(bk);
    __syncthreads();
    const uint4 ck = *reinterpret_cast<const uint4 *>(sm.wcnt[cp]);
    if (mine) {
      const uint32_t woff = (w > 0 ? ck.x : 0u) + (w > 1 ? ck.y : 0u) + (w > 2 ? ck.z : 0u);
      const int pos = filled + (int)(woff + __builtin_amdgcn_mbcnt_hi((uint32_t)(bk >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bk, 0u)));
      const float u = (float)(m.x - fx0), v = (float)(m.y - fy0);
      const float l2o = log2_opacity(co.w);
      build_row<PREC, S>(&sm.A[pos * RS], u, v, co.x, co.y, co.z, l2o);
      sm.col[0][pos] = cl.x;
      sm.col[1][pos] = cl.y;
      sm.col[2][pos] = cl.z;
      sm.qm[pos] = P.all_rows ? (uint8_t)0xF : (uint8_t)quad_mask(u, v, co.x, co.y, co.z, l2o);
    }
    filled += (int)(ck.x + ck.y + ck.z + ck.w);
    cp ^= 1;
  }
  if (live && filled > 0) {
    __syncthreads();
    blend();
  }
  write_tile<AUX>(J, P, tx0 + px, ty0 + py, st, rows_done);
}

// Work item = workgroup id, mapped to bins in the XCD-aware order (4x4 blocks of neighbouring
// bins per XCD in turn, xcd_raster_bin) for one workgroup per bin; giving each XCD one
// contiguous band of tiles instead left the XCDs holding the dense bands running last (105 vs
// 87 us at 1080p / 1M Gaussians).  (Forcing 64 VGPRs for 8 waves per SIMD spilled to scratch and
// was slower than the 72 VGPRs here.)
// The LDS layout and the renderer of one work item: rows in the group frame where its pixel
// operand is exact, per-tile rows otherwise.
// GF: the group-frame path (only where GroupFrame holds; GS_OPT_TILE_ROWS selects the per-tile
// rows there as well, bit-identical to 1x1 tiles).
template <int G, int PREC, int S, bool GF>
struct SharedFor {
  using type = typename std::conditional<GF, MfmaGroupShared<S>,
                                         typename std::conditional<G == 1, MfmaShared<S>, MfmaTileShared<S>>::type>::type;
};

template <int G, int PREC, int S, bool AUX, bool GF, typename SM>
__device__ __forceinline__ void raster_item(const RasterJob &J, const RasterParams &P, int item, SM &sm, short8 B0,
                                            short8 B1, short8 B20, short8 B21) {
  if constexpr (GF)
    raster_bin_mfma_group<G, PREC, S, AUX>(J, P, item, sm);
  else if constexpr (G == 1)
    raster_bin_mfma<PREC, S, AUX>(J, P, item, sm, B0, B1, B20, B21);
  else
    raster_member_tile<G, PREC, S, AUX>(J, P, item, sm, B0, B1, B20, B21);
}

// threads per workgroup: those of the group-frame path's layout, else four waves
template <bool GF, int S>
struct RasterThreads {
  static constexpr int value = GF ? 64 * MfmaGroupShared<S>::NW : kBlock;
};

template <int G, int PREC, int S, bool AUX, bool GF>
__global__ __launch_bounds__((RasterThreads<GF, S>::value)) void k_raster_mfma(RasterJob J, RasterParams P) {
  __shared__ typename SharedFor<G, PREC, S, GF>::type sm;
  short8 B0, B1, B20, B21;
  make_pixel_operand<PREC>(B0, B1, B20, B21);
  // one workgroup per bin (parts == 1) in the XCD-aware order, else one per work item
  const int item = J.parts == 1 ? xcd_raster_bin((int)blockIdx.x, J.GX, J.GY) : (int)blockIdx.x;
  if (item < 0) return;
  raster_item<G, PREC, S, AUX, GF>(J, P, item, sm, B0, B1, B20, B21);
}

// Persistent batched rasterizer: workgroups take (job, item) work items from the counters
// (batch_items) until all `total` are done; job j owns items [jobs[j].bin0, jobs[j].bin0 +
// jobs[j].items).
template <int G, int PREC, int S, bool AUX, bool GF>
__global__ __launch_bounds__((RasterThreads<GF, S>::value)) void k_raster_mfma_batch(const BatchTable tb,
                                                              RasterParams P, uint32_t *counter) {
  __shared__ typename SharedFor<G, PREC, S, GF>::type sm;
  __shared__ int s_item;
  short8 B0, B1, B20, B21;
  make_pixel_operand<PREC>(B0, B1, B20, B21);
  batch_items(counter, tb.total, &s_item, [&](int item) {
    int lo = 0, hi = tb.n_jobs;   // last job with bin0 <= item
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tb.jobs[mid].bin0 <= item) lo = mid; else hi = mid;
    }
    const RasterJob J = tb.jobs[lo];
    raster_item<G, PREC, S, AUX, GF>(J, P, item - J.bin0, sm, B0, B1, B20, B21);
  });
}

struct BatchArgs {
  const BatchTable *table;
  int grid;
  uint32_t *counter;
};

template <int G, int PREC, int S, bool AUX, bool GF>
hipError_t launch_gf(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  constexpr int threads = RasterThreads<GF, S>::value;
  if (b) {
    hipLaunchKernelGGL((k_raster_mfma_batch<G, PREC, S, AUX, GF>), dim3((unsigned)b->grid), dim3(threads), 0, st,
                       *b->table, p, b->counter);
  } else {
    const unsigned grid = j.parts == 1 ? xcd_raster_grid(j.GX, j.GY) : (unsigned)j.items;
    hipLaunchKernelGGL((k_raster_mfma<G, PREC, S, AUX, GF>), dim3(grid), dim3(threads), 0, st, j, p);
  }
  return hipGetLastError();
}

template <int G, int PREC, int S, bool AUX>
hipError_t launch_t(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  if constexpr (GroupFrame<G, PREC>::value) {
    if (!p.tile_rows) return launch_gf<G, PREC, S, AUX, true>(j, p, b, st);
  }
  return launch_gf<G, PREC, S, AUX, false>(j, p, b, st);
}

template <int G, int PREC>
hipError_t launch_s(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  const bool aux = p.aux_flags != 0;
  switch (p.splits) {
    case 1: return aux ? launch_t<G, PREC, 1, true>(j, p, b, st) : launch_t<G, PREC, 1, false>(j, p, b, st);
    case 2: return aux ? launch_t<G, PREC, 2, true>(j, p, b, st) : launch_t<G, PREC, 2, false>(j, p, b, st);
    case 3:
      if (PREC == GS_PREC_FP16_MFMA) return hipErrorInvalidValue;
      return aux ? launch_t<G, PREC, 3, true>(j, p, b, st) : launch_t<G, PREC, 3, false>(j, p, b, st);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC>
hipError_t launch_p(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  switch (p.G) {
    case 1: return launch_s<1, PREC>(j, p, b, st);
    case 2: return launch_s<2, PREC>(j, p, b, st);
    case 4: return launch_s<4, PREC>(j, p, b, st);
    case 8: return launch_s<8, PREC>(j, p, b, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(const RasterJob &j, const RasterParams &p, const BatchArgs *b, hipStream_t st) {
  if (p.prec == GS_PREC_FP16_MFMA) return launch_p<GS_PREC_FP16_MFMA>(j, p, b, st);
  if (p.prec == GS_PREC_BF16_MFMA) return launch_p<GS_PREC_BF16_MFMA>(j, p, b, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_raster_mfma(const RasterJob &j, const RasterParams &p, hipStream_t st) {
  if (j.items == 0) return hipSuccess;
  return dispatch(j, p, nullptr, st);
}

hipError_t launch_raster_mfma_batch(const BatchTable &table, int grid, const RasterParams &p, uint32_t *counter,
                                    hipStream_t st) {
  if (table.total == 0) return hipSuccess;
  BatchArgs b{&table, grid, counter};
  RasterJob dummy{};
  return dispatch(dummy, p, &b, st);
}

}  // namespace gsi
