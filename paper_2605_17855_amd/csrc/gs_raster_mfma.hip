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
// Grouping.  For G > 1 a chunk of the group's list is staged in LDS once; for every member
// tile the entries whose mask bit is set are compacted in order (ballot + mbcnt) and their
// A rows are built in that tile's frame.  Per-tile blending state lives in registers.  Each
// tile sees the same Gaussians in the same order with the same arithmetic as with G = 1, so
// grouped and ungrouped images are bit-identical.
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

template <int G, int S>
struct MfmaShared {
  static constexpr int NT = G * G;
  static constexpr int RS = (S == 3) ? 32 : 16;
  // one buffer where a workgroup has one tile (G = 1, and 4x4 and 8x8 groups split to one member
  // tile per workgroup: the chunk barrier orders each build after the last read); several
  // member tiles double-buffer, so one member tile's rows are built while another's are read
  static constexpr int NBUF = group_item_tiles(G) == 1 ? 1 : 2;
  __align__(16) uint16_t A[NBUF][kBlock * RS];
  float col[NBUF][3][kBlock];       // colour planes r, g, b of the staged rows
  double2 r0[G > 1 ? kBlock : 1];  // FP64 centre; every tile rounds its own offset
  float4 r1[G > 1 ? kBlock : 1];   // (a, b, c, ln o)
  float4 r2[G > 1 ? kBlock : 1];   // (r, g, b, -)
  __align__(16) uint32_t wcnt[2][NT][4];   // by chunk parity: a wave may stage chunk c+1 while
                                   // another still reads chunk c's counts
  uint32_t alive[2][4];
  uint8_t qm[NBUF][kBlock];        // quadrant masks of the staged rows
  uint8_t wl[4][kBlock];           // each wave's row list (wave-private)
  float4 wc[4][32];                // each wave's colours of its current block (wave-private)
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

// Renders work item `item` of job J (one workgroup): member tiles
// [part * G^2 / parts, (part + 1) * G^2 / parts) (row-major) of bin item / parts, part =
// item % parts.  Shared by the single-image and batched kernels.
template <int G, int PREC, int S, bool AUX>
__device__ __forceinline__ void raster_bin_mfma(const RasterJob &J, const RasterParams &P, int item,
                                                MfmaShared<G, S> &sm, short8 B0, short8 B1, short8 B20,
                                                short8 B21) {
  constexpr int NT = G * G;
  // member tiles per workgroup: all of them for G <= 2 (one workgroup per bin, the tile loops
  // below fully unrolled), group_item_tiles(G) for G >= 4 (J.parts workgroups per group)
  constexpr int NTW = group_item_tiles(G);
  constexpr bool SPLIT = NTW < NT;   // the group's member tiles over J.parts workgroups
  constexpr int RS = (S == 3) ? 32 : 16;
  constexpr int kTileUnroll = SPLIT ? 1 : NT;
  using TileMask = typename std::conditional<(NT > 32), uint64_t, uint32_t>::type;
  const int bin = SPLIT ? item / J.parts : item;
  const int k0 = SPLIT ? (item % J.parts) * NTW : 0;
  const int k1 = k0 + NTW;
  const int gx = bin % J.GX, gy = bin / J.GX;
  const int ox = gx * G * kTile, oy = gy * G * kTile;
  const uint32_t start = J.ranges[2 * bin], end = J.ranges[2 * bin + 1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int qx0 = (w & 1) * 8, qy0 = (w >> 1) * 8;
  const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);

  // the workgroup's member tiles k0 + i (G >= 4: private memory, one register copy per step)
  TileState st[NTW];
  TileMask alive_mask = 0;       // uniform: member tiles with pixels still blending (bit k)
  uint32_t rows_done[NTW];       // uniform: entries of each tile consumed so far
#pragma unroll kTileUnroll
  for (int i = 0; i < NTW; ++i) {
    const int k = k0 + i;
    const int tx0 = ox + (k % G) * kTile, ty0 = oy + (k / G) * kTile;
    const bool inside = (tx0 + px < J.W) && (ty0 + py < J.H);
    st[i].T = 1.0f; st[i].C0 = st[i].C1 = st[i].C2 = 0.0f; st[i].W = 0.0f;
    st[i].cut = inside ? kCutLog2 : INFINITY;
    st[i].nstop = 0; st[i].nblend = 0; st[i].last = 0;
    rows_done[i] = 0;
    if (tx0 < J.W && ty0 < J.H) alive_mask |= (TileMask)1 << k;
  }

  int it = 0;          // processing steps so far (LDS double-buffer parity)
  int cp = 0;          // chunk parity
  int last_k = -1;     // tile processed in the previous step, if its alive bits are pending
  for (uint32_t cs = start; cs < end && alive_mask; cs += kBlock) {
    const int cnt = (int)min((uint32_t)kBlock, end - cs);
    if (G == 1) {
      constexpr int buf = 0;
      if (it > 0) {
        // every wave is done with the previous chunk (single buffer) and has posted whether
        // its pixels are still blending
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
        build_row<PREC, S>(&sm.A[buf][t * RS], u, v, co.x, co.y, co.z, l2o);
        sm.col[buf][0][t] = cl.x;
        sm.col[buf][1][t] = cl.y;
        sm.col[buf][2][t] = cl.z;
        sm.qm[buf][t] = P.all_rows ? (uint8_t)0xF : (uint8_t)quad_mask(u, v, co.x, co.y, co.z, l2o);
      }
      __syncthreads();
      const int nw = wave_list(sm.qm[buf], cnt, sm.wl[w]);
      process_rows<PREC, S, AUX>(sm.A[buf], &sm.col[buf][0][0], sm.wl[w], nw, sm.wc[w], B0, B1, B20, B21, st[0],
                                 rows_done[0]);
      rows_done[0] += cnt;
      const uint64_t bal = __ballot(st[0].cut != INFINITY);
      if (lane == 0) sm.alive[it & 1][w] = bal != 0;
      ++it;
    } else {
      // stage the chunk once for every member tile (Algorithm 1: load the chunk into shared memory)
      TileMask mk = 0;
      if (t < cnt) {
        const uint32_t e = cs + t;
        mk = G == 8 ? (TileMask) static_cast<const uint64_t *>(J.masks)[e]
                    : (TileMask) static_cast<const uint16_t *>(J.masks)[e];
        // the records of entries that reach one of this workgroup's member tiles (the others'
        // rows are never built here)
        const TileMask mine = NTW == NT ? ~(TileMask)0 : (TileMask)(((TileMask)1 << NTW) - 1u) << k0;
        if (mk & mine) {
          const uint32_t g = J.vals[e];
          const double2 m = J.xy[g];
          const float4 co = J.conic[g];
          const float4 cl = J.rgb[g];
          sm.r0[t] = m;
          sm.r1[t] = make_float4(co.x, co.y, co.z, log2_opacity(co.w));
          sm.r2[t] = cl;
        }
      }
#pragma unroll kTileUnroll
      for (int k = k0; k < k1; ++k) {
        const uint64_t bk = __ballot((mk >> k) & 1u);
        if (lane == 0) sm.wcnt[cp][k][w] = (uint32_t)__popcll(bk);
      }
      __syncthreads();
      if (last_k >= 0) {
        const uint32_t any = sm.alive[(it - 1) & 1][0] | sm.alive[(it - 1) & 1][1] | sm.alive[(it - 1) & 1][2] |
                             sm.alive[(it - 1) & 1][3];
        if (!any) alive_mask &= ~((TileMask)1 << last_k);
        last_k = -1;
      }
      // G = 2: fully unrolled, all state in registers.  G = 4 and 8: one copy of the step for the
      // workgroup's member tiles (one tile: its state stays in registers)
#pragma unroll kTileUnroll
      for (int k = k0; k < k1; ++k) {
        const uint4 ck = *reinterpret_cast<const uint4 *>(sm.wcnt[cp][k]);
        const uint32_t nk = ck.x + ck.y + ck.z + ck.w;
        if (!((alive_mask >> k) & 1u) || nk == 0) continue;
        const int buf = MfmaShared<G, S>::NBUF == 1 ? 0 : (it & 1);
        // tile-frame origin in absolute pixels, exactly as the G = 1 path forms it
        const double fx0 = (double)(ox + (k % G) * kTile) + 8.5, fy0 = (double)(oy + (k / G) * kTile) + 8.5;
        const uint64_t bk = __ballot((mk >> k) & 1u);
        if ((mk >> k) & 1u) {
          const uint32_t woff = (w > 0 ? ck.x : 0u) + (w > 1 ? ck.y : 0u) + (w > 2 ? ck.z : 0u);
          const uint32_t pos =
              woff + __builtin_amdgcn_mbcnt_hi((uint32_t)(bk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bk, 0u));
          const double2 r0 = sm.r0[t];
          const float4 r1 = sm.r1[t];
          const float u = (float)(r0.x - fx0), v = (float)(r0.y - fy0);
          build_row<PREC, S>(&sm.A[buf][pos * RS], u, v, r1.x, r1.y, r1.z, r1.w);
          const float4 r2 = sm.r2[t];
          sm.col[buf][0][pos] = r2.x;
          sm.col[buf][1][pos] = r2.y;
          sm.col[buf][2][pos] = r2.z;
          sm.qm[buf][pos] = P.all_rows ? (uint8_t)0xF : (uint8_t)quad_mask(u, v, r1.x, r1.y, r1.z, r1.w);
        }
        __syncthreads();
        if (last_k >= 0) {
          const uint32_t any = sm.alive[(it - 1) & 1][0] | sm.alive[(it - 1) & 1][1] | sm.alive[(it - 1) & 1][2] |
                               sm.alive[(it - 1) & 1][3];
          if (!any) alive_mask &= ~((TileMask)1 << last_k);
        }
        TileState cur = st[k - k0];
        const int nw = wave_list(sm.qm[buf], (int)nk, sm.wl[w]);
        process_rows<PREC, S, AUX>(sm.A[buf], &sm.col[buf][0][0], sm.wl[w], nw, sm.wc[w], B0, B1, B20, B21, cur,
                                   rows_done[k - k0]);
        st[k - k0] = cur;
        rows_done[k - k0] += nk;
        const uint64_t ab = __ballot(cur.cut != INFINITY);
        if (lane == 0) sm.alive[it & 1][w] = ab != 0;
        last_k = k;
        ++it;
      }
      cp ^= 1;
    }
  }

  const int64_t HW = (int64_t)J.W * J.H;
#pragma unroll kTileUnroll
  for (int k = k0; k < k1; ++k) {
    const int xx = ox + (k % G) * kTile + px, yy = oy + (k / G) * kTile + py;
    if (xx >= J.W || yy >= J.H) continue;
    const int64_t pix = (int64_t)yy * J.W + xx;
    const TileState &sk = st[k - k0];
    J.image[pix] = sk.C0 + sk.T * P.bg[0];
    J.image[HW + pix] = sk.C1 + sk.T * P.bg[1];
    J.image[2 * HW + pix] = sk.C2 + sk.T * P.bg[2];
    if (AUX) {
      int plane = 0;
      if (P.aux_flags & GS_AUX_TFINAL) J.aux[(plane++) * HW + pix] = sk.T;
      if (P.aux_flags & GS_AUX_WSUM) J.aux[(plane++) * HW + pix] = sk.W;
      if (P.aux_flags & GS_AUX_NEVAL) {
        const bool stopped = sk.cut == INFINITY;
        J.aux[(plane++) * HW + pix] = (float)(stopped ? sk.nstop : rows_done[k - k0]);
      }
      if (P.aux_flags & GS_AUX_NBLEND) J.aux[(plane++) * HW + pix] = (float)sk.nblend;
      if (P.aux_flags & GS_AUX_LAST) J.aux[(plane++) * HW + pix] = (float)sk.last;
    }
  }
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
  using type = typename std::conditional<GF, MfmaGroupShared<S>, MfmaShared<G, S>>::type;
};

template <int G, int PREC, int S, bool AUX, bool GF, typename SM>
__device__ __forceinline__ void raster_item(const RasterJob &J, const RasterParams &P, int item, SM &sm, short8 B0,
                                            short8 B1, short8 B20, short8 B21) {
  if constexpr (GF)
    raster_bin_mfma_group<G, PREC, S, AUX>(J, P, item, sm);
  else
    raster_bin_mfma<G, PREC, S, AUX>(J, P, item, sm, B0, B1, B20, B21);
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
