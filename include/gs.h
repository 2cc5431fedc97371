/*
 * gs.h -- C ABI of the MI355X (gfx950) tile-based 3D Gaussian Splatting renderer.
 *
 * The calls follow the paper's statement of the rendering problem (Background;
 * Algorithm 1 of the design section): Gaussians with a mean, a covariance given
 * by per-axis scale and a rotation quaternion, an opacity and spherical-harmonics
 * colour coefficients, plus a pinhole camera, go in; an RGB image comes out.
 * The four stages are:
 *   gs_preprocess  frustum culling and feature computation, count scan
 *                  (Background: "frustum culling", "feature computation");
 *   gs_bin_sort    duplicated (bin, depth) entries, depth sort, bin ranges
 *                  (Background: "Gaussian sorting"; grouped entries with a
 *                  tile-membership mask from the cross-tile grouping design);
 *   gs_rasterize   per-pixel front-to-back alpha blending with the 1/255 cut
 *                  and the 1e-4 transmittance stop (Background, eq. power_d,
 *                  eq. power; the tensorized power of the design section);
 *   gs_render      the three in order (Algorithm 1).
 *
 * Conventions that hold for every call:
 *   - Pointers are DEVICE memory unless a comment says host.  Structs passed by
 *     pointer are host memory.  The caller allocates and owns every buffer; the
 *     library never allocates, frees or retains a pointer after a call returns (the one
 *     exception is the device scratch array of gs_rasterize_batch_noalloc, which the
 *     library's code object holds on each GPU).
 *   - All device work is enqueued on `stream` (a hipStream_t passed as void*,
 *     NULL = the null stream).  gs_bin_sort and gs_render wait once on the host for
 *     the entry and visible counts (a bounded poll of gs_projected.host_counts, which
 *     the device writes, or a stream synchronization), unless GS_OPT_DEVICE_COUNTS is set.
 *     Every other call is asynchronous.
 *     An error return of gs_bin_sort or gs_render after work was enqueued first waits
 *     for that work, so the caller may reuse every buffer at once.
 *   - Errors are return codes.  Arguments are validated on the host before any
 *     HIP call; an invalid call returns GS_ERR_INVALID_ARG or GS_ERR_UNSUPPORTED
 *     and touches no memory.  A failing HIP call returns GS_ERR_HIP.  A message
 *     for the last error of the calling thread is in gs_last_error().
 *   - Identical inputs give bit-identical outputs.
 *   - Tiles are 16x16 pixels.  The tile grid is TX = ceil(W/16) by
 *     TY = ceil(H/16); tile id = ty*TX + tx.  With group side G, bins are GxG
 *     tile groups: GX = ceil(TX/G), GY = ceil(TY/G), bin id = gy*GX + gx; the
 *     mask bit of member tile (tx, ty) is (ty % G)*G + (tx % G).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = 1,   /* null pointer, negative size, bad enum value */
  GS_ERR_UNSUPPORTED = 2,   /* valid but outside the supported range (SH degree > 3, group not 1/2/4/8, W or H > 16384, n >= 2^31) */
  GS_ERR_CAPACITY = 3,      /* the entry count exceeds gs_bins.capacity; the required count is returned */
  GS_ERR_HIP = 4            /* a HIP runtime call failed; see gs_last_error() */
} gs_status;

typedef enum {
  GS_PREC_FP32 = 0,         /* scalar FP32 rasterizer (the plain form) */
  GS_PREC_FP16_MFMA = 1,    /* power as an FP16 MFMA contraction, FP32 accumulate */
  GS_PREC_BF16_MFMA = 2     /* power as a BF16 MFMA contraction, FP32 accumulate */
} gs_precision;

/* optional per-pixel outputs, written as consecutive H*W float planes in this order */
enum {
  GS_AUX_TFINAL = 1u,       /* transmittance left after the last blended Gaussian */
  GS_AUX_WSUM = 2u,         /* sum over blended Gaussians of alpha*T (so WSUM + TFINAL = 1) */
  GS_AUX_NEVAL = 4u,        /* Gaussians evaluated before the stop, as a float count */
  GS_AUX_NBLEND = 8u,       /* Gaussians blended (alpha >= 1/255, before the stop), as a float count */
  GS_AUX_LAST = 16u         /* end of the blended prefix: 1 + the position, in the pixel's tile list, of the last
                               Gaussian blended (0 if none), as a float; with GS_AUX_TFINAL it is the forward
                               state the MFMA backward pass starts from */
};

/* gs_options.flags */
enum {
  /* Opacity-aware tile culling (the tighter ellipse-tile intersection the paper's method is
   * combined with): a Gaussian is listed in a tile of its footprint square only while some
   * point of the rectangle spanned by the tile's pixel centres satisfies
   * q(p) = (p - mu')^T conic (p - mu') <= 2 ln(255 o) + 0.01, i.e. while its alpha can reach
   * the 1/255 cut there (the 0.01 margin covers FP32/FP16 rounding).  With GxG groups the
   * same test decides each member tile: a group entry holds the mask of the member tiles
   * that pass and exists only when one does.  Every dropped pair has alpha below the cut at
   * every pixel of the tile, so the image, T_final and the weight sum are those of the full
   * lists; entry counts and GS_AUX_NEVAL counts are smaller. */
  GS_OPT_TIGHT = 1u,
  /* The MFMA rasterizers leave out of each 8x8 quadrant's MFMA blocks the rows whose alpha
   * cannot reach the 1/255 cut at any pixel centre of that quadrant (the test is taken with a
   * margin of 1 in q, far above its own and the split operands' rounding, so the image and
   * every aux plane are those of the full rows).  This flag makes every quadrant run every row
   * of its tile, the plain tile loop; it exists to check that equality and changes no result. */
  GS_OPT_ALL_ROWS = 2u,
  /* Grouped MFMA rasterization (group > 1).  By default 2x2 groups build each entry's
   * Gaussian-side row once, in the frame of the whole group, for all its member tiles (the tiles
   * then differ only in the pixel-side operand); the image equals the 1x1 one in exact
   * arithmetic and to the split operands' rounding in FP16/BF16.  Larger groups build the rows
   * of each member tile in its own frame (one workgroup per member tile walking the group's
   * list), which gives images bit-identical to group 1; this flag does the same for 2x2 groups. */
  GS_OPT_TILE_ROWS = 4u,
  /* gs_bin_sort and gs_render without the host wait: the kernels that follow the count scan read
   * the entry and visible counts from device memory, and their grids are sized for
   * bins->capacity entries (those past the count return at once), so the call only enqueues work
   * and can be captured into a HIP graph (every launch is a kernel; no copy, memset or wait).
   * *n_keys is not written (n_keys may be NULL).  The entry count K stays on the device, in
   * proj->offset[n].  If K exceeds bins->capacity (a capacity overflow) no entry is binned: every
   * range is (0, 0) and the image is the background; the caller checks proj->offset[n] <=
   * capacity once the stream has run and renders again with larger buffers.  Images and bins
   * equal those of the call with the host wait.  bins->capacity must be below 2^32. */
  GS_OPT_DEVICE_COUNTS = 8u
};

typedef struct {
  int32_t group;            /* tile-group side G: 1, 2, 4 or 8 (cross-tile grouping; 8 with the MFMA precisions only) */
  int32_t precision;        /* gs_precision */
  int32_t splits;           /* MFMA paths: 1..3 FP16/BF16 pieces per Gaussian coefficient (hi, lo, lo2) */
  float bg[3];              /* background colour added with the final transmittance */
  uint32_t aux_flags;       /* GS_AUX_* */
  uint32_t flags;           /* GS_OPT_* (other bits must be 0) */
} gs_options;

/* Pinhole camera.  World -> camera: p_cam = R p + t, x right, y down, z forward.
 * Pixel (i, j) is sampled at (i + 0.5, j + 0.5); p_cam projects to
 * (fx x/z + cx, fy y/z + cy).  Gaussians with z <= znear are culled. */
typedef struct {
  float R[9];               /* row-major */
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;    /* 1..16384 */
  float znear;              /* > 0 */
} gs_camera;

/* Scene, structure of arrays, FP32, all device pointers. */
typedef struct {
  int64_t n;                /* number of Gaussians, 0 <= n < 2^31 */
  int32_t sh_degree;        /* 0..3 */
  int32_t reserved;
  const float *mean;        /* 3 x n: x row, y row, z row */
  const float *log_scale;   /* 3 x n: log of the per-axis standard deviation */
  const float *quat;        /* 4 x n: (w, x, y, z) rows, normalised by the library */
  const float *opacity;     /* n, in (0, 1) */
  const float *sh;          /* n x (deg+1)^2 x 3: Gaussian, then basis index l*l + l + m, then channel.  Each
                               Gaussian's coefficients are contiguous, so culled ones cost no SH traffic;
                               16-byte aligned */
} gs_scene;

/* Per-Gaussian screen-space records written by gs_preprocess (n entries each;
 * culled Gaussians have count 0 and rect 0 and their other records are unspecified). */
typedef struct {
  double *xy;               /* n x 2: projected centre (x, y) in pixels (FP64) */
  float *conic;             /* n x 4: (a, b, c, opacity), inverse 2D covariance [[a,b],[b,c]] */
  float *rgb;               /* n x 4: (r, g, b, depth), colour from SH + 0.5 clamped at 0, camera-space z */
  uint16_t *rect;           /* n x 4: (x0, y0, x1, y1) half-open tile ranges */
  uint32_t *count;          /* n: number of bins overlapped (tiles for G = 1, groups otherwise) */
  uint64_t *offset;         /* n + 1: exclusive prefix sum of count; offset[n] = entry count */
  uint32_t *order;          /* n: the visible Gaussians (count > 0), first *n_visible entries valid;
                               index order after gs_preprocess, (depth, index) order after gs_bin_sort */
  uint32_t *n_visible;      /* 1: number of visible Gaussians */
  uint64_t *host_counts;    /* HOST memory, 2 values, or NULL: pinned memory the caller allocated with
                               hipHostMalloc (e.g. a pinned tensor), through which gs_bin_sort receives the
                               entry and visible counts from the device without a copy command; with NULL
                               they are copied from the workspace after a wait for the whole stream, which
                               also waits for the depth sort the pinned path overlaps with the host's wait */
} gs_projected;

/* Duplicated and sorted entries (capacity entries each) and per-bin ranges. */
typedef struct {
  uint64_t *keys;           /* (bin << 32) | float bits of depth; ascending after gs_bin_sort */
  uint32_t *vals;           /* Gaussian index of each entry */
  void *masks;              /* tile-membership mask of each entry: uint16_t for G = 2 and 4, uint64_t for G = 8
                               (used when group > 1, may be NULL for group 1) */
  uint64_t capacity;        /* entries the three arrays can hold */
  uint32_t *ranges;         /* n_bins x 2: [start, end) of each bin in the sorted arrays; (0, 0) if empty */
} gs_bins;

/* Number of bins of the camera's tile grid for group side G (0 on invalid input). */
int64_t gs_num_bins(const gs_camera *cam, int32_t group);

/* Workspace bytes gs_preprocess, gs_bin_sort and gs_render need for n Gaussians and
 * `capacity` entries (scan partials, sort double buffer, digit counts). */
size_t gs_workspace_bytes(int64_t n, uint64_t capacity, const gs_camera *cam, const gs_options *opt);

/* Frustum culling and feature computation (Background) plus the count scan.
 * Writes every field of *out; out->offset gets the exclusive prefix sum of out->count. */
gs_status gs_preprocess(const gs_scene *scene, const gs_camera *cam, const gs_options *opt,
                        const gs_projected *out, void *ws, size_t ws_bytes, void *stream);

/* Duplicated entries sorted by (bin, depth, Gaussian index) and bin ranges (Background:
 * "Gaussian sorting"; Algorithm 1's group-level entries when opt->group > 1).
 * Also sorts proj->order[0 .. visible count) by depth (ties by Gaussian index).
 * *n_keys (host) receives the entry count; the call waits once on the host, for that count.
 * If it exceeds bins->capacity nothing is written to *bins and GS_ERR_CAPACITY is returned
 * (proj->order may already be in depth order): grow the buffers and call again.
 * With GS_OPT_DEVICE_COUNTS the call does not wait and the overflow is found on the device
 * (see the flag). */
gs_status gs_bin_sort(const gs_projected *proj, int64_t n, const gs_camera *cam, const gs_options *opt,
                      const gs_bins *bins, uint64_t *n_keys, void *ws, size_t ws_bytes, void *stream);

/* Per-pixel front-to-back blending (Background, eq. power_d, eq. power; tensorized power
 * and grouped rasterization for the MFMA precisions).  image: 3 x H x W FP32 planes.
 * aux: one H x W FP32 plane per GS_AUX_* flag set, or NULL when no flag is set. */
gs_status gs_rasterize(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam,
                       const gs_options *opt, float *image, float *aux, void *stream);

/* gs_preprocess, gs_bin_sort and gs_rasterize in order on one stream (Algorithm 1). */
gs_status gs_render(const gs_scene *scene, const gs_camera *cam, const gs_options *opt,
                    const gs_projected *proj, const gs_bins *bins, float *image, float *aux,
                    uint64_t *n_keys, void *ws, size_t ws_bytes, void *stream);

/* Stable ascending LSD radix sort of (key, value) pairs on key bits [lo_bit, hi_bit).
 * Bits outside the range must be equal across keys for a full-key order.  In place;
 * ws must hold gs_sort_workspace_bytes(n) bytes. */
size_t gs_sort_workspace_bytes(uint64_t n);
gs_status gs_radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t n, int32_t lo_bit, int32_t hi_bit,
                            void *ws, size_t ws_bytes, void *stream);

/* One image of a batched rasterization (serving).  proj/bins point to host structs
 * describing device buffers that hold a finished gs_bin_sort result. */
typedef struct {
  const gs_projected *proj;
  const gs_bins *bins;
  gs_camera cam;
  float *image;             /* 3 x H x W */
  float *aux;               /* NULL or planes as in gs_rasterize */
} gs_job;

/* Rasterizes n_jobs images (at most gs_max_batch()) in one persistent launch: workgroups take
 * (job, bin) items from the work counters in `work_counter` (device memory of
 * GS_BATCH_COUNTER_BYTES bytes, cleared by the call; eight counters 64 bytes apart, each
 * serving an interleaved eighth of the items, so that claims do not all queue on one address)
 * until every bin of every job is done.  Each image is bit-identical to gs_rasterize of the same job alone
 * (the per-bin work does not depend on the launch).  All jobs share opt (group, precision,
 * splits, background, aux).  The job descriptions are copied into the launch, so `jobs` may be
 * reused when the call returns.  Serving: batches the ready requests of a request loop. */
#define GS_BATCH_COUNTER_BYTES 512
int32_t gs_max_batch(void);
gs_status gs_rasterize_batch(const gs_job *jobs, int32_t n_jobs, const gs_options *opt, uint32_t *work_counter,
                             void *stream);

/* Allocation-free variant of gs_rasterize_batch, for callers that cannot allocate device memory
 * or pass a workspace: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same jobs, options, validation and images as gs_rasterize_batch (the same kernels);
 * the work counter that gs_rasterize_batch takes from the caller lives instead in a library-owned
 * device array of GS_NOALLOC_SCRATCH_BYTES bytes, one per GPU, created with the library's code
 * object on that GPU and held until the process ends.  Its device address is looked up on the
 * first call on each device (with that device current); no call allocates or frees memory.
 * The counter is cleared by a kernel on `stream` before each launch (no memset).  Every call on
 * one GPU shares that GPU's array, so calls whose launches overlap on one GPU (different streams,
 * or threads) race on the counter and must be serialized by the caller.  n_jobs above
 * gs_max_batch() returns GS_ERR_UNSUPPORTED; the launch's work counters take
 * GS_BATCH_COUNTER_BYTES of the scratch bytes. */
#define GS_NOALLOC_SCRATCH_BYTES 512
gs_status gs_rasterize_batch_noalloc(const gs_job *jobs, int32_t n_jobs, const gs_options *opt, void *stream);

const char *gs_status_string(gs_status s);
const char *gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
