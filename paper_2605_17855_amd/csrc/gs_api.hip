// C ABI: argument validation (host only, before any HIP call), workspace layout and the
// order of the stages of one frame (Algorithm 1).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <chrono>
#include <mutex>

#include "gs_backward.hpp"
#include "gs_internal.hpp"

// Device scratch of gs_rasterize_batch_noalloc (see scratch_on_current_device below).
static __device__ __align__(256) uint32_t scratch[GS_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t)];

namespace {

thread_local char g_err[512] = "";

gs_status fail(gs_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

gs_status hip_fail(hipError_t e, const char *where) {
  return fail(GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define GS_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

gs_status check_camera(const gs_camera *c) {
  if (!c) return fail(GS_ERR_INVALID_ARG, "camera is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(GS_ERR_INVALID_ARG, "image size %dx%d", c->width, c->height);
  if (c->width > 16384 || c->height > 16384)
    return fail(GS_ERR_UNSUPPORTED, "image size %dx%d above 16384", c->width, c->height);
  if (!(c->fx > 0.0f) || !(c->fy > 0.0f) || !std::isfinite(c->fx) || !std::isfinite(c->fy))
    return fail(GS_ERR_INVALID_ARG, "focal lengths must be positive and finite");
  if (!(c->znear > 0.0f) || !std::isfinite(c->znear)) return fail(GS_ERR_INVALID_ARG, "znear must be positive");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(c->R[i])) return fail(GS_ERR_INVALID_ARG, "R has a non-finite entry");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(c->t[i])) return fail(GS_ERR_INVALID_ARG, "t has a non-finite entry");
  if (!std::isfinite(c->cx) || !std::isfinite(c->cy)) return fail(GS_ERR_INVALID_ARG, "principal point non-finite");
  return GS_OK;
}

gs_status check_options(const gs_options *o) {
  if (!o) return fail(GS_ERR_INVALID_ARG, "options is NULL");
  if (o->group < 1) return fail(GS_ERR_INVALID_ARG, "group %d", o->group);
  if (o->group != 1 && o->group != 2 && o->group != 4 && o->group != 8)
    return fail(GS_ERR_UNSUPPORTED, "group %d not in {1,2,4,8}", o->group);
  if (o->precision < GS_PREC_FP32 || o->precision > GS_PREC_BF16_MFMA)
    return fail(GS_ERR_INVALID_ARG, "precision %d", o->precision);
  if (o->precision != GS_PREC_FP32) {
    if (o->splits < 1 || o->splits > 3) return fail(GS_ERR_INVALID_ARG, "splits %d not in 1..3", o->splits);
    if (o->precision == GS_PREC_FP16_MFMA && o->splits == 3)
      return fail(GS_ERR_UNSUPPORTED, "FP16 supports splits 1..2 (a third FP16 piece would be subnormal)");
  } else if (o->group == 8) {
    return fail(GS_ERR_UNSUPPORTED, "group 8 needs an MFMA precision (the FP32 rasterizer keeps every member tile in registers)");
  }
  if (o->aux_flags & ~(uint32_t)(GS_AUX_TFINAL | GS_AUX_WSUM | GS_AUX_NEVAL | GS_AUX_NBLEND | GS_AUX_LAST))
    return fail(GS_ERR_INVALID_ARG, "aux_flags 0x%x", o->aux_flags);
  if (o->flags & ~(uint32_t)(GS_OPT_TIGHT | GS_OPT_ALL_ROWS | GS_OPT_TILE_ROWS | GS_OPT_DEVICE_COUNTS))
    return fail(GS_ERR_INVALID_ARG, "flags 0x%x", o->flags);
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(o->bg[i])) return fail(GS_ERR_INVALID_ARG, "background non-finite");
  return GS_OK;
}

gs_status check_scene(const gs_scene *s) {
  if (!s) return fail(GS_ERR_INVALID_ARG, "scene is NULL");
  if (s->n < 0) return fail(GS_ERR_INVALID_ARG, "n = %lld", (long long)s->n);
  if (s->n >= (1ll << 31)) return fail(GS_ERR_UNSUPPORTED, "n = %lld >= 2^31", (long long)s->n);
  if (s->sh_degree < 0) return fail(GS_ERR_INVALID_ARG, "sh_degree %d", s->sh_degree);
  if (s->sh_degree > 3) return fail(GS_ERR_UNSUPPORTED, "sh_degree %d > 3", s->sh_degree);
  if (s->n > 0 && (!s->mean || !s->log_scale || !s->quat || !s->opacity || !s->sh))
    return fail(GS_ERR_INVALID_ARG, "scene array is NULL");
  if (reinterpret_cast<uintptr_t>(s->sh) & 15u) return fail(GS_ERR_INVALID_ARG, "scene sh is not 16-byte aligned");
  return GS_OK;
}

gs_status check_projected(const gs_projected *p, int64_t n, bool need_records) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "projected is NULL");
  if (!p->offset || !p->n_visible) return fail(GS_ERR_INVALID_ARG, "projected.offset or n_visible is NULL");
  if (n > 0 && !p->order) return fail(GS_ERR_INVALID_ARG, "projected.order is NULL");
  if (n > 0 && (!p->count || !p->rect || (need_records && (!p->xy || !p->conic || !p->rgb))))
    return fail(GS_ERR_INVALID_ARG, "projected array is NULL");
  return GS_OK;
}

gs_status check_bins(const gs_bins *b, int group, bool need_keys) {
  if (!b) return fail(GS_ERR_INVALID_ARG, "bins is NULL");
  if (!b->ranges || !b->vals || (need_keys && !b->keys))
    return fail(GS_ERR_INVALID_ARG, "bins array is NULL");
  if (group > 1 && !b->masks) return fail(GS_ERR_INVALID_ARG, "bins.masks is NULL with group %d", group);
  return GS_OK;
}

// n_keys is required unless the counts stay on the device, whose 32-bit entry count needs a
// capacity below 2^32.
gs_status check_device_counts(const gs_options *o, const gs_bins *b, const uint64_t *n_keys) {
  if (!(o->flags & GS_OPT_DEVICE_COUNTS)) {
    if (!n_keys) return fail(GS_ERR_INVALID_ARG, "n_keys is NULL");
  } else if (b->capacity >= (1ull << 32)) {
    return fail(GS_ERR_UNSUPPORTED, "capacity %llu >= 2^32 with device counts", (unsigned long long)b->capacity);
  }
  return GS_OK;
}

struct Workspace {
  void *scan;            // scan partials of the count scan
  void *sort;            // radix sort scratch (per-tile digit counts and totals; depth, then bin sort)
  uint32_t *dkey;        // depth keys of the visible Gaussians (n)
  uint32_t *dkey_alt;    // depth sort double buffer (n)
  uint32_t *dval_alt;    // depth sort value buffers (n each)
  uint32_t *dval_b;
  uint64_t *dpos;        // first entry of each visible Gaussian in depth order (n + 1)
  uint32_t *bkey;        // bin key of each entry (capacity)
  uint32_t *bval;        // depth rank of each entry's Gaussian (capacity)
  uint32_t *bkey_alt;    // bin sort double buffer (capacity)
  uint32_t *bval_alt;    // (capacity)
  uint32_t *bfirst;      // first Gaussian (depth rank) of each 1,024-entry block (capacity / 1,024 + 1)
  uint64_t nbfirst;
  uint64_t *counts;      // {K, V}: packed for the one device-to-host copy; then the entry count of
                         // the device-count bin sort (low 32 bits of counts[2])
  size_t total;
};

Workspace carve(void *ws, int64_t n, uint64_t capacity) {
  Workspace w;
  char *p = static_cast<char *>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *q = p ? p + off : nullptr;
    off += align_up(bytes);
    return q;
  };
  const uint64_t nn = (uint64_t)(n > 0 ? n : 1);
  w.scan = take(gsi::scan_tmp_bytes(n));
  const size_t sort_bytes = gsi::radix_tmp_bytes(nn > capacity ? nn : capacity);
  const size_t depth_bytes = gsi::depth_sort_tmp_bytes(nn);
  w.sort = take(sort_bytes > depth_bytes ? sort_bytes : depth_bytes);
  w.dkey = reinterpret_cast<uint32_t *>(take(nn * 4));
  w.dkey_alt = reinterpret_cast<uint32_t *>(take(nn * 4));
  w.dval_alt = reinterpret_cast<uint32_t *>(take(nn * 4));
  w.dval_b = reinterpret_cast<uint32_t *>(take(nn * 4));
  w.dpos = reinterpret_cast<uint64_t *>(take((nn + 1) * 8));
  w.bkey = reinterpret_cast<uint32_t *>(take((size_t)capacity * 4));
  w.bval = reinterpret_cast<uint32_t *>(take((size_t)capacity * 4));
  w.bkey_alt = reinterpret_cast<uint32_t *>(take((size_t)capacity * 4));
  w.bval_alt = reinterpret_cast<uint32_t *>(take((size_t)capacity * 4));
  w.nbfirst = capacity / gsi::kFirstsBlock + 1;
  w.bfirst = reinterpret_cast<uint32_t *>(take(w.nbfirst * 4));
  w.counts = reinterpret_cast<uint64_t *>(take(3 * sizeof(uint64_t)));
  w.total = off;
  return w;
}

// Workgroups per bin.  Groups whose rows are built per member tile take one workgroup per
// member tile: a 1080p frame has only 510 (4x4) or 135 (8x8) groups, and a workgroup walking
// a row of member tiles kept their states in private memory (1M Gaussians at 1080p, FP16:
// raster 4x4 284 -> 142 us, 8x8 883 -> 250 us with one tile per workgroup).  2x2 groups
// with rows built in the group frame take one row of two member tiles per workgroup, blended
// side by side by eight waves (or in turn by four, with three pieces per row): one workgroup
// per group left most CUs idle while the last, densest groups finished.  Every tile still
// sees its rows in the same order with the same arithmetic, so the image does not depend on
// the split.
int raster_parts(const gs_options &o) {
  if (o.precision == GS_PREC_FP32) return 1;
  if (o.group == 2 && !(o.flags & GS_OPT_TILE_ROWS)) return 2;   // the group-frame rows
  return o.group * o.group;
}

gsi::RasterJob make_job(const gs_projected &p, const gs_bins &b, const gsi::Grid &g, float *image, float *aux,
                        int parts) {
  gsi::RasterJob j;
  j.xy = reinterpret_cast<const double2 *>(p.xy);
  j.conic = reinterpret_cast<const float4 *>(p.conic);
  j.rgb = reinterpret_cast<const float4 *>(p.rgb);
  j.vals = b.vals;
  j.masks = b.masks;
  j.ranges = b.ranges;
  j.image = image;
  j.aux = aux;
  j.W = g.W; j.H = g.H; j.TX = g.TX; j.TY = g.TY; j.GX = g.GX; j.GY = g.GY;
  j.nbins = (int)g.nbins;
  j.parts = parts;
  j.items = (int)g.nbins * parts;
  j.bin0 = 0;
  return j;
}

gsi::RasterParams make_params(const gs_options &o) {
  gsi::RasterParams p;
  p.G = o.group;
  p.prec = o.precision;
  p.splits = o.splits;
  for (int i = 0; i < 3; ++i) p.bg[i] = o.bg[i];
  p.aux_flags = o.aux_flags;
  p.all_rows = (o.flags & GS_OPT_ALL_ROWS) != 0;
  p.tile_rows = (o.flags & GS_OPT_TILE_ROWS) != 0;
  return p;
}

// Waits for the entry and visible counts that k_depth_keys writes into the caller's pinned host
// memory (set to a sentinel before the launch): a poll of that memory, bounded in time; should
// the values not arrive, the stream is synchronized and the workspace copy is read instead.
bool poll_counts(volatile uint64_t *h, uint64_t *kv) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0;; ++spin) {
    const uint64_t a = h[0], b = h[1];
    if (a != ~0ull && b != ~0ull) {
      kv[0] = a;
      kv[1] = b;
      return true;
    }
    if ((spin & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) return false;
  }
}

gs_status do_bin_sort(const gs_projected *proj, int64_t n, const gs_camera *cam, const gs_options *opt,
                      const gs_bins *bins, uint64_t *n_keys, void *ws, hipStream_t st) {
  const gsi::Grid g = gsi::make_grid(cam->width, cam->height, opt->group);
  const Workspace w = carve(ws, n, bins->capacity);
  // The one host wait reads the entry count K and the visible count V, which k_depth_keys writes
  // to the caller's pinned host memory (and to the workspace).  The depth sort (which reads V on
  // the device and also places each Gaussian's first entry) is enqueued before the host polls
  // for them, so the GPU keeps working while the host waits.
  // With the counts read on the device (GS_OPT_DEVICE_COUNTS) there is no host wait: the bin
  // sort's grids are sized for the capacity and its kernels take K (0 on overflow) and V from
  // the workspace.
  const bool dev_counts = (opt->flags & GS_OPT_DEVICE_COUNTS) != 0;
  volatile uint64_t *hkv = dev_counts ? nullptr : proj->host_counts;
  if (hkv) hkv[0] = hkv[1] = ~0ull;   // overwritten by the kernel
  const uint64_t nn = (uint64_t)(n > 0 ? n : 1);
  GS_HIP(gsi::launch_depth_keys(proj->order, reinterpret_cast<const float4 *>(proj->rgb), proj->n_visible, nn, w.dkey,
                                proj->offset + n, w.counts, const_cast<uint64_t *>(hkv), bins->capacity, w.sort, st));
  // from here on the kernel may be writing the counts: every exit waits for the stream first
  // depth bits in depth order, and the first entry of each Gaussian in that order (a single
  // Gaussian needs no sort: a gathered scan of its count)
  const uint32_t *dkeys = w.dkey;
  hipError_t e = nn > 1 ? gsi::sort_depth(proj->order, proj->n_visible, nn, w.dkey, w.dkey_alt, w.dval_alt, w.dval_b,
                                          w.sort, st, proj->count, w.dpos, w.bfirst, w.nbfirst)
                        : gsi::launch_scan_gather(proj->count, proj->order, w.dpos, (int64_t)nn, proj->n_visible,
                                                  w.scan, st);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(st);
    return hip_fail(e, "depth sort");
  }
  if (dev_counts) {
    const uint32_t *kdev = reinterpret_cast<const uint32_t *>(w.counts + 2);
    GS_HIP(gsi::bin_and_sort(proj->order, dkeys, w.dpos, nn > 1 ? w.bfirst : nullptr, (uint32_t)nn, bins->capacity,
                             proj->n_visible, kdev, proj->rect, proj->xy, proj->conic,
                             (opt->flags & GS_OPT_TIGHT) != 0, g, w.bkey, w.bval, w.bkey_alt, w.bval_alt,
                             bins->ranges, opt->group > 1 ? bins->masks : nullptr, bins->vals, bins->keys, w.sort,
                             st));
    return GS_OK;
  }
  uint64_t kv[2] = {0, 0};
  if (!hkv || !poll_counts(hkv, kv)) {
    // no pinned buffer, or the values did not arrive through it: the workspace copy, after the
    // stream has drained
    const hipError_t es = hipStreamSynchronize(st);
    if (es != hipSuccess) return hip_fail(es, "hipStreamSynchronize");
    GS_HIP(hipMemcpy(kv, w.counts, sizeof(kv), hipMemcpyDeviceToHost));
  }
  const uint64_t K = kv[0];
  const uint32_t V = (uint32_t)kv[1];
  *n_keys = K;
  // The depth sort and the depth-order scan enqueued above may still be writing the workspace
  // and proj->order: an error return first waits for them, so that the caller may release or
  // reuse the workspace (on any stream) as soon as the call returns.
  const char *why = nullptr;
  gs_status bad = GS_OK;
  if (K > bins->capacity) bad = GS_ERR_CAPACITY, why = "entries exceed capacity";
  else if (K >= (1ull << 32)) bad = GS_ERR_UNSUPPORTED, why = "entries >= 2^32";
  else if ((int64_t)V > n) bad = GS_ERR_INVALID_ARG, why = "visible count exceeds n";
  if (bad != GS_OK) {
    const hipError_t ew = hipStreamSynchronize(st);
    if (ew != hipSuccess) return hip_fail(ew, "hipStreamSynchronize");
    return fail(bad, "%s (%llu entries, capacity %llu, %u visible of %lld)", why, (unsigned long long)K,
                (unsigned long long)bins->capacity, V, (long long)n);
  }
  // one thread per entry (also clears the bin ranges), the bin passes (the last one places the
  // Gaussian indices and 64-bit keys), the ranges and masks
  GS_HIP(gsi::bin_and_sort(proj->order, dkeys, w.dpos, nn > 1 ? w.bfirst : nullptr, V, K, nullptr, nullptr, proj->rect,
                           proj->xy, proj->conic,
                           (opt->flags & GS_OPT_TIGHT) != 0, g, w.bkey, w.bval, w.bkey_alt, w.bval_alt, bins->ranges,
                           opt->group > 1 ? bins->masks : nullptr, bins->vals, bins->keys, w.sort, st));
  return GS_OK;
}

// Validated job table of a batched launch (host only, no HIP call).
gs_status batch_table(const gs_job *jobs, int32_t n_jobs, const gs_options *opt, gsi::BatchTable *table) {
  gs_status s;
  if ((s = check_options(opt))) return s;
  if (n_jobs < 0) return fail(GS_ERR_INVALID_ARG, "n_jobs = %d", n_jobs);
  if (n_jobs > gsi::kMaxBatch) return fail(GS_ERR_UNSUPPORTED, "n_jobs = %d above %d", n_jobs, gsi::kMaxBatch);
  if (n_jobs == 0) return GS_OK;
  if (!jobs) return fail(GS_ERR_INVALID_ARG, "jobs is NULL");
  int64_t total = 0;
  for (int32_t i = 0; i < n_jobs; ++i) {
    const gs_job &jb = jobs[i];
    if ((s = check_camera(&jb.cam))) return fail(s, "job %d: camera", i);
    if ((s = check_bins(jb.bins, opt->group, false))) return fail(s, "job %d: bins", i);
    if (!jb.proj || !jb.proj->xy || !jb.proj->conic || !jb.proj->rgb)
      return fail(GS_ERR_INVALID_ARG, "job %d: projected record is NULL", i);
    if (!jb.image) return fail(GS_ERR_INVALID_ARG, "job %d: image is NULL", i);
    if (opt->aux_flags && !jb.aux) return fail(GS_ERR_INVALID_ARG, "job %d: aux is NULL with aux_flags set", i);
    const gsi::Grid g = gsi::make_grid(jb.cam.width, jb.cam.height, opt->group);
    table->jobs[i] = make_job(*jb.proj, *jb.bins, g, jb.image, jb.aux, raster_parts(*opt));
    table->jobs[i].bin0 = (int)total;
    total += table->jobs[i].items;
    if (total >= (1ll << 31)) return fail(GS_ERR_UNSUPPORTED, "batch has >= 2^31 work items");
  }
  table->n_jobs = n_jobs;
  table->total = (int)total;
  return GS_OK;
}

// One persistent launch over the table; `counter` (GS_BATCH_COUNTER_BYTES of device memory) is
// cleared by a fill kernel on the stream first (no memset node, so the launch can be captured in
// a graph).
gs_status batch_launch(const gsi::BatchTable &table, const gs_options &opt, uint32_t *counter, hipStream_t st) {
  int dev = 0, cus = 0;
  GS_HIP(hipGetDevice(&dev));
  GS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const gsi::RasterParams p = make_params(opt);
  // persistent grid: enough workgroups to fill every CU several times, never more than items
  int64_t grid = (int64_t)cus * 8;
  if (grid > table.total) grid = table.total;
  GS_HIP(gsi::launch_fill_u32(counter, GS_BATCH_COUNTER_BYTES / 4, 0u, st));
  if (opt.precision == GS_PREC_FP32)
    GS_HIP(gsi::launch_raster_fp32_batch(table, (int)grid, p, counter, st));
  else
    GS_HIP(gsi::launch_raster_mfma_batch(table, (int)grid, p, counter, st));
  return GS_OK;
}

// ---- scratch of the allocation-free entry point ------------------------------------------
// A file-scope device array: every GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code `scratch` names a host-side stand-in, so its
// device address is looked up once per device (with that device current) and only that
// address is ever passed to a kernel.
constexpr size_t kScratchBytes = GS_NOALLOC_SCRATCH_BYTES;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_addr[kMaxDevices] = {};

gs_status scratch_on_current_device(uint32_t **out) {
  int dev = 0;
  GS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GS_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(GS_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[dev] = static_cast<uint32_t *>(p);
  }
  *out = g_scratch_addr[dev];
  return GS_OK;
}

gs_status backward_job(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam, const gs_options *opt,
                       const float *dimage, const gs_grads *grads, gsi::BackwardJob *out) {
  gs_status s;
  if ((s = check_camera(cam)) || (s = check_options(opt))) return s;
  if (opt->group != 1) return fail(GS_ERR_UNSUPPORTED, "backward pass over group %d bins (tile bins only)", opt->group);
  if ((s = check_bins(bins, 1, false))) return s;
  if (!proj || !proj->xy || !proj->conic || !proj->rgb) return fail(GS_ERR_INVALID_ARG, "projected record is NULL");
  if (!dimage) return fail(GS_ERR_INVALID_ARG, "dimage is NULL");
  if (!grads || !grads->rgb || !grads->opacity || !grads->conic || !grads->xy)
    return fail(GS_ERR_INVALID_ARG, "gradient buffer is NULL");
  const gsi::Grid g = gsi::make_grid(cam->width, cam->height, 1);
  gsi::BackwardJob &j = *out;
  j.xy = reinterpret_cast<const double2 *>(proj->xy);
  j.conic = reinterpret_cast<const float4 *>(proj->conic);
  j.rgb = reinterpret_cast<const float4 *>(proj->rgb);
  j.vals = bins->vals;
  j.ranges = bins->ranges;
  j.dimage = dimage;
  j.g_rgb = grads->rgb;
  j.g_op = grads->opacity;
  j.g_conic = grads->conic;
  j.g_xy = grads->xy;
  j.W = g.W;
  j.H = g.H;
  j.TX = g.TX;
  j.TY = g.TY;
  for (int c = 0; c < 3; ++c) j.bg[c] = opt->bg[c];
  j.t_final = nullptr;
  j.last = nullptr;
  return GS_OK;
}

}  // namespace

extern "C" {

const char *gs_status_string(gs_status s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID_ARG: return "invalid argument";
    case GS_ERR_UNSUPPORTED: return "unsupported";
    case GS_ERR_CAPACITY: return "capacity exceeded";
    case GS_ERR_HIP: return "HIP error";
  }
  return "unknown status";
}

const char *gs_last_error(void) { return g_err; }

int64_t gs_num_bins(const gs_camera *cam, int32_t group) {
  if (!cam || cam->width <= 0 || cam->height <= 0 || group < 1) return 0;
  return gsi::make_grid(cam->width, cam->height, group).nbins;
}

size_t gs_workspace_bytes(int64_t n, uint64_t capacity, const gs_camera *cam, const gs_options *opt) {
  (void)cam;
  (void)opt;
  if (n < 0) return 0;
  return carve(nullptr, n, capacity).total;
}

gs_status gs_preprocess(const gs_scene *scene, const gs_camera *cam, const gs_options *opt, const gs_projected *out,
                        void *ws, size_t ws_bytes, void *stream) {
  gs_status s;
  if ((s = check_scene(scene)) || (s = check_camera(cam)) || (s = check_options(opt)) ||
      (s = check_projected(out, scene->n, true)))
    return s;
  const size_t need = gsi::scan_tmp_bytes(scene->n);
  if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID_ARG, "workspace %zu bytes, need %zu", ws_bytes, need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const gsi::Grid g = gsi::make_grid(cam->width, cam->height, opt->group);
  GS_HIP(gsi::launch_preprocess(*scene, *cam, g, *out, (opt->flags & GS_OPT_TIGHT) != 0, ws, st));
  GS_HIP(gsi::launch_scan_compact(out->count, out->offset, scene->n, out->order, out->n_visible, ws, true, st));
  return GS_OK;
}

gs_status gs_bin_sort(const gs_projected *proj, int64_t n, const gs_camera *cam, const gs_options *opt,
                      const gs_bins *bins, uint64_t *n_keys, void *ws, size_t ws_bytes, void *stream) {
  gs_status s;
  if (n < 0) return fail(GS_ERR_INVALID_ARG, "n = %lld", (long long)n);
  if (n >= (1ll << 31)) return fail(GS_ERR_UNSUPPORTED, "n = %lld >= 2^31", (long long)n);
  if ((s = check_camera(cam)) || (s = check_options(opt)) || (s = check_projected(proj, n, true)) ||
      (s = check_bins(bins, opt->group, true)))
    return s;
  if ((s = check_device_counts(opt, bins, n_keys))) return s;
  const size_t need = carve(nullptr, n, bins->capacity).total;
  if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID_ARG, "workspace %zu bytes, need %zu", ws_bytes, need);
  return do_bin_sort(proj, n, cam, opt, bins, n_keys, ws, static_cast<hipStream_t>(stream));
}

gs_status gs_rasterize(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam, const gs_options *opt,
                       float *image, float *aux, void *stream) {
  gs_status s;
  if ((s = check_camera(cam)) || (s = check_options(opt)) || (s = check_bins(bins, opt->group, false))) return s;
  if (!proj || !proj->xy || !proj->conic || !proj->rgb) return fail(GS_ERR_INVALID_ARG, "projected record is NULL");
  if (!image) return fail(GS_ERR_INVALID_ARG, "image is NULL");
  if (opt->aux_flags && !aux) return fail(GS_ERR_INVALID_ARG, "aux is NULL with aux_flags set");
  const gsi::Grid g = gsi::make_grid(cam->width, cam->height, opt->group);
  const gsi::RasterJob j = make_job(*proj, *bins, g, image, aux, raster_parts(*opt));
  const gsi::RasterParams p = make_params(*opt);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (opt->precision == GS_PREC_FP32)
    GS_HIP(gsi::launch_raster_fp32(j, p, st));
  else
    GS_HIP(gsi::launch_raster_mfma(j, p, st));
  return GS_OK;
}


gs_status gs_rasterize_backward(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam,
                                const gs_options *opt, const float *dimage, const gs_grads *grads, void *stream) {
  gsi::BackwardJob j;
  const gs_status s = backward_job(proj, bins, cam, opt, dimage, grads, &j);
  if (s) return s;
  GS_HIP(gsi::launch_raster_backward(j, static_cast<hipStream_t>(stream)));
  return GS_OK;
}

gs_status gs_rasterize_backward_mfma(const gs_projected *proj, const gs_bins *bins, const gs_camera *cam,
                                     const gs_options *opt, const float *dimage, const float *t_final,
                                     const float *last, const gs_grads *grads, void *stream) {
  gsi::BackwardJob j;
  gs_status s = backward_job(proj, bins, cam, opt, dimage, grads, &j);
  if (s) return s;
  if (opt->precision != GS_PREC_FP16_MFMA && opt->precision != GS_PREC_BF16_MFMA)
    return fail(GS_ERR_INVALID_ARG, "precision %d is not an MFMA precision", opt->precision);
  if (!t_final || !last) return fail(GS_ERR_INVALID_ARG, "t_final or last is NULL");
  j.t_final = t_final;
  j.last = last;
  GS_HIP(gsi::launch_raster_backward_mfma(j, opt->precision, opt->splits, (opt->flags & GS_OPT_ALL_ROWS) != 0,
                                          static_cast<hipStream_t>(stream)));
  return GS_OK;
}

gs_status gs_render(const gs_scene *scene, const gs_camera *cam, const gs_options *opt, const gs_projected *proj,
                    const gs_bins *bins, float *image, float *aux, uint64_t *n_keys, void *ws, size_t ws_bytes,
                    void *stream) {
  gs_status s;
  if ((s = check_scene(scene)) || (s = check_camera(cam)) || (s = check_options(opt)) ||
      (s = check_projected(proj, scene->n, true)) || (s = check_bins(bins, opt->group, true)))
    return s;
  if (!image) return fail(GS_ERR_INVALID_ARG, "image is NULL");
  if (opt->aux_flags && !aux) return fail(GS_ERR_INVALID_ARG, "aux is NULL with aux_flags set");
  if ((s = check_device_counts(opt, bins, n_keys))) return s;
  const size_t need = carve(nullptr, scene->n, bins->capacity).total;
  if (!ws || ws_bytes < need) return fail(GS_ERR_INVALID_ARG, "workspace %zu bytes, need %zu", ws_bytes, need);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const gsi::Grid g = gsi::make_grid(cam->width, cam->height, opt->group);
  GS_HIP(gsi::launch_preprocess(*scene, *cam, g, *proj, (opt->flags & GS_OPT_TIGHT) != 0, ws, st));
  GS_HIP(gsi::launch_scan_compact(proj->count, proj->offset, scene->n, proj->order, proj->n_visible, ws, true, st));
  if ((s = do_bin_sort(proj, scene->n, cam, opt, bins, n_keys, ws, st))) return s;
  const gsi::RasterJob j = make_job(*proj, *bins, g, image, aux, raster_parts(*opt));
  const gsi::RasterParams p = make_params(*opt);
  if (opt->precision == GS_PREC_FP32)
    GS_HIP(gsi::launch_raster_fp32(j, p, st));
  else
    GS_HIP(gsi::launch_raster_mfma(j, p, st));
  return GS_OK;
}

size_t gs_sort_workspace_bytes(uint64_t n) {
  return align_up((size_t)n * sizeof(uint64_t)) + align_up((size_t)n * sizeof(uint32_t)) +
         align_up(gsi::radix_tmp_bytes(n));
}

gs_status gs_radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t n, int32_t lo_bit, int32_t hi_bit, void *ws,
                            size_t ws_bytes, void *stream) {
  if (n > 0 && (!keys || !vals)) return fail(GS_ERR_INVALID_ARG, "keys or vals is NULL");
  if (lo_bit < 0 || hi_bit > 64 || lo_bit > hi_bit) return fail(GS_ERR_INVALID_ARG, "bit range [%d, %d)", lo_bit, hi_bit);
  if (n >= (1ull << 32)) return fail(GS_ERR_UNSUPPORTED, "n >= 2^32");
  const size_t need = gs_sort_workspace_bytes(n);
  if (n > 1 && (!ws || ws_bytes < need)) return fail(GS_ERR_INVALID_ARG, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (n <= 1) return GS_OK;
  char *p = static_cast<char *>(ws);
  uint64_t *ka = reinterpret_cast<uint64_t *>(p);
  uint32_t *va = reinterpret_cast<uint32_t *>(p + align_up((size_t)n * sizeof(uint64_t)));
  void *tmp = p + align_up((size_t)n * sizeof(uint64_t)) + align_up((size_t)n * sizeof(uint32_t));
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool in_alt = false;
  GS_HIP(gsi::radix_sort(keys, vals, ka, va, n, lo_bit, hi_bit, tmp, st, &in_alt));
  if (in_alt) {
    GS_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    GS_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
  }
  return GS_OK;
}

int32_t gs_max_batch(void) { return gsi::kMaxBatch; }

gs_status gs_rasterize_batch(const gs_job *jobs, int32_t n_jobs, const gs_options *opt, uint32_t *work_counter,
                             void *stream) {
  gsi::BatchTable table{};
  gs_status s = batch_table(jobs, n_jobs, opt, &table);
  if (s || n_jobs == 0) return s;
  if (!work_counter) return fail(GS_ERR_INVALID_ARG, "work_counter is NULL");
  return batch_launch(table, *opt, work_counter, static_cast<hipStream_t>(stream));
}

gs_status gs_rasterize_batch_noalloc(const gs_job *jobs, int32_t n_jobs, const gs_options *opt, void *stream) {
  gsi::BatchTable table{};
  gs_status s = batch_table(jobs, n_jobs, opt, &table);
  if (s || n_jobs == 0) return s;
  // the launch's work counters; the scratch array holds kScratchBytes
  static_assert(GS_BATCH_COUNTER_BYTES <= kScratchBytes, "scratch too small for the work counters");
  uint32_t *counter = nullptr;
  if ((s = scratch_on_current_device(&counter))) return s;
  return batch_launch(table, *opt, counter, static_cast<hipStream_t>(stream));
}

}  // extern "C"
