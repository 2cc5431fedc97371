"""Thin Python binding of the C ABI in include/gs.h (argument marshalling only).

Every stage runs in the HIP library libgs.so; torch provides device memory and
streams.  The binding fails loudly when the library is missing: there is no
CPU path.  Names follow the C ABI: gs_preprocess, gs_bin_sort, gs_rasterize,
gs_render, gs_radix_sort_u64, plus a small `Renderer` that owns the buffers of
one frame and grows the entry buffers when gs_bin_sort reports GS_ERR_CAPACITY.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_UNSUPPORTED, GS_ERR_CAPACITY, GS_ERR_HIP = range(5)
GS_PREC_FP32, GS_PREC_FP16_MFMA, GS_PREC_BF16_MFMA = range(3)
GS_AUX_TFINAL, GS_AUX_WSUM, GS_AUX_NEVAL, GS_AUX_NBLEND, GS_AUX_LAST = 1, 2, 4, 8, 16
GS_OPT_TIGHT = 1
GS_OPT_ALL_ROWS = 2
GS_OPT_TILE_ROWS = 4
GS_OPT_DEVICE_COUNTS = 8
GS_BATCH_COUNTER_BYTES = 512          # work counters of one batched launch (include/gs.h)
BATCH_COUNTER_WORDS = GS_BATCH_COUNTER_BYTES // 4
PRECISIONS = {"fp32": GS_PREC_FP32, "fp16": GS_PREC_FP16_MFMA, "bf16": GS_PREC_BF16_MFMA}
TILE = 16


class GsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gs status {status}: {msg}")
        self.status = status


class gs_options(C.Structure):
    _fields_ = [("group", C.c_int32), ("precision", C.c_int32), ("splits", C.c_int32),
                ("bg", C.c_float * 3), ("aux_flags", C.c_uint32), ("flags", C.c_uint32)]


class gs_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("znear", C.c_float)]


class gs_scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32),
                ("mean", C.c_void_p), ("log_scale", C.c_void_p), ("quat", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class gs_projected(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("conic", C.c_void_p), ("rgb", C.c_void_p), ("rect", C.c_void_p),
                ("count", C.c_void_p), ("offset", C.c_void_p), ("order", C.c_void_p), ("n_visible", C.c_void_p),
                ("host_counts", C.c_void_p)]


class gs_bins(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("vals", C.c_void_p), ("masks", C.c_void_p),
                ("capacity", C.c_uint64), ("ranges", C.c_void_p)]


class gs_grads(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("opacity", C.c_void_p), ("conic", C.c_void_p), ("xy", C.c_void_p)]


class gs_job(C.Structure):
    _fields_ = [("proj", C.POINTER(gs_projected)), ("bins", C.POINTER(gs_bins)), ("cam", gs_camera),
                ("image", C.c_void_p), ("aux", C.c_void_p)]


EXPORTS = ["gs_num_bins", "gs_workspace_bytes", "gs_preprocess", "gs_bin_sort", "gs_rasterize", "gs_render",
           "gs_sort_workspace_bytes", "gs_radix_sort_u64", "gs_max_batch", "gs_rasterize_batch",
           "gs_rasterize_batch_noalloc", "gs_rasterize_backward_mfma",
           "gs_rasterize_backward", "gs_status_string", "gs_last_error"]

_lib = None


def lib():
    """Loads libgs.so (build it with `python -m paper_2605_17855_amd.build`)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library is not built "
                          "(python -m paper_2605_17855_amd.build)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.gs_num_bins.argtypes = [P(gs_camera), C.c_int32]
    L.gs_num_bins.restype = C.c_int64
    L.gs_workspace_bytes.argtypes = [C.c_int64, C.c_uint64, P(gs_camera), P(gs_options)]
    L.gs_workspace_bytes.restype = C.c_size_t
    L.gs_preprocess.argtypes = [P(gs_scene), P(gs_camera), P(gs_options), P(gs_projected), C.c_void_p,
                                C.c_size_t, C.c_void_p]
    L.gs_bin_sort.argtypes = [P(gs_projected), C.c_int64, P(gs_camera), P(gs_options), P(gs_bins),
                              P(C.c_uint64), C.c_void_p, C.c_size_t, C.c_void_p]
    L.gs_rasterize.argtypes = [P(gs_projected), P(gs_bins), P(gs_camera), P(gs_options), C.c_void_p, C.c_void_p,
                               C.c_void_p]
    L.gs_render.argtypes = [P(gs_scene), P(gs_camera), P(gs_options), P(gs_projected), P(gs_bins), C.c_void_p,
                            C.c_void_p, P(C.c_uint64), C.c_void_p, C.c_size_t, C.c_void_p]
    L.gs_sort_workspace_bytes.argtypes = [C.c_uint64]
    L.gs_sort_workspace_bytes.restype = C.c_size_t
    L.gs_radix_sort_u64.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_size_t, C.c_void_p]
    L.gs_max_batch.argtypes = []
    L.gs_max_batch.restype = C.c_int32
    L.gs_rasterize_batch.argtypes = [P(gs_job), C.c_int32, P(gs_options), C.c_void_p, C.c_void_p]
    L.gs_rasterize_batch_noalloc.argtypes = [P(gs_job), C.c_int32, P(gs_options), C.c_void_p]
    L.gs_rasterize_backward_mfma.argtypes = [P(gs_projected), P(gs_bins), P(gs_camera), P(gs_options), C.c_void_p,
                                             C.c_void_p, C.c_void_p, P(gs_grads), C.c_void_p]
    L.gs_rasterize_backward.argtypes = [P(gs_projected), P(gs_bins), P(gs_camera), P(gs_options), C.c_void_p,
                                        P(gs_grads), C.c_void_p]
    for f in ("gs_preprocess", "gs_bin_sort", "gs_rasterize", "gs_render", "gs_radix_sort_u64",
              "gs_rasterize_batch", "gs_rasterize_batch_noalloc", "gs_rasterize_backward",
              "gs_rasterize_backward_mfma"):
        getattr(L, f).restype = C.c_int
    L.gs_status_string.argtypes = [C.c_int]
    L.gs_status_string.restype = C.c_char_p
    L.gs_last_error.argtypes = []
    L.gs_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int):
    if status != GS_OK:
        raise GsError(status, lib().gs_last_error().decode())


def options(group: int = 1, precision="fp32", splits: int = 2, bg=(0.0, 0.0, 0.0), aux_flags: int = 0,
            tight: bool = False, all_rows: bool = False, tile_rows: bool = False,
            device_counts: bool = False) -> gs_options:
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    o = gs_options()
    o.group, o.precision, o.splits = group, precision, splits
    o.bg = (C.c_float * 3)(*bg)
    o.aux_flags = aux_flags
    o.flags = (GS_OPT_TIGHT if tight else 0) | (GS_OPT_ALL_ROWS if all_rows else 0) | \
        (GS_OPT_TILE_ROWS if tile_rows else 0) | (GS_OPT_DEVICE_COUNTS if device_counts else 0)
    return o


def camera(cam) -> gs_camera:
    """gs_camera from a scenes.Camera (or anything with R, t, fx, fy, cx, cy, width, height, znear)."""
    c = gs_camera()
    c.R = (C.c_float * 9)(*np.asarray(cam.R, np.float32).reshape(-1).tolist())
    c.t = (C.c_float * 3)(*np.asarray(cam.t, np.float32).reshape(-1).tolist())
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    c.width, c.height, c.znear = cam.width, cam.height, cam.znear
    return c


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def gs_num_bins(cam, group: int = 1) -> int:
    return int(lib().gs_num_bins(C.byref(camera(cam)), group))


class DeviceScene:
    """Scene arrays resident in device memory (float32, SoA) and their gs_scene struct."""

    def __init__(self, scene, device="cuda"):
        import torch
        self.n = scene.n
        self.sh_degree = scene.sh_degree
        self.mean = torch.from_numpy(np.ascontiguousarray(scene.mean)).to(device)
        self.log_scale = torch.from_numpy(np.ascontiguousarray(scene.log_scale)).to(device)
        self.quat = torch.from_numpy(np.ascontiguousarray(scene.quat)).to(device)
        self.opacity = torch.from_numpy(np.ascontiguousarray(scene.opacity)).to(device)
        # per-Gaussian contiguous coefficients (n, (deg+1)^2 * 3), the library's layout
        sh = np.asarray(scene.sh).reshape((self.sh_degree + 1) ** 2 * 3, self.n)
        self.sh = torch.from_numpy(np.ascontiguousarray(sh.T)).to(device)
        s = gs_scene()
        s.n, s.sh_degree, s.reserved = self.n, self.sh_degree, 0
        s.mean, s.log_scale, s.quat = _ptr(self.mean), _ptr(self.log_scale), _ptr(self.quat)
        s.opacity, s.sh = _ptr(self.opacity), _ptr(self.sh)
        self.struct = s

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in (self.mean, self.log_scale, self.quat, self.opacity, self.sh))


class Projected:
    """Device buffers of gs_projected for n Gaussians."""

    def __init__(self, n: int, device="cuda"):
        import torch
        self.n = n
        m = max(n, 1)
        self.xy = torch.empty((m, 2), dtype=torch.float64, device=device)
        self.conic = torch.empty((m, 4), dtype=torch.float32, device=device)
        self.rgb = torch.empty((m, 4), dtype=torch.float32, device=device)
        self.rect = torch.empty((m, 4), dtype=torch.int16, device=device)
        self.count = torch.empty((m,), dtype=torch.int32, device=device)
        self.offset = torch.empty((n + 1,), dtype=torch.int64, device=device)
        self.order = torch.empty((m,), dtype=torch.int32, device=device)
        self.n_visible = torch.empty((1,), dtype=torch.int32, device=device)
        # pinned host memory the library's count readback polls (entry and visible counts)
        self.host_counts = torch.empty((2,), dtype=torch.int64, pin_memory=True)
        p = gs_projected()
        p.xy, p.conic, p.rgb = _ptr(self.xy), _ptr(self.conic), _ptr(self.rgb)
        p.rect, p.count, p.offset = _ptr(self.rect), _ptr(self.count), _ptr(self.offset)
        p.order, p.n_visible = _ptr(self.order), _ptr(self.n_visible)
        p.host_counts = _ptr(self.host_counts)
        self.struct = p


class Bins:
    """Device buffers of gs_bins: `capacity` entries and the bin ranges of one camera/group."""

    def __init__(self, capacity: int, nbins: int, device="cuda", group: int = 1):
        import torch
        self.capacity = int(capacity)
        c = max(self.capacity, 1)
        self.keys = torch.empty((c,), dtype=torch.int64, device=device)
        self.vals = torch.empty((c,), dtype=torch.int32, device=device)
        self.masks = torch.empty((c,), dtype=torch.int64 if group == 8 else torch.int16, device=device)
        self.ranges = torch.empty((max(nbins, 1), 2), dtype=torch.int32, device=device)
        b = gs_bins()
        b.keys, b.vals, b.masks = _ptr(self.keys), _ptr(self.vals), _ptr(self.masks)
        b.capacity = self.capacity
        b.ranges = _ptr(self.ranges)
        self.struct = b

    @classmethod
    def from_tensors(cls, keys, vals, masks, ranges, capacity: int) -> "Bins":
        """Bins over caller-provided device tensors (e.g. views of a memory pool)."""
        self = cls.__new__(cls)
        self.capacity = int(capacity)
        self.keys, self.vals, self.masks, self.ranges = keys, vals, masks, ranges
        b = gs_bins()
        b.keys, b.vals, b.masks = _ptr(keys), _ptr(vals), _ptr(masks)
        b.capacity = self.capacity
        b.ranges = _ptr(ranges)
        self.struct = b
        return self


def gs_preprocess(scene: DeviceScene, cam, opt: gs_options, proj: Projected, ws, stream=None):
    _check(lib().gs_preprocess(C.byref(scene.struct), C.byref(camera(cam)), C.byref(opt), C.byref(proj.struct),
                               _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def gs_bin_sort(proj: Projected, cam, opt: gs_options, bins: Bins, ws, stream=None):
    """Returns the entry count; raises GsError (status GS_ERR_CAPACITY with .n_keys) when bins is too small.
    With GS_OPT_DEVICE_COUNTS returns None: the count stays on the device (entry_count)."""
    n_keys = C.c_uint64(0)
    st = lib().gs_bin_sort(C.byref(proj.struct), proj.n, C.byref(camera(cam)), C.byref(opt), C.byref(bins.struct),
                           C.byref(n_keys), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    if st != GS_OK:
        err = GsError(st, lib().gs_last_error().decode())
        err.n_keys = int(n_keys.value)
        raise err
    return None if opt.flags & GS_OPT_DEVICE_COUNTS else int(n_keys.value)


def entry_count(proj: Projected) -> int:
    """The entry count that the last gs_preprocess/gs_render left on the device (offset[n]);
    reads device memory, so it waits for the work before it on the current stream."""
    return int(proj.offset[proj.n].item())


def gs_rasterize(proj: Projected, bins: Bins, cam, opt: gs_options, image, aux=None, stream=None):
    _check(lib().gs_rasterize(C.byref(proj.struct), C.byref(bins.struct), C.byref(camera(cam)), C.byref(opt),
                              _ptr(image), _ptr(aux), _stream(stream)))


class Grads:
    """Device buffers of gs_grads for n Gaussians (FP32, zeroed; gs_rasterize_backward adds to them)."""

    def __init__(self, n: int, device="cuda"):
        import torch
        m = max(n, 1)
        self.rgb = torch.zeros((m, 3), dtype=torch.float32, device=device)
        self.opacity = torch.zeros((m,), dtype=torch.float32, device=device)
        self.conic = torch.zeros((m, 3), dtype=torch.float32, device=device)
        self.xy = torch.zeros((m, 2), dtype=torch.float32, device=device)
        g = gs_grads()
        g.rgb, g.opacity, g.conic, g.xy = _ptr(self.rgb), _ptr(self.opacity), _ptr(self.conic), _ptr(self.xy)
        self.struct = g

    def zero_(self):
        for t in (self.rgb, self.opacity, self.conic, self.xy):
            t.zero_()


def gs_rasterize_backward(proj: Projected, bins: Bins, cam, opt: gs_options, dimage, grads: Grads, stream=None):
    """Adds to `grads` the gradients of sum(dimage * image) for the image gs_rasterize writes
    (FP32 arithmetic, tile bins)."""
    _check(lib().gs_rasterize_backward(C.byref(proj.struct), C.byref(bins.struct), C.byref(camera(cam)),
                                       C.byref(opt), _ptr(dimage), C.byref(grads.struct), _stream(stream)))


def gs_rasterize_backward_mfma(proj: Projected, bins: Bins, cam, opt: gs_options, dimage, t_final, last,
                               grads: Grads, stream=None):
    """Adds to `grads` the gradients of sum(dimage * image) for the image of the MFMA forward
    (opt.precision fp16/bf16, opt.splits), starting from the forward's GS_AUX_TFINAL and
    GS_AUX_LAST planes (t_final, last: (H, W) float32 device tensors)."""
    _check(lib().gs_rasterize_backward_mfma(C.byref(proj.struct), C.byref(bins.struct), C.byref(camera(cam)),
                                            C.byref(opt), _ptr(dimage), _ptr(t_final), _ptr(last),
                                            C.byref(grads.struct), _stream(stream)))


def gs_render(scene: DeviceScene, cam, opt: gs_options, proj: Projected, bins: Bins, image, aux, ws,
              stream=None):
    """Returns the entry count; raises GsError (status GS_ERR_CAPACITY with .n_keys) when bins is too small.
    With GS_OPT_DEVICE_COUNTS returns None without waiting: the count stays on the device (entry_count),
    and a count above bins.capacity leaves the background image."""
    n_keys = C.c_uint64(0)
    st = lib().gs_render(C.byref(scene.struct), C.byref(camera(cam)), C.byref(opt), C.byref(proj.struct),
                         C.byref(bins.struct), _ptr(image), _ptr(aux), C.byref(n_keys), _ptr(ws),
                         ws.numel() * ws.element_size(), _stream(stream))
    if st != GS_OK:
        err = GsError(st, lib().gs_last_error().decode())
        err.n_keys = int(n_keys.value)
        raise err
    return None if opt.flags & GS_OPT_DEVICE_COUNTS else int(n_keys.value)


def gs_radix_sort_u64(keys, vals, lo_bit: int, hi_bit: int, ws=None, stream=None):
    import torch
    n = keys.numel()
    need = int(lib().gs_sort_workspace_bytes(n))
    if ws is None:
        ws = torch.empty((max(need, 1),), dtype=torch.uint8, device=keys.device)
    _check(lib().gs_radix_sort_u64(_ptr(keys), _ptr(vals), n, lo_bit, hi_bit, _ptr(ws), ws.numel(),
                                   _stream(stream)))


def gs_rasterize_batch(items, opt: gs_options, counter, stream=None):
    """items: list of (Projected, Bins, camera, image, aux-or-None).  One persistent launch.
    counter: device memory of GS_BATCH_COUNTER_BYTES (e.g. BATCH_COUNTER_WORDS int32)."""
    n = len(items)
    arr = (gs_job * max(n, 1))()
    for i, (proj, bins, cam, image, aux) in enumerate(items):
        arr[i].proj = C.pointer(proj.struct)
        arr[i].bins = C.pointer(bins.struct)
        arr[i].cam = camera(cam)
        arr[i].image = _ptr(image)
        arr[i].aux = _ptr(aux)
    _check(lib().gs_rasterize_batch(arr, n, C.byref(opt), _ptr(counter), _stream(stream)))


def _job_array(items):
    n = len(items)
    arr = (gs_job * max(n, 1))()
    for i, (proj, bins, cam, image, aux) in enumerate(items):
        arr[i].proj = C.pointer(proj.struct)
        arr[i].bins = C.pointer(bins.struct)
        arr[i].cam = camera(cam)
        arr[i].image = _ptr(image)
        arr[i].aux = _ptr(aux)
    return arr, n


def gs_rasterize_batch_noalloc(items, opt: gs_options, stream=None):
    """gs_rasterize_batch with the work counter in the library's own device scratch (no buffer
    from the caller, nothing allocated).  Calls that overlap on one GPU race on that counter."""
    arr, n = _job_array(items)
    _check(lib().gs_rasterize_batch_noalloc(arr, n, C.byref(opt), _stream(stream)))


def aux_planes(flags: int) -> int:
    return bin(flags & 31).count("1")


class Renderer:
    """Owns the device buffers of one frame for a given scene size and camera size."""

    def __init__(self, n: int, width: int, height: int, group: int = 1, capacity: int = 0, device="cuda"):
        import torch
        self.device = device
        self.n, self.width, self.height, self.group = n, width, height, group
        self.proj = Projected(n, device)
        tx, ty = (width + TILE - 1) // TILE, (height + TILE - 1) // TILE
        self.nbins = ((tx + group - 1) // group) * ((ty + group - 1) // group)
        self.bins = None
        self.ws = None
        self._alloc_bins(capacity or max(4 * n, 1024))
        self.image = torch.empty((3, height, width), dtype=torch.float32, device=device)
        self.aux = None

    def _alloc_bins(self, capacity: int):
        import torch
        self.bins = Bins(capacity, self.nbins, self.device, self.group)
        c = camera_stub(self.width, self.height)
        o = options(self.group)
        need = int(lib().gs_workspace_bytes(self.n, capacity, C.byref(c), C.byref(o)))
        self.ws = torch.empty((max(need, 1),), dtype=torch.uint8, device=self.device)

    def render(self, scene: DeviceScene, cam, opt: gs_options, stream=None):
        import torch
        assert cam.width == self.width and cam.height == self.height and opt.group == self.group
        npl = aux_planes(opt.aux_flags)
        if npl and (self.aux is None or self.aux.shape[0] != npl):
            self.aux = torch.empty((npl, self.height, self.width), dtype=torch.float32, device=self.device)
        if opt.flags & GS_OPT_DEVICE_COUNTS:
            # no host wait and so no retry: the caller checks entry_count(self.proj) <= capacity
            return gs_render(scene, cam, opt, self.proj, self.bins, self.image, self.aux if npl else None,
                             self.ws, stream)
        for _ in range(2):
            try:
                return gs_render(scene, cam, opt, self.proj, self.bins, self.image,
                                 self.aux if npl else None, self.ws, stream)
            except GsError as e:
                if e.status != GS_ERR_CAPACITY:
                    raise
                self._alloc_bins(int(e.n_keys * 1.25) + 1024)
        raise GsError(GS_ERR_CAPACITY, "capacity still short after growing")


def camera_stub(width: int, height: int):
    class _C:
        pass
    c = _C()
    c.R = np.eye(3, dtype=np.float32)
    c.t = np.zeros(3, np.float32)
    c.fx = c.fy = float(width)
    c.cx, c.cy = width / 2.0, height / 2.0
    c.width, c.height, c.znear = width, height, 0.2
    return camera(c)
