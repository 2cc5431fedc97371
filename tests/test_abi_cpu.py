"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects invalid calls on the host before any HIP call."""
import ctypes as C
import os
import re

import pytest

from paper_2605_17855_amd import gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = gs.lib()
    names = declared_functions()
    assert "gs_render" in names and "gs_rasterize" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(gs.EXPORTS)


def test_status_strings():
    L = gs.lib()
    assert L.gs_status_string(gs.GS_OK) == b"ok"
    assert L.gs_status_string(gs.GS_ERR_CAPACITY) == b"capacity exceeded"


def _cam(w=64, h=48):
    return gs.camera_stub(w, h)


def test_num_bins():
    L = gs.lib()
    c = _cam(1920, 1080)
    assert L.gs_num_bins(C.byref(c), 1) == 120 * 68
    assert L.gs_num_bins(C.byref(c), 2) == 60 * 34
    assert L.gs_num_bins(C.byref(c), 4) == 30 * 17
    assert L.gs_num_bins(C.byref(c), 8) == 15 * 9
    assert L.gs_num_bins(None, 1) == 0


@pytest.mark.parametrize("field,value,status", [
    ("group", 0, gs.GS_ERR_INVALID_ARG),
    ("group", 3, gs.GS_ERR_UNSUPPORTED),
    ("group", 16, gs.GS_ERR_UNSUPPORTED),
    ("precision", 7, gs.GS_ERR_INVALID_ARG),
    ("splits", 0, gs.GS_ERR_INVALID_ARG),
    ("aux_flags", 32, gs.GS_ERR_INVALID_ARG),
    ("aux_flags", 64, gs.GS_ERR_INVALID_ARG),
    ("flags", 16, gs.GS_ERR_INVALID_ARG),
    ("flags", 0x80000000, gs.GS_ERR_INVALID_ARG),
])
def test_rasterize_rejects_bad_options(field, value, status):
    L = gs.lib()
    o = gs.options(precision="fp16")
    setattr(o, field, value)
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    img = C.c_void_p(1)
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(o), img, None, None) == status
    assert L.gs_last_error()


def test_group_eight_needs_mfma():
    L = gs.lib()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    o = gs.options(precision="fp32", group=8)
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(o), C.c_void_p(1), None,
                          None) == gs.GS_ERR_UNSUPPORTED
    assert b"MFMA" in L.gs_last_error()


def test_fp16_three_splits_unsupported():
    L = gs.lib()
    o = gs.options(precision="fp16", splits=3)
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(o), C.c_void_p(1), None,
                          None) == gs.GS_ERR_UNSUPPORTED


@pytest.mark.parametrize("w,h,status", [(0, 10, gs.GS_ERR_INVALID_ARG), (10, -1, gs.GS_ERR_INVALID_ARG),
                                        (16385, 10, gs.GS_ERR_UNSUPPORTED)])
def test_rasterize_rejects_bad_camera(w, h, status):
    L = gs.lib()
    c = _cam()
    c.width, c.height = w, h
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(c), C.byref(gs.options()), C.c_void_p(1), None,
                          None) == status


def test_camera_value_checks():
    L = gs.lib()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    for field, value in (("fx", 0.0), ("fy", -1.0), ("znear", 0.0), ("fx", float("nan"))):
        c = _cam()
        setattr(c, field, value)
        assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(c), C.byref(gs.options()), C.c_void_p(1), None,
                              None) == gs.GS_ERR_INVALID_ARG, field


def test_null_arguments():
    L = gs.lib()
    o = gs.options()
    c = _cam()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    assert L.gs_rasterize(None, C.byref(b), C.byref(c), C.byref(o), C.c_void_p(1), None, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_rasterize(C.byref(p), None, C.byref(c), C.byref(o), C.c_void_p(1), None, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_rasterize(C.byref(p), C.byref(b), None, C.byref(o), C.c_void_p(1), None, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(c), None, C.c_void_p(1), None, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(c), C.byref(o), None, None, None) == gs.GS_ERR_INVALID_ARG
    o2 = gs.options(aux_flags=gs.GS_AUX_TFINAL)
    assert L.gs_rasterize(C.byref(p), C.byref(b), C.byref(c), C.byref(o2), C.c_void_p(1), None,
                          None) == gs.GS_ERR_INVALID_ARG
    # grouped rasterization needs the mask array
    b2 = gs.gs_bins(1, 1, None, 16, 1)
    assert L.gs_rasterize(C.byref(p), C.byref(b2), C.byref(c), C.byref(gs.options(group=2)), C.c_void_p(1), None,
                          None) == gs.GS_ERR_INVALID_ARG


def test_scene_checks():
    L = gs.lib()
    o = gs.options()
    c = _cam()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    ws = C.c_void_p(1)
    for n, deg, status in ((-1, 0, gs.GS_ERR_INVALID_ARG), (1 << 31, 0, gs.GS_ERR_UNSUPPORTED),
                           (10, 4, gs.GS_ERR_UNSUPPORTED), (10, -1, gs.GS_ERR_INVALID_ARG)):
        s = gs.gs_scene(n, deg, 0, 1, 1, 1, 1, 1)
        assert L.gs_preprocess(C.byref(s), C.byref(c), C.byref(o), C.byref(p), ws, 1 << 20, None) == status
    s = gs.gs_scene(10, 0, 0, 1, 1, None, 1, 1)
    assert L.gs_preprocess(C.byref(s), C.byref(c), C.byref(o), C.byref(p), ws, 1 << 20,
                           None) == gs.GS_ERR_INVALID_ARG
    # the SH coefficients are read as 16-byte vectors
    s = gs.gs_scene(10, 3, 0, 1, 1, 1, 1, 20)
    assert L.gs_preprocess(C.byref(s), C.byref(c), C.byref(o), C.byref(p), ws, 1 << 20,
                           None) == gs.GS_ERR_INVALID_ARG
    assert b"aligned" in L.gs_last_error()
    # workspace too small
    s = gs.gs_scene(100000, 0, 0, 1, 1, 1, 1, 16)
    assert L.gs_preprocess(C.byref(s), C.byref(c), C.byref(o), C.byref(p), ws, 8, None) == gs.GS_ERR_INVALID_ARG
    assert b"workspace" in L.gs_last_error()


def test_sort_argument_checks():
    L = gs.lib()
    assert L.gs_radix_sort_u64(None, None, 5, 0, 64, C.c_void_p(1), 1 << 20, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_radix_sort_u64(C.c_void_p(1), C.c_void_p(1), 5, 10, 5, C.c_void_p(1), 1 << 20,
                               None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_radix_sort_u64(C.c_void_p(1), C.c_void_p(1), 5, 0, 65, C.c_void_p(1), 1 << 20,
                               None) == gs.GS_ERR_INVALID_ARG
    # n <= 1 is already sorted: no device work, no workspace needed
    assert L.gs_radix_sort_u64(C.c_void_p(1), C.c_void_p(1), 1, 0, 64, None, 0, None) == gs.GS_OK


def test_workspace_sizes_grow_with_inputs():
    L = gs.lib()
    c = _cam(1920, 1080)
    o = gs.options()
    a = L.gs_workspace_bytes(1000, 1000, C.byref(c), C.byref(o))
    b = L.gs_workspace_bytes(1000, 100000, C.byref(c), C.byref(o))
    assert b > a >= 1000 * 12
    assert L.gs_sort_workspace_bytes(1 << 20) >= (1 << 20) * 12


def test_batch_argument_checks():
    L = gs.lib()
    assert L.gs_max_batch() == 32
    o = gs.options()
    jobs = (gs.gs_job * 40)()
    counter = C.c_void_p(1)
    assert L.gs_rasterize_batch(jobs, 0, C.byref(o), counter, None) == gs.GS_OK
    assert L.gs_rasterize_batch(jobs, -1, C.byref(o), counter, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_rasterize_batch(jobs, 33, C.byref(o), counter, None) == gs.GS_ERR_UNSUPPORTED
    assert L.gs_rasterize_batch(None, 2, C.byref(o), counter, None) == gs.GS_ERR_INVALID_ARG
    # a job without projected records is rejected before any device work
    jobs[0].cam = _cam()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    jobs[0].bins = C.pointer(b)
    assert L.gs_rasterize_batch(jobs, 1, C.byref(o), counter, None) == gs.GS_ERR_INVALID_ARG
    jobs[0].proj = C.pointer(p)
    jobs[0].image = None
    assert L.gs_rasterize_batch(jobs, 1, C.byref(o), counter, None) == gs.GS_ERR_INVALID_ARG
    bad = gs.options(group=3)
    assert L.gs_rasterize_batch(jobs, 1, C.byref(bad), counter, None) == gs.GS_ERR_UNSUPPORTED


def test_rasterizer_operands_rounded_from_fp32(tmp_path):
    """The MFMA rasterizer's FP16/BF16 operands are rounded from materialised FP32 values: the
    gfx950 code holds no mixed-precision FMA with a 16-bit result (those round once, straight
    from the unrounded product, and the compiler may form them in one kernel and not another,
    so the grouped, ungrouped and batched rasterizers would disagree)."""
    import re
    import subprocess
    from paper_2605_17855_amd import build
    src = os.path.join(build.CSRC, "gs_raster_mfma.hip")
    out = tmp_path / "raster.s"
    flags = [f for f in build.FLAGS]
    r = subprocess.run([build.HIPCC, *flags, "--offload-device-only", "-S", "-c", src, "-o", str(out)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    assert "v_mfma_f32_32x32x16_f16" in asm
    assert not re.search(r"v_(fma|mad)_mix(lo|hi)_(f16|bf16)", asm)


def test_backward_rejects_invalid_calls():
    """gs_rasterize_backward validates on the host: group bins, NULL buffers, bad camera."""
    L = gs.lib()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    b = gs.gs_bins(1, 1, 1, 16, 1)
    g = gs.gs_grads(1, 1, 1, 1)
    d = C.c_void_p(1)
    call = L.gs_rasterize_backward
    assert call(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(gs.options(group=2)), d, C.byref(g),
                None) == gs.GS_ERR_UNSUPPORTED
    assert b"tile bins" in L.gs_last_error()
    assert call(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(gs.options()), None, C.byref(g),
                None) == gs.GS_ERR_INVALID_ARG
    assert call(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(gs.options()), d, None, None) == gs.GS_ERR_INVALID_ARG
    g0 = gs.gs_grads(1, None, 1, 1)
    assert call(C.byref(p), C.byref(b), C.byref(_cam()), C.byref(gs.options()), d, C.byref(g0),
                None) == gs.GS_ERR_INVALID_ARG
    assert b"gradient" in L.gs_last_error()
    p0 = gs.gs_projected(1, None, 1, 1, 1, 1, 1, 1)
    assert call(C.byref(p0), C.byref(b), C.byref(_cam()), C.byref(gs.options()), d, C.byref(g),
                None) == gs.GS_ERR_INVALID_ARG
    c = _cam()
    c.width = 0
    assert call(C.byref(p), C.byref(b), C.byref(c), C.byref(gs.options()), d, C.byref(g), None) == gs.GS_ERR_INVALID_ARG


def test_python_constants_match_header():
    """The binding's copies of the header's sizes and flags."""
    import re
    hdr = open(os.path.join(ROOT, "include", "gs.h")).read()
    defs = dict(re.findall(r"#define (GS_[A-Z_]+) (\d+)", hdr))
    assert int(defs["GS_BATCH_COUNTER_BYTES"]) == gs.GS_BATCH_COUNTER_BYTES
    assert gs.BATCH_COUNTER_WORDS * 4 == gs.GS_BATCH_COUNTER_BYTES
    assert int(defs["GS_NOALLOC_SCRATCH_BYTES"]) >= gs.GS_BATCH_COUNTER_BYTES
    # the option flags
    enum = dict(re.findall(r"\b(GS_OPT_[A-Z_]+) = (\d+)u", hdr))
    assert {k: int(v) for k, v in enum.items()} == {k: getattr(gs, k) for k in enum}
    assert set(enum) == {"GS_OPT_TIGHT", "GS_OPT_ALL_ROWS", "GS_OPT_TILE_ROWS", "GS_OPT_DEVICE_COUNTS"}


def test_device_counts_argument_checks():
    """With GS_OPT_DEVICE_COUNTS n_keys may be NULL (the count stays on the device) and the
    capacity must fit the device's 32-bit entry count; without it n_keys is required.  All of it
    is decided on the host, before any HIP call (a tiny workspace is the first check after)."""
    L = gs.lib()
    c = _cam()
    p = gs.gs_projected(1, 1, 1, 1, 1, 1, 1, 1)
    s = gs.gs_scene(10, 0, 0, 1, 1, 1, 1, 16)
    ws = C.c_void_p(1)
    dev = gs.options(device_counts=True)
    assert dev.flags == gs.GS_OPT_DEVICE_COUNTS
    b = gs.gs_bins(1, 1, 1, 1 << 20, 1)
    nk = C.c_uint64(0)
    for opt, n_keys, status, msg in ((gs.options(), None, gs.GS_ERR_INVALID_ARG, b"n_keys"),
                                     (dev, None, gs.GS_ERR_INVALID_ARG, b"workspace"),
                                     (dev, C.byref(nk), gs.GS_ERR_INVALID_ARG, b"workspace")):
        assert L.gs_bin_sort(C.byref(p), 10, C.byref(c), C.byref(opt), C.byref(b), n_keys, ws, 8,
                             None) == status
        assert msg in L.gs_last_error()
        assert L.gs_render(C.byref(s), C.byref(c), C.byref(opt), C.byref(p), C.byref(b), C.c_void_p(1), None, n_keys,
                           ws, 8, None) == status
        assert msg in L.gs_last_error()
    big = gs.gs_bins(1, 1, 1, 1 << 32, 1)
    assert L.gs_bin_sort(C.byref(p), 10, C.byref(c), C.byref(dev), C.byref(big), None, ws, 8,
                         None) == gs.GS_ERR_UNSUPPORTED
    assert b"2^32" in L.gs_last_error()
    assert L.gs_render(C.byref(s), C.byref(c), C.byref(dev), C.byref(p), C.byref(big), C.c_void_p(1), None, None, ws,
                       8, None) == gs.GS_ERR_UNSUPPORTED
