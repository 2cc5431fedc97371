"""GPU parity tests: the HIP library against the FP64 oracle (and, for the sort, against a
library stable sort of the same seeded keys).  All calls go through the C ABI binding."""
import ctypes as C
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2605_17855_amd import gs, scenes
from gpu_helpers import check_flagged_pixels, bins_numpy, check_bins, note, projected_numpy, psnr, render, sampled_tiles, tile_mask

pytestmark = pytest.mark.gpu

AUX_ALL = gs.GS_AUX_TFINAL | gs.GS_AUX_WSUM | gs.GS_AUX_NEVAL


@pytest.fixture(scope="module")
def small():
    sc, cam = scenes.small_camera_space()
    ref = oracle.render(sc, cam)
    return sc, cam, ref, gs.DeviceScene(sc)


@pytest.fixture(scope="module")
def big():
    note("build 1M-Gaussian 1080p scene and its oracle records")
    sc, cam = scenes.clustered_1m()
    rec = oracle.preprocess(sc, cam)
    return sc, cam, rec, gs.DeviceScene(sc)


def _compare_records(rec, gp, amb_ok):
    vis_o = rec["visible"]
    vis_g = gp["count"] > 0
    amb = (rec["flags"] & (oracle.AMB_ZNEAR | oracle.AMB_EDGES)) != 0
    assert np.array_equal(vis_o[~amb], vis_g[~amb])
    assert amb.sum() <= amb_ok
    both = vis_o & vis_g & ~amb
    assert both.sum() > 0
    assert np.abs(gp["xy"][both] - rec["xy"][both]).max() < 1e-7
    a, b, c = (rec["conic"][both, i] for i in range(3))
    ga, gb, gc = (gp["conic"][both, i].astype(np.float64) for i in range(3))
    scale = np.sqrt(a * c)
    assert (np.abs(ga - a) / a).max() < 2e-5
    assert (np.abs(gc - c) / c).max() < 2e-5
    assert (np.abs(gb - b) / scale).max() < 2e-5
    assert np.abs(gp["rgb"][both, :3] - rec["rgb"][both]).max() < 2e-5
    assert (np.abs(gp["rgb"][both, 3] - rec["depth"][both]) / rec["depth"][both]).max() < 1e-7
    assert np.array_equal(gp["rect"][both], rec["rect"][both])
    r = rec["rect"][both]
    assert np.array_equal(gp["count"][both], (r[:, 2] - r[:, 0]) * (r[:, 3] - r[:, 1]))
    assert int(gp["offset"][-1]) == int(gp["count"].astype(np.uint64).sum())


def test_preprocess_small(small):
    sc, cam, ref, ds = small
    note("preprocess parity 4096 / 128x128")
    out = render(ds, cam)
    gp = projected_numpy(out["renderer"])
    _compare_records(ref["records"], gp, amb_ok=10)
    assert out["n_keys"] == int(gp["offset"][-1])


def test_preprocess_1m_1080p(big):
    sc, cam, rec, ds = big
    note("preprocess parity 1M / 1920x1080")
    out = render(ds, cam, precision="fp16")
    gp = projected_numpy(out["renderer"])
    _compare_records(rec, gp, amb_ok=2000)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 2047, 2048, 2049, 100_003, 3_000_000])
def test_radix_sort_bit_exact(n):
    import torch
    note(f"radix sort n={n}")
    keys, vals = scenes.random_keys(n, seed=100 + n % 97)
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    gs.gs_radix_sort_u64(kd, vd, 0, 45)
    torch.cuda.synchronize()
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), keys[order])
    assert np.array_equal(vd.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("lo,hi", [(0, 8), (3, 17), (32, 45), (0, 64)])
def test_radix_sort_bit_ranges(lo, hi):
    import torch
    note(f"radix sort bits [{lo},{hi})")
    rng = np.random.default_rng(lo * 100 + hi)
    n = 50_001
    keys = rng.integers(0, 1 << 62, n, dtype=np.uint64) * np.uint64(3)
    vals = np.arange(n, dtype=np.uint32)
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    gs.gs_radix_sort_u64(kd, vd, lo, hi)
    torch.cuda.synchronize()
    field = (keys >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1 if hi - lo < 64 else 0xFFFFFFFFFFFFFFFF)
    order = np.argsort(field, kind="stable")
    assert np.array_equal(vd.cpu().numpy().view(np.uint32), vals[order])


@pytest.mark.parametrize("lo,hi,n", [(0, 9, 1_500_001), (32, 41, 2_100_000), (3, 12, 1_048_577)])
def test_radix_sort_nine_bit_single_pass(lo, hi, n):
    """Above 2^20 keys a 9-bit range is sorted in one pass of 512 digits (the bins of 4x4 groups
    at 1080p): bit-exact against a stable argsort, duplicates included."""
    import torch
    note(f"radix sort {n} keys, bits [{lo},{hi})")
    rng = np.random.default_rng(lo * 1000 + hi + n)
    keys = rng.integers(0, 1 << 62, n, dtype=np.uint64)
    keys[rng.random(n) < 0.3] = np.uint64(12345) << np.uint64(lo)   # a heavy duplicate digit
    vals = np.arange(n, dtype=np.uint32)
    kd = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vd = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    gs.gs_radix_sort_u64(kd, vd, lo, hi)
    torch.cuda.synchronize()
    field = (keys >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1)
    order = np.argsort(field, kind="stable")
    assert np.array_equal(vd.cpu().numpy().view(np.uint32), vals[order])
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), keys[order])


@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_bin_sort_small(small, group):
    sc, cam, ref, ds = small
    note(f"bin sort 4096 / 128x128 group {group}")
    out = render(ds, cam, group=group, precision="fp16")
    check_bins(ref["records"], cam, out["renderer"], out["n_keys"], group)


@pytest.mark.parametrize("group", [1, 2, 8])
def test_bin_sort_1m(big, group):
    sc, cam, rec, ds = big
    note(f"bin sort 1M / 1080p group {group}")
    out = render(ds, cam, group=group, precision="fp16")
    check_bins(rec, cam, out["renderer"], out["n_keys"], group)


def test_fp32_image_small(small):
    sc, cam, ref, ds = small
    note("fp32 image 4096 / 128x128")
    out = render(ds, cam, precision="fp32", aux=AUX_ALL)
    ok = ref["ambiguous"] == 0
    assert ok.mean() > 0.999
    err = np.abs(out["image"] - ref["image"])
    assert err[:, ok].max() <= 1e-4, err[:, ok].max()
    assert np.abs(out["tfinal"] - ref["tfinal"])[ok].max() <= 1e-5
    assert np.abs(out["wsum"] + out["tfinal"] - 1.0).max() <= 1e-5
    assert np.array_equal(out["neval"][ok], ref["neval"][ok].astype(np.float64))
    check_flagged_pixels("fp32 small", out["image"], out["tfinal"], ref, ref["records"], cam, ref["start"],
                         ref["ids"])


@pytest.mark.parametrize("prec,splits,required", [("fp16", 1, False), ("fp16", 2, True), ("bf16", 1, False),
                                                  ("bf16", 2, False), ("bf16", 3, True)])
def test_mfma_image_small(small, prec, splits, required):
    sc, cam, ref, ds = small
    note(f"mfma image {prec} splits {splits} 4096 / 128x128")
    out = render(ds, cam, precision=prec, splits=splits, aux=AUX_ALL)
    p = psnr(out["image"], ref["image"])
    mae = float(np.mean(np.abs(out["image"] - ref["image"])))
    print(f"{prec} splits={splits}: PSNR {p:.2f} dB, MAE {mae:.3e}, max abs "
          f"{np.abs(out['image'] - ref['image']).max():.3e}")
    assert np.abs(out["wsum"] + out["tfinal"] - 1.0).max() <= 1e-5
    if required:
        assert p >= 45.0 and mae <= 2e-3


@pytest.mark.parametrize("prec,splits", [("fp16", 2), ("bf16", 3), ("fp16", 1)])
@pytest.mark.parametrize("size", [(128, 128), (100, 70)])
def test_grouping_bit_identical(prec, splits, size):
    """Per-member-tile rows (GS_OPT_TILE_ROWS; always for the frames the group-frame operand
    cannot hold exactly): every grouped image and aux plane equals the 1x1 one bit for bit."""
    sc, _ = scenes.small_camera_space()
    cam = scenes.pinhole(size[0], size[1], 60.0)
    ds = gs.DeviceScene(sc)
    note(f"grouping identity {prec}/{splits} {size}")
    base = render(ds, cam, group=1, precision=prec, splits=splits, aux=AUX_ALL | gs.GS_AUX_LAST)
    for g in (2, 4, 8):
        out = render(ds, cam, group=g, precision=prec, splits=splits, aux=AUX_ALL | gs.GS_AUX_LAST, tile_rows=True)
        for k in ("image", "tfinal", "wsum", "neval", "last"):
            assert np.array_equal(out[k], base[k]), (g, k)


@pytest.mark.parametrize("prec,splits,group", [("fp16", 2, 2), ("bf16", 3, 2)])
@pytest.mark.parametrize("size", [(128, 128), (100, 70)])
def test_group_frame_rows_match_oracle(small, prec, splits, group, size):
    """Rows built once per group (the default for 2x2 groups): the image against
    the FP64 oracle (PSNR >= 45 dB, MAE <= 2e-3, max abs <= 1e-3 outside the guard bands and an
    admissible result within 1e-3 inside them), W + T_final = 1, and the evaluation and
    blended-prefix counts equal to the 1x1 render's wherever no decision is in a guard band."""
    sc, _, _, _ = small
    cam = scenes.pinhole(size[0], size[1], 60.0)
    ref = oracle.render(sc, cam)
    ok = ref["ambiguous"] == 0
    ds = gs.DeviceScene(sc)
    note(f"group-frame rows {prec}/{splits} group {group} {size}")
    aux = AUX_ALL | gs.GS_AUX_LAST
    base = render(ds, cam, group=1, precision=prec, splits=splits, aux=aux)
    out = render(ds, cam, group=group, precision=prec, splits=splits, aux=aux)
    err = np.abs(out["image"] - ref["image"])
    p = psnr(out["image"], ref["image"])
    print(f"group frame {prec}/{splits} G{group} {size}: PSNR {p:.2f} dB, MAE {err.mean():.3e}, max abs "
          f"{err[:, ok].max():.3e}, vs 1x1 max abs {np.abs(out['image'] - base['image']).max():.3e}")
    assert p >= 45.0 and err.mean() <= 2e-3 and err[:, ok].max() <= 1e-3
    assert np.abs(out["wsum"] + out["tfinal"] - 1.0).max() <= 1e-5
    assert np.abs(out["tfinal"] - ref["tfinal"])[ok].max() <= 2e-3
    check_flagged_pixels(f"group frame {prec} G{group} {size}", out["image"], out["tfinal"], ref, ref["records"], cam,
                         ref["start"], ref["ids"], tol=1e-3, tol_t=2e-3)
    for k in ("neval", "last"):
        assert np.array_equal(out[k][ok], base[k][ok]), k


def test_fp32_grouped_matches_oracle(small):
    sc, cam, ref, ds = small
    ok = ref["ambiguous"] == 0
    for g in (2, 4):
        note(f"fp32 grouped {g}")
        out = render(ds, cam, group=g, precision="fp32")
        assert np.abs(out["image"] - ref["image"])[:, ok].max() <= 1e-4
        check_flagged_pixels(f"fp32 group {g}", out["image"], None, ref, ref["records"], cam, ref["start"],
                             ref["ids"])


def test_determinism(small):
    sc, cam, ref, ds = small
    note("determinism")
    a = render(ds, cam, precision="fp16", aux=AUX_ALL)
    b = render(ds, cam, precision="fp16", aux=AUX_ALL)
    assert np.array_equal(a["image"], b["image"]) and np.array_equal(a["neval"], b["neval"])
    c = render(ds, cam, precision="fp32")
    d = render(ds, cam, precision="fp32")
    assert np.array_equal(c["image"], d["image"])


def test_empty_and_culled_scenes():
    cam = scenes.pinhole(80, 48, 60.0)
    bg = (0.25, 0.5, 0.75)
    sc = scenes.camera_box_scene(0, seed=1)
    note("empty scene")
    for prec in ("fp32", "fp16"):
        out = render(gs.DeviceScene(sc), cam, precision=prec, bg=bg)
        assert out["n_keys"] == 0
        assert np.allclose(out["image"], np.asarray(bg)[:, None, None])
    # everything behind the camera
    sc = scenes.camera_box_scene(500, seed=2)
    sc.mean[2] *= -1.0
    note("culled scene")
    out = render(gs.DeviceScene(sc), cam, precision="fp16", bg=bg)
    assert out["n_keys"] == 0
    assert np.allclose(out["image"], np.asarray(bg)[:, None, None])


@pytest.mark.parametrize("size", [(1, 1), (17, 33), (100, 70), (250, 16)])
def test_ragged_sizes(size):
    sc = scenes.camera_box_scene(1500, seed=9)
    cam = scenes.pinhole(size[0], size[1], 60.0)
    ref = oracle.render(sc, cam, bg=(0.1, 0.2, 0.3))
    ds = gs.DeviceScene(sc)
    ok = ref["ambiguous"] == 0
    for prec, tol in (("fp32", 1e-4), ("fp16", 2e-3)):
        note(f"ragged {size} {prec}")
        out = render(ds, cam, precision=prec, bg=(0.1, 0.2, 0.3))
        assert out["image"].shape == (3, size[1], size[0])
        assert np.abs(out["image"] - ref["image"])[:, ok].max() <= tol
        check_flagged_pixels(f"ragged {size} {prec}", out["image"], None, ref, ref["records"], cam, ref["start"],
                             ref["ids"], bg=(0.1, 0.2, 0.3), tol=tol)


def test_single_gaussian():
    cam = scenes.pinhole(64, 64, 60.0)
    sc = scenes.Scene(np.array([[0.01], [-0.02], [2.0]], np.float32), np.full((3, 1), math.log(0.05), np.float32),
                      np.array([[0.9], [0.1], [0.3], [-0.2]], np.float32), np.array([0.8], np.float32),
                      np.array([[[0.4], [0.1], [-0.2]]], np.float32), 0)
    ref = oracle.render(sc, cam)
    ds = gs.DeviceScene(sc)
    for prec in ("fp32", "fp16", "bf16"):
        note(f"single gaussian {prec}")
        out = render(ds, cam, precision=prec, splits=3 if prec == "bf16" else 2)
        tol = 1e-4 if prec == "fp32" else 2e-3
        assert np.abs(out["image"] - ref["image"]).max() <= tol


def test_capacity_error_reports_count(small):
    import torch
    sc, cam, ref, ds = small
    note("capacity error")
    r = gs.Renderer(ds.n, cam.width, cam.height, capacity=100)
    opt = gs.options()
    with pytest.raises(gs.GsError) as ei:
        gs.gs_render(ds, cam, opt, r.proj, r.bins, r.image, None, r.ws)
    assert ei.value.status == gs.GS_ERR_CAPACITY
    assert ei.value.n_keys == int(ref["start"][-1])
    torch.cuda.synchronize()


def test_1080psampled_tiles(big):
    sc, cam, rec, ds = big
    tiles = sampled_tiles(cam, 400, 7)
    st, ids, _ = oracle.lists(rec, cam, 1)
    ref = oracle.composite(rec, cam, st, ids, nthreads=8, tiles=tiles)
    m = tile_mask(cam, tiles)
    ok = m & (ref["ambiguous"] == 0)
    for prec, splits in (("fp32", 2), ("fp16", 2), ("bf16", 3)):
        note(f"1080p sampled tiles {prec}")
        out = render(ds, cam, precision=prec, splits=splits, aux=AUX_ALL)
        err = np.abs(out["image"] - ref["image"])
        p = psnr(out["image"][:, m], ref["image"][:, m])
        mae = float(err[:, m].mean())
        print(f"1080p {prec}: max abs {err[:, ok].max():.3e}, PSNR {p:.2f}, MAE {mae:.3e}, "
              f"neval match {(out['neval'][ok] == ref['neval'][ok]).mean():.5f}")
        assert p >= 45.0 and mae <= 2e-3
        if prec == "fp32":
            assert err[:, ok].max() <= 1e-4
        check_flagged_pixels(f"1080p {prec}", out["image"], out["tfinal"], ref, rec, cam, st, ids, mask=m,
                             tol=1e-4 if prec == "fp32" else 1e-3, tol_t=1e-5 if prec == "fp32" else 2e-3)
        assert np.abs(out["wsum"] + out["tfinal"] - 1.0).max() <= 1e-5


_BATCH_REFS = {}


def _batch_oracle(k, sc, cam, bg):
    """The FP64 oracle's render of batch job k (computed once per module)."""
    if k not in _BATCH_REFS:
        _BATCH_REFS[k] = oracle.render(sc, cam, bg=bg)
    return _BATCH_REFS[k]


@pytest.mark.parametrize("prec,group", [("fp16", 1), ("fp32", 1), ("bf16", 2), ("fp16", 2), ("fp16", 8)])
def test_batch_matches_single_renders(prec, group):
    """Persistent batched rasterization: every image equals rendering its job alone (bit-identical),
    and every batched image and its T_final plane meet the oracle's bars (flagged pixels: one of
    their admissible results)."""
    import torch
    jobs = []
    specs = [(scenes.camera_box_scene(3000, seed=21), scenes.pinhole(128, 96, 60.0)),
             (scenes.camera_box_scene(1500, seed=22), scenes.pinhole(70, 33, 50.0)),
             (scenes.clustered_scene(20000, seed=23, clusters=8), scenes.look_at([3.0, 1.0, 1.5], 160, 90)),
             (scenes.camera_box_scene(10, seed=24), scenes.pinhole(16, 16, 60.0))]
    aux = AUX_ALL | gs.GS_AUX_NBLEND
    opt = gs.options(group=group, precision=prec, splits=3 if prec == "bf16" else 2, bg=(0.2, 0.1, 0.0),
                     aux_flags=aux)
    singles = []
    for sc, cam in specs:
        ds = gs.DeviceScene(sc)
        r = gs.Renderer(sc.n, cam.width, cam.height, group=group)
        note(f"batch reference {prec} g{group} {cam.width}x{cam.height}")
        r.render(ds, cam, opt)
        torch.cuda.synchronize()
        singles.append((r.image.clone(), r.aux.clone()))
        img = torch.full_like(r.image, -1.0)
        ax = torch.full_like(r.aux, -1.0)
        jobs.append((r.proj, r.bins, cam, img, ax, r, ds))
    counter = torch.zeros(gs.BATCH_COUNTER_WORDS, dtype=torch.int32, device="cuda")
    note(f"batch launch {prec} g{group}")
    gs.gs_rasterize_batch([(j[0], j[1], j[2], j[3], j[4]) for j in jobs], opt, counter)
    torch.cuda.synchronize()
    for (img, ax), j in zip(singles, jobs):
        assert torch.equal(img, j[3]) and torch.equal(ax, j[4])
    bg = (0.2, 0.1, 0.0)
    tol, tol_t = (1e-4, 1e-5) if prec == "fp32" else (1e-3, 2e-3)
    for k, ((sc, cam), j) in enumerate(zip(specs, jobs)):
        ref = _batch_oracle(k, sc, cam, bg)
        img = j[3].double().cpu().numpy()
        tf = j[4][0].double().cpu().numpy()
        ok = ref["ambiguous"] == 0
        err = np.abs(img - ref["image"])[:, ok]
        assert (err.max() if err.size else 0.0) <= tol, (k, float(err.max()))
        assert np.abs(tf - ref["tfinal"])[ok].max() <= tol_t
        check_flagged_pixels(f"batch {prec} g{group} job {k}", img, tf, ref, ref["records"], cam, ref["start"],
                             ref["ids"], bg=bg, tol=tol, tol_t=tol_t)
    # the same jobs twice in one launch, in another order
    order = [2, 0, 3, 1, 2]
    outs = [(torch.full_like(jobs[k][3], -1.0), torch.full_like(jobs[k][4], -1.0)) for k in order]
    gs.gs_rasterize_batch([(jobs[k][0], jobs[k][1], jobs[k][2], o[0], o[1]) for k, o in zip(order, outs)], opt,
                          counter)
    torch.cuda.synchronize()
    for k, o in zip(order, outs):
        assert torch.equal(o[0], singles[k][0]) and torch.equal(o[1], singles[k][1])


def test_ply_scene_renders_like_its_source(tmp_path):
    """A scene written and read back in the trained-scene PLY layout renders as the original
    (opacity and quaternion pass through logit/normalisation, so equal up to rounding)."""
    from paper_2605_17855_amd import ply
    sc = scenes.clustered_scene(20000, seed=23, clusters=8)
    cam = scenes.look_at([3.0, 1.0, 1.5], 160, 90)
    ply.save_ply(sc, str(tmp_path / "s.ply"))
    back = ply.load_ply(str(tmp_path / "s.ply"))
    note("ply round trip render")
    a = render(gs.DeviceScene(sc), cam, precision="fp16")
    b = render(gs.DeviceScene(back), cam, precision="fp16")
    assert psnr(a["image"], b["image"]) >= 90.0


@pytest.mark.parametrize("n", [5000, 1 << 20, (1 << 20) + 1, 17_000_000])
def test_count_scan_and_compaction(n):
    """The preprocess's count scan and visible-list compaction, bit-exact against a host
    cumulative sum of the same counts: one-tile, 2^20 (1,024-value tiles), just above (4,096-
    value tiles), and 17M values (more than 4,096 tiles: the tile sums are scanned by one
    workgroup first).  Degree-0 splats in front of a small camera, most of them visible."""
    import torch
    rng = np.random.default_rng(3)
    sc = scenes.camera_box_scene(n, seed=4) if n <= 5000 else None
    if sc is None:
        sc = scenes.Scene(np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)]).astype(np.float32),
                          np.full((3, n), np.log(0.01), np.float32), np.tile(np.array([[1], [0], [0], [0]], np.float32), (1, n)),
                          np.full(n, 0.5, np.float32), np.zeros((1, 3, n), np.float32), 0)
        sc.mean[2, ::7] = -1.0      # some behind the camera
    cam = scenes.pinhole(64, 48, 60.0)
    note(f"count scan n={n}")
    ds = gs.DeviceScene(sc)
    proj = gs.Projected(n)
    opt = gs.options()
    c = gs.camera_stub(cam.width, cam.height)
    ws = torch.empty((int(gs.lib().gs_workspace_bytes(n, 1024, C.byref(c), C.byref(opt))),), dtype=torch.uint8,
                     device="cuda")
    gs.gs_preprocess(ds, cam, opt, proj, ws)
    torch.cuda.synchronize()
    count = proj.count.cpu().numpy().view(np.uint32)[:n].astype(np.uint64)
    offset = proj.offset.cpu().numpy().view(np.uint64)[: n + 1]
    want = np.zeros(n + 1, np.uint64)
    want[1:] = np.cumsum(count)
    assert np.array_equal(offset, want)
    vis = np.nonzero(count)[0]
    V = int(proj.n_visible.cpu().numpy().view(np.uint32)[0])
    assert V == vis.size and 0 < V < n
    assert np.array_equal(proj.order.cpu().numpy().view(np.uint32)[:V].astype(np.int64), vis)
    del ds, proj, ws
    torch.cuda.empty_cache()


def test_maximum_width():
    """The widest image the library accepts (16,384 pixels: 1,024 tile columns), one tile row
    and a ragged second one, against the oracle."""
    sc = scenes.camera_box_scene(3000, seed=12)
    cam = scenes.pinhole(16384, 24, 120.0)
    ref = oracle.render(sc, cam, bg=(0.1, 0.2, 0.3))
    ok = ref["ambiguous"] == 0
    ds = gs.DeviceScene(sc)
    for prec, tol, group in (("fp32", 1e-4, 1), ("fp16", 2e-3, 1), ("fp16", 2e-3, 8)):
        note(f"maximum width {prec} group {group}")
        out = render(ds, cam, precision=prec, bg=(0.1, 0.2, 0.3), group=group)
        assert out["image"].shape == (3, 24, 16384)
        assert np.abs(out["image"] - ref["image"])[:, ok].max() <= tol
        check_flagged_pixels(f"maximum width {prec} group {group}", out["image"], None, ref, ref["records"], cam,
                             ref["start"], ref["ids"], bg=(0.1, 0.2, 0.3), tol=tol)
