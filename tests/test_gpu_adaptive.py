"""Per-scene (group side, culling) choice on the GPU: with per-member-tile rows every frame equals
the G = 1 render bit for bit (the MFMA rasterizers give the same image for every variant); with
rows built once per group (the default) the grouped frames equal it to the 16-bit operands'
rounding; the probes visit every variant (one per frame in turn, or every variant on each probe
frame's view), and the committed one is the fastest probed."""
import numpy as np
import pytest

from paper_2605_17855_amd import gs, scenes
from paper_2605_17855_amd.adaptive import AdaptiveRenderer
from gpu_helpers import note, render

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,sides,tile_rows", [("fp16", {1, 2, 4, 8}, True), ("fp16", {1, 2, 4, 8}, False),
                                                  ("fp32", {1, 2, 4}, False)])
def test_adaptive_group_choice_keeps_images(prec, sides, tile_rows):
    import torch
    sc = scenes.clustered_scene(20000, seed=23, clusters=8)
    cam = scenes.look_at([3.0, 1.0, 1.5], 320, 180)
    ds = gs.DeviceScene(sc)
    note(f"adaptive groups {prec}")
    ref = render(ds, cam, group=1, precision=prec)["image"]
    ar = AdaptiveRenderer(sc.n, cam.width, cam.height, precision=prec, probes=2, tile_rows=tile_rows, paired=False)
    used = []
    variants = {(g, t) for g in sides for t in (False, True)}
    for _ in range(2 * len(variants) + 4):
        img, (g, _t) = ar.render(ds, cam)
        torch.cuda.synchronize()
        used.append(ar.last_variant)
        if (prec == "fp16" and (tile_rows or g != 2)) or g == 1:
            assert np.array_equal(img.cpu().numpy().astype(np.float64), ref), g
        elif prec == "fp16":   # 2x2 group-frame rows: the operands' rounding against larger phi
            assert np.abs(img.cpu().numpy() - ref).max() <= 1e-3, g
        else:   # FP32 grouped tiles sum in the same order but are compiled separately
            assert np.abs(img.cpu().numpy() - ref).max() <= 1e-5
    assert set(used[:2 * len(variants)]) == variants
    t = ar.chooser.times
    assert ar.chooser.chosen == min(t, key=lambda s: (min(t[s]), s))
    assert all(u == ar.chooser.chosen for u in used[2 * len(variants):])


def _check_image(img, ref, prec, g, tile_rows):
    if (prec == "fp16" and (tile_rows or g != 2)) or g == 1:
        assert np.array_equal(img, ref), g
    elif prec == "fp16":   # 2x2 group-frame rows: the operands' rounding against larger phi
        assert np.abs(img - ref).max() <= 1e-3, g
    else:
        assert np.abs(img - ref).max() <= 1e-5


@pytest.mark.parametrize("prec,tile_rows", [("fp16", False), ("bf16", True)])
def test_adaptive_paired_probes(prec, tile_rows):
    """Paired probing: each probe frame renders its view with every variant (the images of all of
    them checked), then the fastest by its best probe is used for every later frame."""
    import torch
    sc = scenes.clustered_scene(20000, seed=29, clusters=8)
    cams = [scenes.look_at([3.0, 1.0, 1.5], 320, 180), scenes.look_at([-2.5, 2.0, 1.0], 320, 180)]
    ds = gs.DeviceScene(sc)
    note(f"adaptive paired probes {prec}")
    splits = 3 if prec == "bf16" else 2
    refs = [render(ds, c, group=1, precision=prec, splits=splits)["image"] for c in cams]
    ar = AdaptiveRenderer(sc.n, 320, 180, precision=prec, splits=splits, probes=2, tile_rows=tile_rows)
    for i in range(2):
        img, v = ar.render(ds, cams[i])
        torch.cuda.synchronize()
        assert v == ar.variants[-1]
        for g in {vv[0] for vv in ar.variants}:   # every group side's last image is this view's
            im = ar.renderers[g].image.cpu().numpy().astype(np.float64)
            _check_image(im, refs[i], prec, g, tile_rows)
    t = ar.chooser.times
    assert all(len(x) == 2 for x in t.values()) and set(t) == set(ar.variants)
    assert ar.chooser.chosen == min(t, key=lambda s: (min(t[s]), s))
    for i in range(3):
        img, v = ar.render(ds, cams[i % 2])
        torch.cuda.synchronize()
        assert v == ar.chooser.chosen
        _check_image(img.cpu().numpy().astype(np.float64), refs[i % 2], prec, v[0], tile_rows)
