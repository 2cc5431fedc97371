"""Per-scene (group side, culling) choice on the GPU: with per-member-tile rows every frame equals
the G = 1 render bit for bit (the MFMA rasterizers give the same image for every variant); with
rows built once per group (the default) the grouped frames equal it to the 16-bit operands'
rounding; the probes visit every variant, and the committed one is the fastest probed."""
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
    ar = AdaptiveRenderer(sc.n, cam.width, cam.height, precision=prec, probes=2, tile_rows=tile_rows)
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
