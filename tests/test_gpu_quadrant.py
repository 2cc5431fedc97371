"""Quadrant culling in the MFMA rasterizers changes no result: every output (image, final
transmittance, weight sum, evaluation and blend counts) is bit-identical with GS_OPT_ALL_ROWS,
where every wave runs every row of its tile.  A left-out row is one whose alpha misses the
1/255 cut at every pixel centre of the wave's quadrant by a margin of 1 in q (0.72 in log2),
and the 16-bit split operands with 2 or 3 pieces carry ~2^-22 relative error, so equality is
the bar for them.  With one piece (11 or 8 bits) a row whose exact alpha misses the cut could
in principle pass it through operand rounding alone; those cases are reported, not asserted.

Scenes: the 4096-Gaussian camera-space scene (128x128 and a ragged 100x70), a 20k scene with
a wide spread of scales (log-scale sigma 1.5: tiny to very large, elongated footprints), and
the 1M-Gaussian 1080p workload with 1x1 and 4x4 groups and with opacity-aware culling."""
import math

import numpy as np
import pytest

from paper_2605_17855_amd import gs, scenes
from gpu_helpers import note, render

pytestmark = pytest.mark.gpu

AUX = gs.GS_AUX_TFINAL | gs.GS_AUX_WSUM | gs.GS_AUX_NEVAL | gs.GS_AUX_NBLEND
KEYS = ("image", "tfinal", "wsum", "neval", "nblend")


def _pair(ds, cam, **kw):
    a = render(ds, cam, aux=AUX, **kw)
    b = render(ds, cam, aux=AUX, all_rows=True, **kw)
    return a, b


def _assert_same(a, b, tag):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (tag, k, int((a[k] != b[k]).sum()))


@pytest.fixture(scope="module", params=["small128", "small100x70", "wide20k"])
def scene(request):
    if request.param == "wide20k":
        sc = scenes.camera_box_scene(20000, seed=31, log_scale_mu=math.log(0.03), log_scale_sigma=1.5)
        cam = scenes.pinhole(320, 200, 60.0)
    else:
        sc, _ = scenes.small_camera_space()
        cam = scenes.pinhole(128, 128, 60.0) if request.param == "small128" else scenes.pinhole(100, 70, 60.0)
    return request.param, sc, cam, gs.DeviceScene(sc)


@pytest.mark.parametrize("prec,splits", [("fp16", 2), ("bf16", 3), ("bf16", 2)])
@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_quadrant_culling_bit_identical(scene, prec, splits, group):
    name, sc, cam, ds = scene
    note(f"quadrant culling {name} {prec}/{splits} group {group}")
    a, b = _pair(ds, cam, group=group, precision=prec, splits=splits)
    _assert_same(a, b, (name, prec, splits, group))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_quadrant_culling_one_piece_reported(scene, prec):
    name, sc, cam, ds = scene
    note(f"quadrant culling {name} {prec}/1")
    a, b = _pair(ds, cam, group=1, precision=prec, splits=1)
    diff = {k: int((a[k] != b[k]).sum()) for k in KEYS}
    print(f"{name} {prec} splits 1: differing values {diff}")
    assert np.abs(a["wsum"] + a["tfinal"] - 1.0).max() <= 1e-5


def test_quadrant_culling_1m_1080p():
    sc, cam = scenes.clustered_1m()
    ds = gs.DeviceScene(sc)
    for group, tight in ((1, False), (4, False), (8, False), (1, True)):
        note(f"quadrant culling 1M 1080p fp16/2 group {group} tight {tight}")
        a, b = _pair(ds, cam, group=group, precision="fp16", splits=2, tight=tight)
        _assert_same(a, b, (group, tight))
        ev = a["neval"].sum()
        print(f"1M 1080p group {group} tight {tight}: evaluations {ev:.4g}, blends {a['nblend'].sum():.4g}")
