"""Opacity-aware tile culling (GS_OPT_TIGHT), ungrouped and with 2x2, 4x4 and 8x8 groups:
bins (keys, Gaussians, member-tile masks) against the oracle's culled lists, and images, final
transmittance and weight sums bit-identical to rendering the full lists."""
import numpy as np
import pytest

from oracle import oracle
from paper_2605_17855_amd import gs, scenes
from gpu_helpers import check_bins, note, render

pytestmark = pytest.mark.gpu

AUX = gs.GS_AUX_TFINAL | gs.GS_AUX_WSUM | gs.GS_AUX_NEVAL


def _render(ds, cam, prec, tight, splits, group=1):
    import torch
    r = gs.Renderer(ds.n, cam.width, cam.height, group=group)
    opt = gs.options(group=group, precision=prec, splits=splits, aux_flags=AUX, tight=tight)
    n_keys = r.render(ds, cam, opt)
    torch.cuda.synchronize()
    planes = r.aux.cpu().numpy()
    return dict(image=r.image.cpu().numpy(), tfinal=planes[0], wsum=planes[1], neval=planes[2], n_keys=n_keys,
                renderer=r)


@pytest.fixture(scope="module", params=["small", "1m"])
def workload(request):
    if request.param == "small":
        sc, cam = scenes.small_camera_space()
    else:
        note("build 1M-Gaussian scene for tight culling")
        sc, cam = scenes.clustered_1m()
    return sc, cam, oracle.preprocess(sc, cam), gs.DeviceScene(sc)


@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_tight_bins_match_oracle(workload, group):
    sc, cam, rec, ds = workload
    note(f"tight bins {sc.n} group {group}")
    out = _render(ds, cam, "fp16", True, 2, group)
    check_bins(rec, cam, out["renderer"], out["n_keys"], group, tight=True)
    full = _render(ds, cam, "fp16", False, 2, group)
    print(f"{sc.n} G{group}: entries {full['n_keys']} -> {out['n_keys']} ({out['n_keys'] / full['n_keys']:.3f})")
    # small splats lose few footprint tiles; the 1M scene's anisotropic ones about half
    # (fewer with groups, whose entries already cover several tiles each)
    if group == 1:
        assert out["n_keys"] < (0.7 if sc.n > 100_000 else 0.95) * full["n_keys"]
    else:
        assert out["n_keys"] <= full["n_keys"]


@pytest.mark.parametrize("prec,splits,group", [("fp32", 2, 1), ("fp16", 2, 1), ("bf16", 3, 1), ("fp32", 2, 2),
                                              ("fp16", 2, 4), ("bf16", 3, 2), ("fp16", 2, 8)])
def test_tight_image_equals_full_lists(workload, prec, splits, group):
    sc, cam, rec, ds = workload
    note(f"tight image {sc.n} {prec} group {group}")
    full = _render(ds, cam, prec, False, splits, group)
    tight = _render(ds, cam, prec, True, splits, group)
    for k in ("image", "tfinal", "wsum"):
        assert np.array_equal(full[k], tight[k]), k
    assert (tight["neval"] <= full["neval"]).all()
    print(f"{sc.n} {prec} G{group}: evaluations {full['neval'].sum():.4g} -> {tight['neval'].sum():.4g}")
