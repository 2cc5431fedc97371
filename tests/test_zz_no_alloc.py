"""gs_rasterize_batch_noalloc (work counter in the library's own device scratch) against
gs_rasterize_batch (work counter from the caller) on the same prepared jobs: bit-identical
images and auxiliary planes, on two calls in a row, the second with a smaller batch.  Both
launches run the same kernels, so the bar is equality; gs_rasterize_batch itself is held to
single renders, and those to the FP64 oracle, by the other parity tests."""
import numpy as np
import pytest

from paper_2605_17855_amd import gs, scenes
from gpu_helpers import note

pytestmark = pytest.mark.gpu

AUX = gs.GS_AUX_TFINAL | gs.GS_AUX_WSUM | gs.GS_AUX_NEVAL | gs.GS_AUX_NBLEND


def _prepare(specs, opt, group):
    import torch
    jobs = []
    for sc, cam in specs:
        ds = gs.DeviceScene(sc)
        r = gs.Renderer(sc.n, cam.width, cam.height, group=group)
        note(f"noalloc: prepare {cam.width}x{cam.height}, {sc.n} Gaussians, group {group}")
        r.render(ds, cam, opt)
        torch.cuda.synchronize()
        jobs.append((r, ds, cam))
    return jobs


def _launch(jobs, opt, noalloc):
    import torch
    outs = []
    items = []
    for r, _, cam in jobs:
        img = torch.full_like(r.image, -1.0)
        ax = torch.full_like(r.aux, -1.0)
        outs.append((img, ax))
        items.append((r.proj, r.bins, cam, img, ax))
    if noalloc:
        gs.gs_rasterize_batch_noalloc(items, opt)
    else:
        counter = torch.zeros(gs.BATCH_COUNTER_WORDS, dtype=torch.int32, device="cuda")
        gs.gs_rasterize_batch(items, opt, counter)
    torch.cuda.synchronize()
    return [(i.cpu().numpy(), a.cpu().numpy()) for i, a in outs]


@pytest.mark.parametrize("prec,group", [("fp16", 1), ("fp32", 1), ("bf16", 2)])
def test_noalloc_batch_matches_batch(prec, group):
    opt = gs.options(group=group, precision=prec, splits=3 if prec == "bf16" else 2, bg=(0.2, 0.1, 0.0),
                     aux_flags=AUX)
    specs = [(scenes.camera_box_scene(3000, seed=31), scenes.pinhole(128, 96, 60.0)),
             (scenes.clustered_scene(20000, seed=32, clusters=8), scenes.look_at([3.0, 1.0, 1.5], 160, 90)),
             (scenes.camera_box_scene(1500, seed=33), scenes.pinhole(70, 33, 50.0))]
    jobs = _prepare(specs, opt, group)
    # first call: all three jobs; second call: one smaller job (the scratch keeps the first call's
    # counter value, which the call must clear)
    for batch in (jobs, jobs[2:]):
        note(f"noalloc: {prec} group {group}, {len(batch)} jobs, caller counter")
        want = _launch(batch, opt, noalloc=False)
        note(f"noalloc: {prec} group {group}, {len(batch)} jobs, library scratch")
        got = _launch(batch, opt, noalloc=True)
        for (wi, wa), (gi, ga) in zip(want, got):
            # every pixel written (colours, background, T, weights and counts are all >= 0)
            assert (wi >= 0).all() and (wa >= 0).all()
            assert np.array_equal(wi, gi) and np.array_equal(wa, ga)


def test_noalloc_rejects_oversized_batch():
    opt = gs.options(precision="fp16")
    sc, cam = scenes.camera_box_scene(10, seed=34), scenes.pinhole(16, 16, 60.0)
    jobs = _prepare([(sc, cam)], opt, 1)
    r = jobs[0][0]
    items = [(r.proj, r.bins, cam, r.image, None)] * (gs.lib().gs_max_batch() + 1)
    with pytest.raises(gs.GsError) as e:
        gs.gs_rasterize_batch_noalloc(items, opt)
    assert e.value.status == gs.GS_ERR_UNSUPPORTED
