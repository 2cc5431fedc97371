"""Serving on the GPU: continuous batching through the HIP library, each result equal to its alone render."""
import numpy as np
import pytest

from paper_2605_17855_amd import scenes, server

from gpu_helpers import note

pytestmark = pytest.mark.gpu

SMALL_RES = ((160, 90), (320, 180), (256, 256), (480, 270))


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_served_images_equal_alone_renders(prec):
    import torch
    from paper_2605_17855_amd import gs
    scs = scenes.serving_scenes(count=4, scale=0.02)            # 10k .. 60k Gaussians
    dss = [gs.DeviceScene(s) for s in scs]
    reqs = scenes.serving_requests(48, rate_hz=1e5, n_scenes=4, seed=49, resolutions=SMALL_RES)
    opt = gs.options(group=1, precision=prec, splits=2, bg=(0.1, 0.2, 0.3))
    # a pool that holds only a few requests at once, and a keys-per-pixel guess far too low, so
    # both the memory bound and the retry-with-exact-size path are exercised
    pool = 8 << 20
    be = server.GpuBackend(dss, slots=8, pool_bytes=pool, opt=opt, max_pixels=max(w * h for w, h in SMALL_RES),
                           keys_per_pixel={i: 1e-3 for i in range(4)}, keep_results=True)
    note(f"serving {prec}: 48 requests, 4 scenes, pool {pool}")
    try:
        st = server.Server(be, pool, slots=8, max_batch=32).run(reqs)
    finally:
        be.close()
    torch.cuda.synchronize()
    assert st.completed == 48 and st.failed == 0
    assert st.max_reserved_bytes <= pool
    assert st.retries >= 1
    assert st.batches < 48                      # some launches rendered several requests
    assert st.max_inflight_jobs > 1
    for r in reqs:
        cam = scenes.look_at(r.position, r.width, r.height)
        ren = gs.Renderer(dss[r.scene].n, r.width, r.height)
        note(f"serving {prec}: alone render of request {r.rid}")
        ren.render(dss[r.scene], cam, opt)
        torch.cuda.synchronize()
        assert torch.equal(ren.image, be.results[r.rid]), f"request {r.rid} differs from its alone render"


def test_serving_rejects_request_larger_than_pool():
    import torch
    from paper_2605_17855_amd import gs
    scs = scenes.serving_scenes(count=2, scale=0.02)
    dss = [gs.DeviceScene(s) for s in scs]
    reqs = scenes.serving_requests(6, rate_hz=1e5, n_scenes=2, seed=50, resolutions=((320, 180),))
    for r in reqs:
        r.scene = 1                                            # the larger scene only
    opt = gs.options(group=1, precision="fp16", splits=2)
    pool = server.job_bytes(scs[1].n, 0, 320 * 180) + 4096    # room for per-Gaussian scratch only
    be = server.GpuBackend(dss, slots=4, pool_bytes=pool, opt=opt, max_pixels=320 * 180,
                           keys_per_pixel={0: 1.0, 1: 1.0}, keep_results=True)
    note("serving: oversized requests")
    try:
        st = server.Server(be, pool, slots=4).run(reqs)
    finally:
        be.close()
    torch.cuda.synchronize()
    assert st.failed == 6 and st.completed == 0
    assert st.retries == 6          # each tried once at the pool's size, then rejected on its exact size
