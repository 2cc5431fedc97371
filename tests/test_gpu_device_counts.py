"""The frame without the host wait (GS_OPT_DEVICE_COUNTS).  The bin sort then reads the entry
and visible counts on the device, with its grids sized for the capacity.

Checks:
- its bins and images equal those of the frame that waits for the counts, bit for bit; that
  frame is held to the oracle by the parity tests, and the small case here is checked against
  the oracle as well;
- a capacity overflow leaves every range empty and the background image, and the entry count
  stays readable on the device;
- the frame consists of kernel launches only, so it can be captured into a HIP graph and
  replayed over scene data that changed in place."""
import numpy as np
import pytest

from oracle import oracle
from paper_2605_17855_amd import gs, scenes
from gpu_helpers import bins_numpy, note, psnr

pytestmark = pytest.mark.gpu

BG = (0.25, 0.5, 0.75)


def _frame(ds, cam, capacity, device_counts, **kw):
    """One gs_render through a fresh Renderer; returns (renderer, entry count on the device)."""
    import torch
    r = gs.Renderer(ds.n, cam.width, cam.height, group=kw.get("group", 1), capacity=capacity)
    opt = gs.options(bg=BG, device_counts=device_counts, **kw)
    out = r.render(ds, cam, opt)
    torch.cuda.synchronize()
    k = gs.entry_count(r.proj)
    if device_counts:
        assert out is None
    else:
        assert out == k
    return r, k


def _same_frame(a, b, k, group):
    """Images, ranges and the first k sorted entries (keys, values, masks) identical."""
    import torch
    assert torch.equal(a.image, b.image)
    ba, bb = bins_numpy(a, k), bins_numpy(b, k)
    assert np.array_equal(ba["ranges"], bb["ranges"])
    assert np.array_equal(ba["keys"], bb["keys"])
    assert np.array_equal(ba["vals"], bb["vals"])
    if group > 1:
        assert np.array_equal(ba["masks"], bb["masks"])
    assert torch.equal(a.proj.order[: int(a.proj.n_visible.item())], b.proj.order[: int(b.proj.n_visible.item())])


@pytest.fixture(scope="module")
def small():
    sc, cam = scenes.small_camera_space()
    return sc, cam, gs.DeviceScene(sc)


@pytest.mark.parametrize("group,precision,tight", [
    (1, "fp32", False), (1, "fp16", False), (1, "fp16", True), (2, "fp16", False), (2, "bf16", True),
    (2, "fp32", False), (4, "fp16", False), (4, "fp16", True), (8, "fp16", False)])
def test_small_equals_host_count_frame(small, group, precision, tight):
    sc, cam, ds = small
    note(f"device counts 4096 / 128x128 G={group} {precision} tight={tight}")
    kw = dict(group=group, precision=precision, tight=tight, splits=3 if precision == "bf16" else 2)
    host, k = _frame(ds, cam, 0, False, **kw)
    dev, k2 = _frame(ds, cam, host.bins.capacity, True, **kw)
    assert k == k2 and k > 1000
    _same_frame(host, dev, k, group)
    # exactly at capacity: still every entry
    full, k3 = _frame(ds, cam, k, True, **kw)
    assert k3 == k
    _same_frame(host, full, k, group)


def test_small_against_oracle(small):
    sc, cam, ds = small
    note("device counts 4096 / 128x128 against the oracle")
    dev, _ = _frame(ds, cam, 0, True, precision="fp16")
    ref = oracle.render(sc, cam, bg=BG)
    img = dev.image.cpu().numpy().astype(np.float64)
    assert psnr(img, ref["image"]) > 45.0
    assert np.abs(img - ref["image"]).mean() < 2e-3


@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_overflow_leaves_background(small, group):
    sc, cam, ds = small
    note(f"device counts overflow 4096 / 128x128 G={group}")
    import torch
    _, k = _frame(ds, cam, 0, False, group=group, precision="fp16")
    r, k2 = _frame(ds, cam, k - 1, True, group=group, precision="fp16")
    assert k2 == k   # the count that did not fit, left on the device
    assert int(r.bins.ranges.abs().sum().item()) == 0
    bg = torch.tensor(BG, dtype=torch.float32, device=r.image.device).view(3, 1, 1).expand_as(r.image)
    assert torch.equal(r.image, bg)


def test_no_visible_and_single_entry(small):
    sc, cam, ds = small
    import torch
    note("device counts: camera facing away (no entries)")
    away = scenes.Camera(R=(cam.R * np.array([[1.0], [-1.0], [-1.0]], np.float32)).astype(np.float32),
                         t=cam.t.copy(), fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy, width=cam.width,
                         height=cam.height, znear=cam.znear)
    r, k = _frame(ds, away, 64, True, precision="fp16")
    assert k == 0
    bg = torch.tensor(BG, dtype=torch.float32, device=r.image.device).view(3, 1, 1).expand_as(r.image)
    assert torch.equal(r.image, bg)
    assert int(r.bins.ranges.abs().sum().item()) == 0
    # one Gaussian with one tile: a single entry, with capacity 1 (no sort at all) and 64
    note("device counts: a single entry")
    host0, _ = _frame(ds, cam, 0, False, precision="fp16")
    c0 = host0.proj.count.cpu().numpy()
    one = np.flatnonzero(c0 == 1)
    assert one.size > 0
    ds1 = gs.DeviceScene(sc.subset([int(one[0])]))
    h1, k1 = _frame(ds1, cam, 0, False, precision="fp16")
    assert k1 == 1
    for cap in (1, 64):
        d1, kd = _frame(ds1, cam, cap, True, precision="fp16")
        assert kd == 1
        _same_frame(h1, d1, 1, 1)


def test_1m_1080p_equals_host_count_frame():
    note("device counts 1M / 1080p G=1,2 fp16")
    sc, cam = scenes.clustered_1m()
    ds = gs.DeviceScene(sc)
    for group in (1, 2):
        host, k = _frame(ds, cam, 0, False, group=group, precision="fp16")
        dev, k2 = _frame(ds, cam, host.bins.capacity, True, group=group, precision="fp16")
        assert k == k2 and k > 100_000
        _same_frame(host, dev, k, group)


def test_graph_replay_follows_scene_updates(small):
    """A captured frame replayed three times, the Gaussians moved in place between replays (and
    eager work and synchronizations in between): every replay equals an eager frame of the moved
    scene."""
    import torch
    sc, cam, _ = small
    note("device counts: graph capture of a 4096 / 128x128 frame")
    ds = gs.DeviceScene(sc)
    r = gs.Renderer(ds.n, cam.width, cam.height, group=2, capacity=8 * ds.n)
    opt = gs.options(group=2, precision="fp16", bg=BG, device_counts=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        r.render(ds, cam, opt, stream=side)   # eager warm-up
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.render(ds, cam, opt)
    torch.cuda.synchronize()
    base = ds.mean.clone()
    rng = np.random.default_rng(7)
    for rep in range(3):
        shift = torch.from_numpy(rng.normal(0.0, 0.05, size=(3, 1)).astype(np.float32)).to(ds.mean.device)
        ds.mean.copy_(base + shift)
        torch.cuda.synchronize()
        note(f"graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        got = r.image.clone()
        k = gs.entry_count(r.proj)
        assert k <= r.bins.capacity
        eager, ke = _frame(ds, cam, 0, False, group=2, precision="fp16")
        assert ke == k
        assert torch.equal(got, eager.image), rep
        if rep == 0:
            first = got
        else:
            assert not torch.equal(got, first)
