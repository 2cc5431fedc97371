"""Parity of the backward pass of the tensorized (FP16/BF16 MFMA) forward,
gs_rasterize_backward_mfma, with the FP64 oracle's oracle.composite_backward.

Set-up as for the FP32 backward: both sides get the oracle's records (conic, colour and
opacity rounded to FP32) and its depth-sorted tile lists; the upstream gradient is N(0, 1),
zeroed on the pixels whose forward decisions lie in a guard band.  The GPU side first renders
the MFMA forward over those records and lists with GS_AUX_TFINAL | GS_AUX_LAST, then runs the
backward from that state.

Bar, per gradient field: max |gpu - ref| <= 1e-3 max|ref| + 1e-3 |ref| and relative L2 error
<= 2e-4.  Derivation: the split 16-bit power carries |d log2 alpha| <= 3.5e-5 (FP16, two pieces;
BF16 three pieces ~1e-6), so each alpha is within 2.5e-5 relative of the FP64 one; T_i is a
product of (1 - alpha) factors whose errors add as alpha / (1 - alpha) times that, and the
alpha-derivative divides by 1 - alpha >= 0.01: a few 1e-4 of a field's largest value at worst,
and far less on average (L2).  The FP32 arithmetic of the gradient terms (~1e-6) is below that."""
import numpy as np
import pytest

from oracle import oracle
from paper_2605_17855_amd import gs, scenes
from gpu_helpers import note, sampled_tiles
from test_gpu_backward import FIELDS, _fp32_records, _upload

pytestmark = pytest.mark.gpu

SPLITS = {"fp16": 2, "bf16": 3}


def _forward_state(proj, bins, cam, opt):
    """The MFMA forward over (proj, bins) with the T_final and blended-prefix-end planes."""
    import torch
    o = gs.options(precision=opt.precision, splits=opt.splits, bg=tuple(opt.bg),
                   aux_flags=gs.GS_AUX_TFINAL | gs.GS_AUX_LAST, all_rows=bool(opt.flags & gs.GS_OPT_ALL_ROWS))
    image = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device="cuda")
    aux = torch.empty((2, cam.height, cam.width), dtype=torch.float32, device="cuda")
    gs.gs_rasterize(proj, bins, cam, o, image, aux)
    return image, aux


def _gpu_backward_mfma(proj, bins, cam, dimg, bg, n, prec, all_rows=False, calls=1):
    import torch
    opt = gs.options(precision=prec, splits=SPLITS[prec], bg=bg, all_rows=all_rows)
    _, aux = _forward_state(proj, bins, cam, opt)
    grads = gs.Grads(n)
    d = torch.from_numpy(np.ascontiguousarray(dimg, np.float32)).cuda()
    for _ in range(calls):
        gs.gs_rasterize_backward_mfma(proj, bins, cam, opt, d, aux[0], aux[1], grads)
    torch.cuda.synchronize()
    return {f: getattr(grads, f).cpu().numpy().astype(np.float64)[:n] for f in FIELDS}


def _compare(tag, got, ref, rel=1e-3, l2_bar=2e-4):
    for f in FIELDS:
        a, b = got[f].reshape(-1), ref[f].reshape(-1)
        scale = float(np.abs(b).max()) if b.size else 0.0
        err = np.abs(a - b)
        mx = float(err.max()) if b.size else 0.0
        l2 = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        print(f"{tag} {f}: max|ref| {scale:.3e}, max err {mx:.3e} ({mx / max(scale, 1e-30):.2e} of max), "
              f"rel L2 {l2:.3e}", flush=True)
        assert np.all(err <= rel * scale + rel * np.abs(b)), (tag, f)
        assert l2 <= l2_bar or scale == 0.0, (tag, f, l2)


def _case(sc, cam, bg, seed):
    rec = _fp32_records(oracle.preprocess(sc, cam))
    start, ids, _ = oracle.lists(rec, cam, 1)
    rng = np.random.default_rng(seed)
    dimg = rng.normal(size=(3, cam.height, cam.width))
    fwd = oracle.composite(rec, cam, start, ids, bg=bg)
    dimg[:, fwd["ambiguous"] != 0] = 0.0
    ref = oracle.composite_backward(rec, cam, start, ids, dimg, bg)
    proj, bins = _upload(rec, start, ids)
    return rec, start, ids, dimg, fwd, ref, proj, bins


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.3, 0.6, 0.1)])
def test_backward_mfma_matches_oracle_ragged(prec, bg):
    """1,500 Gaussians at 200x120: 13x8 tiles with a ragged last column and row."""
    note(f"backward mfma ragged {prec} bg={bg}")
    sc = scenes.camera_box_scene(1500, seed=61, log_scale_mu=np.log(0.04))
    cam = scenes.pinhole(200, 120, 60.0)
    rec, start, ids, dimg, fwd, ref, proj, bins = _case(sc, cam, bg, 62)
    got = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, prec)
    _compare(f"mfma ragged {prec}", got, ref)
    assert np.count_nonzero(ref["opacity"]) > 500


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_backward_mfma_dense_stops_and_clamps(prec):
    """Large, partly opaque splats: most pixels stop and a tenth of the splats have opacity
    0.999 (clamped alphas at their centres)."""
    note(f"backward mfma dense {prec}")
    sc = scenes.camera_box_scene(2500, seed=63, log_scale_mu=np.log(0.12), log_scale_sigma=0.3)
    sc.opacity[::10] = 0.999
    cam = scenes.pinhole(96, 80, 60.0)
    bg = (0.2, 0.2, 0.2)
    rec, start, ids, dimg, fwd, ref, proj, bins = _case(sc, cam, bg, 64)
    assert (fwd["tfinal"] < 1e-3).mean() > 0.25
    got = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, prec)
    _compare(f"mfma dense {prec}", got, ref)


def test_backward_mfma_quadrant_culling_changes_nothing():
    """Every row in every quadrant (GS_OPT_ALL_ROWS) gives the same gradients, to the rounding of
    the atomic sums' order; two calls add up."""
    note("backward mfma all rows")
    sc = scenes.camera_box_scene(2000, seed=73, log_scale_mu=np.log(0.05))
    cam = scenes.pinhole(128, 96, 60.0)
    bg = (0.0, 0.0, 0.0)
    rec, start, ids, dimg, fwd, ref, proj, bins = _case(sc, cam, bg, 74)
    a = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, "fp16")
    b = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, "fp16", all_rows=True)
    c = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, "fp16", calls=2)
    for f in FIELDS:
        scale = float(np.abs(a[f]).max())
        assert np.abs(a[f] - b[f]).max() <= 1e-5 * scale, f
        assert np.abs(c[f] / 2.0 - a[f]).max() <= 1e-5 * scale, f


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_backward_mfma_headline_sampled_tiles(prec):
    """The 1M-Gaussian, 1920x1080 workload on 48 sampled tiles."""
    note(f"backward mfma 1M 1080p sampled tiles {prec}")
    sc, cam = scenes.clustered_1m()
    rec = _fp32_records(oracle.preprocess(sc, cam))
    tiles = sampled_tiles(cam, 48, 70)
    start, ids = oracle.tile_lists(rec, cam, tiles)
    bg = (0.0, 0.0, 0.0)
    rng = np.random.default_rng(71)
    dimg = rng.normal(size=(3, cam.height, cam.width))
    fwd = oracle.composite(rec, cam, start, ids, bg=bg, tiles=tiles, nthreads=8)
    dimg[:, fwd["ambiguous"] != 0] = 0.0
    ref = oracle.composite_backward(rec, cam, start, ids, dimg, bg)
    proj, bins = _upload(rec, start, ids)
    got = _gpu_backward_mfma(proj, bins, cam, dimg, bg, sc.n, prec)
    _compare(f"mfma 1M sampled {prec}", got, ref)
    assert int(start[-1]) > 5000


def test_backward_mfma_conservation_full_size():
    """1M Gaussians at 1920x1080 on the library's own bins, FP16: with every colour and the
    background 1 the image is 1 everywhere, so the opacity, conic and centre gradients vanish
    to rounding, while with the scene's colours they do not."""
    import torch
    note("backward mfma conservation 1M 1080p")
    sc, cam = scenes.clustered_1m()
    ds = gs.DeviceScene(sc)
    r = gs.Renderer(sc.n, cam.width, cam.height)
    opt = gs.options(precision="fp16", splits=2, bg=(1.0, 1.0, 1.0))
    r.render(ds, cam, opt)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(72)
    d = torch.randn((3, cam.height, cam.width), generator=gen, device="cuda")
    _, aux = _forward_state(r.proj, r.bins, cam, opt)
    own = gs.Grads(sc.n)
    gs.gs_rasterize_backward_mfma(r.proj, r.bins, cam, opt, d, aux[0], aux[1], own)
    r.proj.rgb[:, :3] = 1.0
    _, aux1 = _forward_state(r.proj, r.bins, cam, opt)
    ones = gs.Grads(sc.n)
    gs.gs_rasterize_backward_mfma(r.proj, r.bins, cam, opt, d, aux1[0], aux1[1], ones)
    torch.cuda.synchronize()
    assert torch.allclose(ones.rgb, own.rgb, rtol=1e-4, atol=1e-4 * float(own.rgb.abs().max()))
    for f in ("opacity", "conic", "xy"):
        scale = float(getattr(own, f).abs().max())
        resid = float(getattr(ones, f).abs().max())
        print(f"mfma conservation {f}: max |grad| with scene colours {scale:.3e}, with colours 1 {resid:.3e}")
        assert scale > 0 and resid <= 1e-4 * scale, (f, scale, resid)


def test_backward_mfma_rejects_fp32_and_groups():
    import torch
    sc = scenes.camera_box_scene(10, seed=75)
    cam = scenes.pinhole(32, 32, 60.0)
    rec = _fp32_records(oracle.preprocess(sc, cam))
    start, ids, _ = oracle.lists(rec, cam, 1)
    proj, bins = _upload(rec, start, ids)
    grads = gs.Grads(sc.n)
    d = torch.zeros((3, 32, 32), dtype=torch.float32, device="cuda")
    t = torch.ones((32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(gs.GsError) as e:
        gs.gs_rasterize_backward_mfma(proj, bins, cam, gs.options(precision="fp32"), d, t, t, grads)
    assert e.value.status == gs.GS_ERR_INVALID_ARG
    with pytest.raises(gs.GsError) as e:
        gs.gs_rasterize_backward_mfma(proj, bins, cam, gs.options(precision="fp16", group=2), d, t, t, grads)
    assert e.value.status == gs.GS_ERR_UNSUPPORTED
