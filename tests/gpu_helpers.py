"""Helpers for the GPU tests: run the HIP library through its binding, pull results to numpy."""
import sys

import numpy as np

from paper_2605_17855_amd import gs


def note(msg: str):
    """Names the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def render(dscene, cam, group=1, precision="fp32", splits=2, bg=(0.0, 0.0, 0.0), aux=0, capacity=0):
    import torch
    r = gs.Renderer(dscene.n, cam.width, cam.height, group=group, capacity=capacity)
    opt = gs.options(group=group, precision=precision, splits=splits, bg=bg, aux_flags=aux)
    n_keys = r.render(dscene, cam, opt)
    torch.cuda.synchronize()
    out = dict(image=r.image.cpu().numpy().astype(np.float64), n_keys=n_keys, renderer=r)
    if aux:
        planes = r.aux.cpu().numpy()
        k = 0
        for flag, name in ((gs.GS_AUX_TFINAL, "tfinal"), (gs.GS_AUX_WSUM, "wsum"), (gs.GS_AUX_NEVAL, "neval"),
                           (gs.GS_AUX_NBLEND, "nblend")):
            if aux & flag:
                out[name] = planes[k].astype(np.float64)
                k += 1
    return out


def projected_numpy(r: "gs.Renderer"):
    p = r.proj
    count = p.count.cpu().numpy().view(np.uint32)[: p.n]
    return dict(xy=p.xy.cpu().numpy()[: p.n], conic=p.conic.cpu().numpy()[: p.n], rgb=p.rgb.cpu().numpy()[: p.n],
                rect=p.rect.cpu().numpy().view(np.uint16)[: p.n].astype(np.int64), count=count,
                offset=p.offset.cpu().numpy().view(np.uint64))


def bins_numpy(r: "gs.Renderer", n_keys: int):
    b = r.bins
    return dict(keys=b.keys.cpu().numpy().view(np.uint64)[:n_keys], vals=b.vals.cpu().numpy().view(np.uint32)[:n_keys],
                masks=b.masks.cpu().numpy().view(np.uint16)[:n_keys],
                ranges=b.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2))


def psnr(a, b):
    mse = np.mean((np.clip(a, 0, 1) - np.clip(b, 0, 1)) ** 2)
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def tile_mask(cam, tiles):
    tx = (cam.width + 15) // 16
    m = np.zeros((cam.height, cam.width), bool)
    for t in tiles:
        x, y = (t % tx) * 16, (t // tx) * 16
        m[y:y + 16, x:x + 16] = True
    return m
