"""Helpers for the GPU tests: run the HIP library through its binding, pull results to numpy."""
import sys

import numpy as np

from oracle import oracle
from paper_2605_17855_amd import gs


def note(msg: str):
    """Names the case before a GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def render(dscene, cam, group=1, precision="fp32", splits=2, bg=(0.0, 0.0, 0.0), aux=0, capacity=0, tight=False,
           all_rows=False, tile_rows=False):
    import torch
    r = gs.Renderer(dscene.n, cam.width, cam.height, group=group, capacity=capacity)
    opt = gs.options(group=group, precision=precision, splits=splits, bg=bg, aux_flags=aux, tight=tight,
                     all_rows=all_rows, tile_rows=tile_rows)
    n_keys = r.render(dscene, cam, opt)
    torch.cuda.synchronize()
    out = dict(image=r.image.cpu().numpy().astype(np.float64), n_keys=n_keys, renderer=r)
    if aux:
        planes = r.aux.cpu().numpy()
        k = 0
        for flag, name in ((gs.GS_AUX_TFINAL, "tfinal"), (gs.GS_AUX_WSUM, "wsum"), (gs.GS_AUX_NEVAL, "neval"),
                           (gs.GS_AUX_NBLEND, "nblend"), (gs.GS_AUX_LAST, "last")):
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
                masks=b.masks.cpu().numpy().view(np.uint64 if r.group == 8 else np.uint16)[:n_keys],
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


def sampled_tiles(cam, count, seed):
    tx, ty = (cam.width + 15) // 16, (cam.height + 15) // 16
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(tx * ty, size=min(count, tx * ty), replace=False))


def check_bins(rec, cam, r, n_keys, group, tight=False):
    b = bins_numpy(r, n_keys)
    keys, vals = b["keys"], b["vals"]
    # ascending keys; key = (bin << 32) | float bits of the GPU depth of its Gaussian
    assert np.all(keys[1:] >= keys[:-1])
    gdepth = r.proj.rgb.cpu().numpy()[:, 3]
    assert np.array_equal(keys & np.uint64(0xFFFFFFFF), gdepth[vals].view(np.uint32).astype(np.uint64))
    # stable: equal keys keep Gaussian-index order
    same = keys[1:] == keys[:-1]
    assert np.all(vals[1:][same] > vals[:-1][same])
    # ranges equal a linear scan of the sorted keys
    bins_of = (keys >> np.uint64(32)).astype(np.int64)
    nb = gs.gs_num_bins(cam, group)
    want = np.zeros((nb, 2), np.int64)
    if n_keys:
        starts = np.r_[0, np.nonzero(bins_of[1:] != bins_of[:-1])[0] + 1]
        ends = np.r_[starts[1:], n_keys]
        want[bins_of[starts], 0] = starts
        want[bins_of[starts], 1] = ends
    assert np.array_equal(b["ranges"][:nb].astype(np.int64), want)
    # entries against the oracle's lists (footprint-edge ambiguous Gaussians excluded)
    st, ids, masks = oracle.lists(rec, cam, group)
    amb = (rec["flags"] & (oracle.AMB_ZNEAR | oracle.AMB_EDGES)) != 0
    ob = np.repeat(np.arange(nb), np.diff(st))
    keep_o = ~amb[ids]
    keep_g = ~amb[vals]
    if tight:
        # the culled lists; entries with a member-tile decision in the guard band are left out
        # on both sides
        masks, keep_t, amb_t = oracle.tight_group_keep(rec, cam, group, st, ids, masks)
        bad = set(zip(ids[amb_t].tolist(), ob[amb_t].tolist()))
        keep_o &= keep_t & ~amb_t
        keep_g &= np.array([(int(g), int(b)) not in bad for g, b in zip(vals, bins_of)], bool) if bad else True
    assert np.array_equal(ob[keep_o], bins_of[keep_g])
    og, gg = ids[keep_o], vals[keep_g].astype(np.int64)
    mismatch = np.nonzero(og != gg)[0]
    # order may differ only between Gaussians at (nearly) equal depth
    for i in mismatch:
        za, zb = rec["depth"][og[i]], rec["depth"][gg[i]]
        assert abs(za - zb) <= 1e-6 * za, (i, og[i], gg[i])
    # the visible list after sorting: every visible Gaussian once, ordered by (depth bits, index)
    V = int(r.proj.n_visible.cpu().numpy()[0])
    order = r.proj.order.cpu().numpy().view(np.uint32)[:V].astype(np.int64)
    count = r.proj.count.cpu().numpy().view(np.uint32)
    assert np.array_equal(np.sort(order), np.nonzero(count[: r.proj.n])[0])
    dbits = gdepth.view(np.uint32)[order]
    assert np.all((dbits[1:] > dbits[:-1]) | ((dbits[1:] == dbits[:-1]) & (order[1:] > order[:-1])))
    if group > 1:
        gm = b["masks"][keep_g].astype(np.uint64)
        om = masks[keep_o]
        ok = og == gg
        assert np.array_equal(gm[ok], om[ok])


def check_flagged_pixels(tag, image, tfinal, ref, rec, cam, start, ids, mask=None, bg=(0.0, 0.0, 0.0),
                         tol=1e-4, tol_t=1e-5):
    """The pixels exempt from the element-wise bar (a decision in a guard band): each must match
    one of the oracle's admissible results for that pixel (oracle.alternatives) within the same
    bar.  Pixels with more readings than the enumeration holds stay unchecked; they must be
    under 0.1 % of the compared pixels.  mask: the compared pixels (sampled tiles), or all."""
    amb = np.asarray(ref["ambiguous"]).copy()
    if mask is not None:
        amb[~mask] = 0
    r = oracle.check_flagged(image, tfinal, rec, cam, start, ids, amb, bg=bg, tol_img=tol, tol_t=tol_t)
    total = int(mask.sum()) if mask is not None else amb.size
    print(f"{tag}: flagged {r['checked']} of {total} pixels ({r['checked'] / max(total, 1):.4%}): "
          f"{r['matched']} match an admissible result, {r['failed']} fail, {r['unresolved']} unresolved", flush=True)
    if r["failed"]:
        W = cam.width
        bad = r["failed_pixels"][:8]
        print(f"{tag}: failing pixels (y, x) {[(int(p // W), int(p % W)) for p in bad]}", flush=True)
    assert r["failed"] == 0
    assert r["unresolved"] <= 1e-3 * total
    return r
