"""Python front end of the FP64 CPU reference renderer (gs_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg use it; the GPU library never does, and this
module imports nothing from the GPU package.

The arithmetic lives in gs_oracle.c (double precision).  This module builds
that file with gcc, marshals numpy arrays, and derives the per-tile sets of
Gaussians whose tile membership lies within the footprint-edge or near-plane
guard bands (the compositing step flags pixels those could change).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TILE = 16
GUARD_PX = 1e-3
GUARD_Z = 1e-6
VISIBLE = 1
AMB_ZNEAR = 2
AMB_EDGES = 4 | 8 | 16 | 32
PIX_ALPHA, PIX_T, PIX_TIE, PIX_MEMBER = 1, 2, 4, 8
# Opacity-aware tile culling (the tighter ellipse-tile intersection the paper combines its
# method with): a Gaussian stays in a tile's list while the minimum of its quadratic form over
# the rectangle spanned by the tile's pixel centres is at most 2 ln(255 o) + TIGHT_MARGIN.  The
# margin keeps every pair whose alpha could reach the 1/255 cut under FP32/FP16 rounding;
# TIGHT_GUARD is the band around the boundary inside which FP32 inputs may decide differently.
TIGHT_MARGIN = 0.01
TIGHT_GUARD = 1e-3

_dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile gs_oracle.c into liboracle.so (plain C, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            L.oracle_sh_basis.argtypes = [C.c_int, _dp, _dp]
            L.oracle_sh_basis.restype = None
            L.oracle_preprocess.argtypes = [C.c_int64, C.c_int, _fp, _fp, _fp, _fp, _fp, C.c_int,
                                            C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _i32p, _u8p]
            L.oracle_preprocess.restype = None
            L.oracle_lists.argtypes = [C.c_int64, _i32p, _dp, _u8p, C.c_int, C.c_int, C.c_int,
                                       C.c_void_p, C.c_void_p, C.c_void_p]
            L.oracle_lists.restype = C.c_int64
            L.oracle_composite.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _i64p, _i64p,
                                           _i64p, _i64p, _dp, C.c_int, C.c_void_p, C.c_int64,
                                           _dp, _dp, _dp, _i64p, _u8p]
            L.oracle_composite.restype = None
            L.oracle_alternatives.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _i64p, _i64p,
                                              _i64p, _i64p, _dp, C.c_int64, _i64p, C.c_int, _dp, _i32p]
            L.oracle_alternatives.restype = None
            _lib = L
    return _lib


def sh_basis(deg: int, direction) -> np.ndarray:
    d = np.ascontiguousarray(direction, np.float64)
    out = np.zeros(16, np.float64)
    lib().oracle_sh_basis(deg, d, out)
    return out[: (deg + 1) ** 2]


def _c32(a):
    return np.ascontiguousarray(a, np.float32)


def preprocess(scene, cam) -> dict:
    """Per-Gaussian records: xy (n,2), depth, cov2d (n,3: xx,xy,yy), conic (n,3: a,b,c), rgb (n,3),
    radius, rect (n,4: x0,y0,x1,y1 half-open tile ranges), flags."""
    n = scene.n
    out = dict(xy=np.zeros((n, 2)), depth=np.zeros(n), cov2d=np.zeros((n, 3)), conic=np.zeros((n, 3)),
               rgb=np.zeros((n, 3)), radius=np.zeros(n), rect=np.zeros((n, 4), np.int32),
               flags=np.zeros(n, np.uint8))
    lib().oracle_preprocess(n, scene.sh_degree, _c32(scene.mean), _c32(scene.log_scale), _c32(scene.quat),
                            _c32(scene.sh), cam.packed(), cam.width, cam.height, out["xy"], out["depth"],
                            out["cov2d"], out["conic"], out["rgb"], out["radius"], out["rect"],
                            out["flags"])
    out["opacity"] = scene.opacity.astype(np.float64)
    out["visible"] = (out["flags"] & VISIBLE) != 0
    return out


def grid(cam, group: int = 1):
    tx = (cam.width + TILE - 1) // TILE
    ty = (cam.height + TILE - 1) // TILE
    return tx, ty, (tx + group - 1) // group, (ty + group - 1) // group


def lists(rec: dict, cam, group: int = 1):
    """CSR lists per bin (tile for group 1, GxG group otherwise): start (nbins+1), ids, masks.
    Each bin's entries are ordered by (depth, index)."""
    n = rec["depth"].shape[0]
    _, _, gx, gy = grid(cam, group)
    L = lib()
    total = L.oracle_lists(n, rec["rect"], rec["depth"], rec["flags"], cam.width, cam.height, group,
                           None, None, None)
    start = np.zeros(gx * gy + 1, np.int64)
    ids = np.zeros(max(total, 1), np.int64)
    masks = np.zeros(max(total, 1), np.uint64)
    L.oracle_lists(n, rec["rect"], rec["depth"], rec["flags"], cam.width, cam.height, group,
                   start.ctypes.data, ids.ctypes.data, masks.ctypes.data)
    return start, ids[:total], masks[:total]


def tile_lists(rec: dict, cam, tiles):
    """The tile lists of `lists(rec, cam, 1)` for the tiles in `tiles` only, as the same CSR
    layout with every other tile empty (Background, Gaussian sorting: a tile's list holds
    the visible Gaussians whose tile rectangle contains it, ordered by depth, ties by index).
    Written in numpy from the definition, for workloads whose full lists are too large."""
    tx, ty, _, _ = grid(cam, 1)
    vis = np.nonzero(rec["visible"])[0]
    vis = vis[np.lexsort((vis, rec["depth"][vis]))]
    rect = rec["rect"][vis]
    counts = np.zeros(tx * ty, np.int64)
    per = {}
    for t in np.unique(np.asarray(tiles, np.int64)):
        x, y = int(t % tx), int(t // tx)
        inside = (rect[:, 0] <= x) & (x < rect[:, 2]) & (rect[:, 1] <= y) & (y < rect[:, 3])
        per[int(t)] = vis[inside]
        counts[t] = per[int(t)].size
    start = np.zeros(tx * ty + 1, np.int64)
    start[1:] = np.cumsum(counts)
    ids = np.zeros(max(int(start[-1]), 1), np.int64)
    for t, g in per.items():
        ids[start[t]:start[t + 1]] = g
    return start, ids[:int(start[-1])]


def tile_qmin(rec: dict, gids, tiles, cam):
    """Minimum over the rectangle of pixel centres of tile t of q(p) = (p - mu')^T conic
    (p - mu'), for each (Gaussian gids[i], tile tiles[i]).  Zero when the centre lies in
    the rectangle; otherwise the minimum lies on an edge, where q is a convex parabola in the
    free coordinate, minimised by clamping its vertex to the edge."""
    tx_n = (cam.width + TILE - 1) // TILE
    gids = np.asarray(gids, np.int64)
    tiles = np.asarray(tiles, np.int64)
    a, b, c = rec["conic"][gids, 0], rec["conic"][gids, 1], rec["conic"][gids, 2]
    ux, uy = rec["xy"][gids, 0], rec["xy"][gids, 1]
    x0 = (tiles % tx_n) * TILE + 0.5
    y0 = (tiles // tx_n) * TILE + 0.5
    x1, y1 = x0 + TILE - 1, y0 + TILE - 1
    q = np.full(gids.shape, np.inf)
    for ey in (y0, y1):
        dy = ey - uy
        dx = np.clip(-b * dy / a, x0 - ux, x1 - ux)
        q = np.minimum(q, a * dx * dx + 2 * b * dx * dy + c * dy * dy)
    for ex in (x0, x1):
        dx = ex - ux
        dy = np.clip(-b * dx / c, y0 - uy, y1 - uy)
        q = np.minimum(q, a * dx * dx + 2 * b * dx * dy + c * dy * dy)
    inside = (ux >= x0) & (ux <= x1) & (uy >= y0) & (uy <= y1)
    return np.where(inside, 0.0, q)


def tight_keep(rec: dict, gids, tiles, cam):
    """(keep, ambiguous) for each (Gaussian, tile) pair under opacity-aware culling."""
    gids = np.asarray(gids, np.int64)
    bound = 2.0 * np.log(255.0 * rec["opacity"][gids]) + TIGHT_MARGIN
    q = tile_qmin(rec, gids, tiles, cam)
    return q <= bound, np.abs(q - bound) < TIGHT_GUARD


def tight_lists(rec: dict, cam, start, ids):
    """The tile lists (start, ids) of `lists(rec, cam, 1)` without the pairs that
    opacity-aware culling drops; also the per-entry ambiguity of the decision."""
    tx, ty, _, _ = grid(cam, 1)
    tiles = np.repeat(np.arange(tx * ty), np.diff(start))
    keep, amb = tight_keep(rec, ids, tiles, cam)
    counts = np.bincount(tiles[keep], minlength=tx * ty)
    st = np.zeros(tx * ty + 1, np.int64)
    st[1:] = np.cumsum(counts)
    return st, ids[keep], amb, keep


def tight_group_keep(rec: dict, cam, group: int, start, ids, masks):
    """Opacity-aware culling of the GxG group lists (start, ids, masks) of `lists`: each member
    tile of an entry's mask is tested with tight_keep; returns, per entry of those lists, the
    mask of the member tiles that pass, whether any passes (the entry is kept), and whether
    any member decision lies in the guard band."""
    tx, _, gx, _ = grid(cam, group)
    G = group
    nb = len(start) - 1
    bins = np.repeat(np.arange(nb), np.diff(start))
    bit = np.arange(G * G, dtype=np.uint64)
    has = ((np.asarray(masks, np.uint64)[:, None] >> bit[None, :]) & np.uint64(1)) != 0
    e, k = np.nonzero(has)
    ly, lx = k // G, k % G
    tiles = ((bins[e] // gx) * G + ly) * tx + (bins[e] % gx) * G + lx
    keep, amb = tight_keep(rec, ids[e], tiles, cam)
    newm = np.zeros(len(ids), np.uint64)
    np.bitwise_or.at(newm, e[keep], np.left_shift(np.uint64(1), k[keep].astype(np.uint64)))
    eamb = np.zeros(len(ids), bool)
    eamb[e[amb]] = True
    return newm, newm != 0, eamb


def tight_group_lists(rec: dict, cam, group: int):
    """The group lists of `lists(rec, cam, group)` under opacity-aware culling (start, ids,
    masks), and the per-entry ambiguity of the decision."""
    st, ids, masks = lists(rec, cam, group)
    newm, kept, eamb = tight_group_keep(rec, cam, group, st, ids, masks)
    nb = len(st) - 1
    bins = np.repeat(np.arange(nb), np.diff(st))
    counts = np.bincount(bins[kept], minlength=nb)
    out = np.zeros(nb + 1, np.int64)
    out[1:] = np.cumsum(counts)
    return out, ids[kept], newm[kept], eamb[kept]


def ambiguous_membership(rec: dict, cam):
    """Per tile, the Gaussians whose membership flips inside the footprint-edge (1e-3 px) or
    near-plane (1e-6) guard band.  Returns CSR (start, ids)."""
    tx, ty, _, _ = grid(cam, 1)
    fl = rec["flags"]
    cand = np.nonzero((fl & (AMB_ZNEAR | AMB_EDGES)) != 0)[0]
    eps = GUARD_PX / TILE
    per_tile = [[] for _ in range(tx * ty)]
    for g in cand:
        mx, my = rec["xy"][g]
        r = rec["radius"][g]
        lo = np.array([(mx - r) / TILE, (my - r) / TILE])
        hi = np.array([(mx + r) / TILE, (my + r) / TILE])
        may0 = np.floor(lo - eps).astype(int)
        may1 = np.floor(hi + eps).astype(int)
        sure0 = np.floor(lo + eps).astype(int)
        sure1 = np.floor(hi - eps).astype(int)
        lim = np.array([tx - 1, ty - 1])
        may0 = np.maximum(may0, 0)
        may1 = np.minimum(may1, lim)
        zamb = bool(fl[g] & AMB_ZNEAR)
        for yy in range(may0[1], may1[1] + 1):
            for xx in range(may0[0], may1[0] + 1):
                sure = (sure0[0] <= xx <= sure1[0]) and (sure0[1] <= yy <= sure1[1])
                if zamb or not sure:
                    per_tile[yy * tx + xx].append(int(g))
    start = np.zeros(tx * ty + 1, np.int64)
    start[1:] = np.cumsum([len(p) for p in per_tile])
    ids = np.array([g for p in per_tile for g in p] or [0], np.int64)
    return start, ids


def composite(rec: dict, cam, start, ids, bg=(0.0, 0.0, 0.0), nthreads: int = 1, tiles=None,
              amb=None) -> dict:
    W, H = cam.width, cam.height
    if amb is None:
        amb = ambiguous_membership(rec, cam)
    astart, aids = amb
    image = np.zeros((3, H, W))
    tfinal = np.zeros((H, W))
    wsum = np.zeros((H, W))
    neval = np.zeros((H, W), np.int64)
    ambig = np.zeros((H, W), np.uint8)
    sel = None if tiles is None else np.ascontiguousarray(tiles, np.int64)
    lib().oracle_composite(W, H, np.ascontiguousarray(rec["xy"]), rec["depth"],
                           np.ascontiguousarray(rec["conic"]), np.ascontiguousarray(rec["rgb"]),
                           rec["opacity"], start, np.ascontiguousarray(ids if ids.size else np.zeros(1, np.int64)),
                           astart, aids, np.ascontiguousarray(bg, np.float64), int(nthreads),
                           None if sel is None else sel.ctypes.data, 0 if sel is None else sel.size,
                           image, tfinal, wsum, neval, ambig)
    return dict(image=image, tfinal=tfinal, wsum=wsum, neval=neval, ambiguous=ambig)


def alternatives(rec: dict, cam, start, ids, pixels, bg=(0.0, 0.0, 0.0), amb=None, max_alt: int = 64):
    """Every admissible result of the given pixels (row-major indices) under the readings of
    the decisions that fall inside a guard band (1/255 cut, 1e-4 stop, order of near-equal
    depths, tile membership at a footprint edge or the near plane): each combination of the
    two ways of taking them, composited from the definition as `composite` does.
    Returns (results (npix, max_alt, 4): colour with background and T_final; counts (npix,):
    the number of results, or -1 when there are more than max_alt)."""
    W, H = cam.width, cam.height
    if amb is None:
        amb = ambiguous_membership(rec, cam)
    astart, aids = amb
    pix = np.ascontiguousarray(pixels, np.int64).ravel()
    out = np.zeros((max(pix.size, 1), max_alt, 4))
    cnt = np.zeros(max(pix.size, 1), np.int32)
    if pix.size:
        lib().oracle_alternatives(W, H, np.ascontiguousarray(rec["xy"]), rec["depth"],
                                  np.ascontiguousarray(rec["conic"]), np.ascontiguousarray(rec["rgb"]),
                                  rec["opacity"], start,
                                  np.ascontiguousarray(ids if ids.size else np.zeros(1, np.int64)), astart, aids,
                                  np.ascontiguousarray(bg, np.float64), pix.size, pix, int(max_alt), out, cnt)
    return out[: pix.size], cnt[: pix.size]


def check_flagged(image, tfinal, rec: dict, cam, start, ids, ambiguous, bg=(0.0, 0.0, 0.0), tol_img: float = 1e-4,
                  tol_t: float = 1e-5, amb=None, max_alt: int = 64) -> dict:
    """Checks a renderer's pixels that the oracle flagged (a decision inside a guard band):
    each must be within tol_img per channel (and tol_t in T_final, if given) of one of that
    pixel's admissible results.  image (3, H, W), tfinal (H, W) or None, ambiguous (H, W) from
    `composite`.  Returns counts: checked, matched, failed, unresolved (more than max_alt
    readings: left unchecked) and the flagged pixels' indices by outcome."""
    W = cam.width
    pix = np.flatnonzero(np.asarray(ambiguous) != 0)
    alts, cnt = alternatives(rec, cam, start, ids, pix, bg, amb, max_alt)
    img = np.asarray(image).reshape(3, -1)[:, pix].T          # (P, 3)
    d = np.abs(alts[:, :, :3] - img[:, None, :]).max(axis=2)  # (P, A)
    ok = d <= tol_img
    if tfinal is not None:
        t = np.asarray(tfinal).ravel()[pix]
        ok &= np.abs(alts[:, :, 3] - t[:, None]) <= tol_t
    valid = np.arange(max_alt)[None, :] < np.maximum(cnt, 0)[:, None]
    matched = (ok & valid).any(axis=1) & (cnt > 0)
    unresolved = cnt < 0
    failed = ~matched & ~unresolved
    return dict(checked=int(pix.size), matched=int(matched.sum()), failed=int(failed.sum()),
                unresolved=int(unresolved.sum()), failed_pixels=pix[failed], unresolved_pixels=pix[unresolved],
                width=W)


def render(scene, cam, bg=(0.0, 0.0, 0.0), nthreads: int = 1) -> dict:
    """Full FP64 render: records, tile lists, image (3,H,W), T_final, W = sum(alpha T), evaluation
    counts, ambiguity flags, and the Gaussian-pixel evaluation total E_pix."""
    rec = preprocess(scene, cam)
    start, ids, _ = lists(rec, cam, 1)
    out = composite(rec, cam, start, ids, bg, nthreads)
    out.update(records=rec, start=start, ids=ids, e_pix=int(out["neval"].sum()))
    return out


def load_reduction(rec: dict, cam, group: int) -> tuple:
    """(N_total, N_group, 1 - N_group/N_total) for GxG groups (Cross-tile grouping observation)."""
    s1, _, _ = lists(rec, cam, 1)
    sg, _, _ = lists(rec, cam, group)
    n_total = int(s1[-1])
    n_group = int(sg[-1])
    return n_total, n_group, (1.0 - n_group / n_total) if n_total else 0.0


def composite_backward(rec: dict, cam, start, ids, dimage, bg=(0.0, 0.0, 0.0)) -> dict:
    """Gradients of L = sum over channels and pixels of dimage * image, where image is the
    front-to-back composite of `composite` (Background: alpha = min(0.99, o exp(power)),
    power = -1/2 d^T conic d with d = pixel centre - centre, pairs with alpha < 1/255 skipped,
    C = sum alpha_i T_i c_i + T bg, stop before the Gaussian that would take T below 1e-4),
    with respect to each Gaussian's colour (n, 3), opacity (n), conic (a, b, c) (n, 3) and
    image-plane centre (n, 2).

    Written from the derivative of that recurrence (the method has no backward pass of its
    own; this is the exact gradient of its forward on the branch the forward takes: clamped
    alphas, skipped pairs and the stop are held fixed).  Per pixel and blended Gaussian i:
        dC/dc_i = alpha_i T_i
        dC/dalpha_i = c_i T_i - (S_i + T_end bg) / (1 - alpha_i),  S_i = sum_{j > i} c_j alpha_j T_j
    and, unless clamped, dalpha/do = alpha / o, dalpha/dpower = alpha, dpower/d(a, b, c) =
    -(dx^2 / 2, dx dy, dy^2 / 2), dpower/d(x, y) = (a dx + b dy, b dx + c dy).  FP64, numpy over
    the pixels of one tile at a time; for small workloads only."""
    W, H = cam.width, cam.height
    tx_n = (W + TILE - 1) // TILE
    ty_n = (H + TILE - 1) // TILE
    n = rec["depth"].shape[0]
    xy, conic, rgb, op = rec["xy"], rec["conic"], rec["rgb"], rec["opacity"]
    bg = np.asarray(bg, np.float64)
    dimage = np.asarray(dimage, np.float64).reshape(3, H, W)
    g_rgb = np.zeros((n, 3))
    g_op = np.zeros(n)
    g_conic = np.zeros((n, 3))
    g_xy = np.zeros((n, 2))
    for tile in range(tx_n * ty_n):
        s, e = int(start[tile]), int(start[tile + 1])
        if s == e:
            continue
        tx, ty = tile % tx_n, tile // tx_n
        yy, xx = np.meshgrid(np.arange(ty * TILE, min(ty * TILE + TILE, H)),
                             np.arange(tx * TILE, min(tx * TILE + TILE, W)), indexing="ij")
        xx, yy = xx.ravel(), yy.ravel()
        px, py = xx + 0.5, yy + 0.5
        gp = dimage[:, yy, xx]                       # (3, P)
        lst = np.asarray(ids[s:e], np.int64)
        L, P = lst.size, px.size
        A = np.zeros((L, P))
        TT = np.zeros((L, P))
        ACT = np.zeros((L, P), bool)
        FREE = np.zeros((L, P), bool)                # alpha not clamped at 0.99
        T = np.ones(P)
        alive = np.ones(P, bool)
        for k, g in enumerate(lst):
            dx, dy = px - xy[g, 0], py - xy[g, 1]
            a, b, c = conic[g]
            raw = op[g] * np.exp(-0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy))
            al = np.minimum(0.99, raw)
            ok = alive & (al >= 1.0 / 255.0)
            Tn = T * (1.0 - al)
            stop = ok & (Tn < 1e-4)
            act = ok & ~stop
            alive &= ~stop
            A[k], TT[k], ACT[k], FREE[k] = al, T, act, raw < 0.99
            T = np.where(act, Tn, T)
        Tend = T
        S = np.zeros((3, P))
        for k in range(L - 1, -1, -1):
            act = ACT[k]
            if not act.any():
                continue
            g = lst[k]
            al, Tk = A[k], TT[k]
            c3 = rgb[g][:, None]
            w = al * Tk * act
            g_rgb[g] += (gp * w).sum(axis=1)
            dC_da = c3 * Tk - (S + bg[:, None] * Tend) / (1.0 - al)
            dL_da = (gp * dC_da).sum(axis=0) * act
            dL_dp = dL_da * al * FREE[k]
            g_op[g] += (dL_da * FREE[k] * al / op[g]).sum()
            dx, dy = px - xy[g, 0], py - xy[g, 1]
            a, b, c = conic[g]
            g_conic[g] += [(-0.5 * dx * dx * dL_dp).sum(), (-dx * dy * dL_dp).sum(), (-0.5 * dy * dy * dL_dp).sum()]
            g_xy[g] += [((a * dx + b * dy) * dL_dp).sum(), ((b * dx + c * dy) * dL_dp).sum()]
            S += c3 * w
    return dict(rgb=g_rgb, opacity=g_op, conic=g_conic, xy=g_xy)
