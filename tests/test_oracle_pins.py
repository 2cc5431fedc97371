"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against a closed form, a textbook or library
routine, an invariant, or brute force written along a different route, so that
a dropped term, a wrong sign or index, or a transposed operand in the oracle
fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy import special

from oracle import oracle
from paper_2605_17855_amd import scenes

Y00 = 0.5 / math.sqrt(math.pi)


def one_scene(means, log_scales, quats, opac, sh, deg=0):
    return scenes.Scene(np.asarray(means, np.float32).reshape(3, -1),
                        np.asarray(log_scales, np.float32).reshape(3, -1),
                        np.asarray(quats, np.float32).reshape(4, -1),
                        np.asarray(opac, np.float32).reshape(-1),
                        np.asarray(sh, np.float32).reshape((deg + 1) ** 2, 3, -1), deg)


def real_sh_scipy(l, m, direction):
    """Real orthonormal SH from scipy's complex Y_l^m (Condon-Shortley phase included)."""
    x, y, z = direction
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    am = abs(m)
    Y = special.sph_harm_y(l, am, theta, phi)
    if m > 0:
        return math.sqrt(2.0) * Y.real
    if m < 0:
        return math.sqrt(2.0) * Y.imag
    return Y.real


# ---------------------------------------------------------------- SH basis ---

def test_sh_textbook_low_orders():
    # Y00 = 1/(2 sqrt(pi)); Y1,-1 = -c y, Y1,0 = c z, Y1,1 = -c x with c = sqrt(3/(4 pi)).
    c = math.sqrt(3.0 / (4.0 * math.pi))
    rng = np.random.default_rng(0)
    for _ in range(20):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(1, d)
        assert Y[0] == pytest.approx(Y00, abs=1e-15)
        assert Y[1] == pytest.approx(-c * d[1], abs=1e-14)
        assert Y[2] == pytest.approx(c * d[2], abs=1e-14)
        assert Y[3] == pytest.approx(-c * d[0], abs=1e-14)


def test_sh_matches_scipy_degree3():
    rng = np.random.default_rng(1)
    for _ in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert Y[l * l + l + m] == pytest.approx(real_sh_scipy(l, m, d), abs=1e-13), (l, m)


def test_sh_orthonormal_by_quadrature():
    xs, ws = np.polynomial.legendre.leggauss(24)
    nphi = 48
    gram = np.zeros((16, 16))
    for ct, w in zip(xs, ws):
        st = math.sqrt(1.0 - ct * ct)
        for k in range(nphi):
            phi = 2.0 * math.pi * k / nphi
            Y = oracle.sh_basis(3, np.array([st * math.cos(phi), st * math.sin(phi), ct]))
            gram += np.outer(Y, Y) * w * (2.0 * math.pi / nphi)
    assert np.abs(gram - np.eye(16)).max() < 1e-12


# ------------------------------------------------------------- projection ---

def test_isotropic_on_axis_closed_form():
    cam = scenes.pinhole(64, 48, 60.0)
    s, z0 = 0.03, 3.0
    sc = one_scene([0, 0, z0], [math.log(s)] * 3, [1, 0, 0, 0], [0.5], [0.2, 0.1, -0.3])
    rec = oracle.preprocess(sc, cam)
    s32 = float(np.float32(math.log(s)))
    var = (cam.fx * math.exp(s32) / float(np.float32(z0))) ** 2 + 0.3
    assert rec["xy"][0] == pytest.approx([cam.cx, cam.cy], abs=1e-12)
    assert rec["cov2d"][0] == pytest.approx([var, 0.0, var], rel=1e-12, abs=1e-12)
    assert rec["conic"][0] == pytest.approx([1 / var, 0.0, 1 / var], rel=1e-12, abs=1e-12)
    assert rec["radius"][0] == pytest.approx(3.0 * math.sqrt(var), rel=1e-12)
    assert rec["depth"][0] == pytest.approx(z0, rel=1e-7)
    # SH degree 0 colour: k * Y00 + 0.5 per channel, clamped at 0
    assert rec["rgb"][0] == pytest.approx([max(0.0, float(np.float32(k)) * Y00 + 0.5)
                                          for k in (0.2, 0.1, -0.3)], abs=1e-12)


def _proj(p, cam):
    return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])


def _rand_camera(rng, W=200, H=150):
    pos = scenes.sphere_position(rng, 4.0)
    return scenes.look_at(pos, W, H)


def test_ewa_covariance_vs_finite_difference_jacobian():
    rng = np.random.default_rng(2)
    cam = _rand_camera(rng)
    n = 40
    # Gaussians near the origin, which the camera looks at: inside the clamp range
    means = rng.uniform(-0.6, 0.6, (3, n))
    ls = rng.normal(math.log(0.05), 0.4, (3, n))
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0)
    sc = one_scene(means, ls, q, np.full(n, 0.5), np.zeros((1, 3, n)))
    rec = oracle.preprocess(sc, cam)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    for g in range(n):
        m = sc.mean[:, g].astype(np.float64)
        pc = R @ m + t
        # Sigma = M S^2 M^T with M from scipy's quaternion convention (x, y, z, w)
        w, x, y, z = sc.quat[:, g].astype(np.float64)
        M = Rotation.from_quat([x, y, z, w]).as_matrix()
        S2 = np.diag(np.exp(2.0 * sc.log_scale[:, g].astype(np.float64)))
        V = R @ M @ S2 @ M.T @ R.T
        h = 1e-6 * pc[2]
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (_proj(pc + e, cam) - _proj(pc - e, cam)) / (2 * h)
        S = J @ V @ J.T
        got = rec["cov2d"][g]
        assert got[0] - 0.3 == pytest.approx(S[0, 0], rel=1e-6)
        assert got[1] == pytest.approx(S[0, 1], rel=1e-6, abs=1e-9 * abs(S[0, 0]))
        assert got[2] - 0.3 == pytest.approx(S[1, 1], rel=1e-6)
        # conic is the inverse
        a, b, c = rec["conic"][g]
        Sp = np.array([[got[0], got[1]], [got[1], got[2]]])
        assert np.abs(np.array([[a, b], [b, c]]) @ Sp - np.eye(2)).max() < 1e-12
        # projected mean: a point maps through the pinhole
        assert rec["xy"][g] == pytest.approx(_proj(pc, cam), abs=1e-9)
        # radius: three times the square root of the largest eigenvalue (library routine)
        assert rec["radius"][g] == pytest.approx(3.0 * math.sqrt(np.linalg.eigvalsh(Sp).max()),
                                                 rel=1e-12)
        assert rec["depth"][g] == pytest.approx(pc[2], rel=1e-12)


def test_lateral_clamp_invariance():
    # Beyond 1.3x the half-FOV tangent, the Jacobian is taken at the clamp: moving the
    # Gaussian further out at the same depth leaves the 2D covariance unchanged.
    cam = scenes.pinhole(100, 80, 60.0)
    z = 2.0
    lim = 1.3 * (cam.width / 2) / cam.fx
    xs = [lim * z * 1.0001, lim * z * 1.5, lim * z * 3.0]
    q = [0.9, 0.2, -0.3, 0.1]
    scs = [one_scene([x, 0.1, z], [-3.0, -2.5, -2.8], q, [0.5], [0, 0, 0]) for x in xs]
    cov = [oracle.preprocess(s, cam)["cov2d"][0] for s in scs]
    assert np.abs(cov[1] - cov[0]).max() < 1e-9 * np.abs(cov[0]).max()
    assert np.abs(cov[2] - cov[0]).max() < 1e-9 * np.abs(cov[0]).max()
    # just inside the clamp, the covariance differs (the clamp is not a no-op)
    inside = one_scene([lim * z * 0.5, 0.1, z], [-3.0, -2.5, -2.8], q, [0.5], [0, 0, 0])
    assert np.abs(oracle.preprocess(inside, cam)["cov2d"][0] - cov[0]).max() > 1e-6


def test_near_plane_cull():
    cam = scenes.pinhole(64, 64, 60.0, znear=0.2)
    sc = one_scene([[0, 0, 0], [0, 0, 0], [0.1, 0.2001, 1.0]], [-3] * 9, [1, 0, 0, 0] * 3, [0.5] * 3,
                   np.zeros(9))
    sc.mean = np.array([[0, 0, 0], [0, 0, 0], [0.1, 0.2001, 1.0]], np.float32)
    sc.quat = np.tile(np.array([[1], [0], [0], [0]], np.float32), 3)
    rec = oracle.preprocess(sc, cam)
    assert list(rec["visible"]) == [False, True, True]


def test_rect_by_brute_force_tile_overlap():
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    tx, ty, _, _ = oracle.grid(cam)
    for g in range(0, sc.n, 7):
        if not rec["flags"][g] and rec["radius"][g] == 0:
            continue
        mx, my = rec["xy"][g]
        r = rec["radius"][g]
        cols = [k for k in range(tx) if 16 * k <= mx + r and 16 * k + 16 > mx - r]
        rows = [k for k in range(ty) if 16 * k <= my + r and 16 * k + 16 > my - r]
        if rec["visible"][g]:
            x0, y0, x1, y1 = rec["rect"][g]
            assert cols == list(range(x0, x1)) and rows == list(range(y0, y1)), g
        elif rec["depth"][g] > cam.znear:
            assert not cols or not rows, g


# ------------------------------------------------------------- compositing ---

def _pix_centres(W, H):
    return np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)


def test_single_gaussian_closed_form_image():
    cam = scenes.pinhole(96, 64, 60.0)
    s, z0, o = 0.04, 2.5, 0.8
    k = np.array([0.3, -0.2, 0.6], np.float32)
    # on the optical axis the first-order projection of an isotropic Gaussian is isotropic
    sc = one_scene([0.0, 0.0, z0], [math.log(s)] * 3, [1, 0, 0, 0], [o], k)
    bg = (0.1, 0.2, 0.3)
    out = oracle.render(sc, cam, bg=bg)
    # closed form: isotropic std fx s / z in screen space plus the 0.3 px^2 dilation
    s32, z32, o32 = math.exp(float(np.float32(math.log(s)))), float(np.float32(z0)), float(np.float32(o))
    var = (cam.fx * s32 / z32) ** 2 + 0.3
    mu = np.array([cam.cx, cam.cy])
    X, Y = _pix_centres(cam.width, cam.height)
    alpha = np.minimum(0.99, o32 * np.exp(-((X - mu[0]) ** 2 + (Y - mu[1]) ** 2) / (2 * var)))
    r = 3 * math.sqrt(var)
    tile_in = ((np.floor(X / 16) >= math.floor((mu[0] - r) / 16)) & (np.floor(X / 16) <= math.floor((mu[0] + r) / 16)) &
               (np.floor(Y / 16) >= math.floor((mu[1] - r) / 16)) & (np.floor(Y / 16) <= math.floor((mu[1] + r) / 16)))
    alpha = np.where(tile_in & (alpha >= 1 / 255), alpha, 0.0)
    col = k.astype(np.float64) * Y00 + 0.5
    for ch in range(3):
        want = alpha * col[ch] + (1 - alpha) * bg[ch]
        assert np.abs(out["image"][ch] - want).max() < 1e-12
    assert np.abs(out["tfinal"] - (1 - alpha)).max() < 1e-12


def test_two_cocentred_gaussians_porter_duff_over():
    W = H = 32
    cam = scenes.pinhole(W, H, 60.0)
    # both centres on the centre of pixel (16, 16): mu' = 16.5; listed far first so that
    # index order and depth order disagree
    z1, z2 = 2.0, 3.0
    pts = [[0.5 * z / cam.fx, 0.5 * z / cam.fx, z] for z in (z2, z1)]
    o2, o1 = 0.7, 0.6
    k1 = np.array([0.5, -0.5, 0.1], np.float32)
    k2 = np.array([-0.4, 0.4, 0.9], np.float32)
    sc = scenes.Scene(np.array(pts, np.float32).T.copy(), np.full((3, 2), math.log(0.02), np.float32),
                      np.array([[1, 1], [0, 0], [0, 0], [0, 0]], np.float32),
                      np.array([o2, o1], np.float32), np.stack([k2, k1], axis=1)[None].copy(), 0)
    out = oracle.render(sc, cam, bg=(0.0, 0.0, 0.0))
    rec = out["records"]
    assert np.abs(rec["xy"] - 16.5).max() < 2e-5
    c1 = k1.astype(np.float64) * Y00 + 0.5
    c2 = k2.astype(np.float64) * Y00 + 0.5

    def alpha(g, o):
        d = rec["xy"][g] - 16.5   # float32 inputs leave a tiny offset from the pixel centre
        a, b, c = rec["conic"][g]
        return float(np.float32(o)) * math.exp(-0.5 * (a * d[0] ** 2 + 2 * b * d[0] * d[1] + c * d[1] ** 2))

    a1, a2 = alpha(1, o1), alpha(0, o2)
    assert a1 == pytest.approx(o1, rel=1e-6) and a2 == pytest.approx(o2, rel=1e-6)
    want = a1 * c1 + (1 - a1) * a2 * c2
    assert out["image"][:, 16, 16] == pytest.approx(want, abs=1e-12)
    assert out["tfinal"][16, 16] == pytest.approx((1 - a1) * (1 - a2), abs=1e-12)


def test_telescoping_identity_and_counts():
    sc, cam = scenes.small_camera_space()
    out = oracle.render(sc, cam)
    assert np.abs(out["wsum"] + out["tfinal"] - 1.0).max() < 1e-12
    assert (out["tfinal"] >= 1e-4 - 1e-15).all()
    # per-pixel evaluation count never exceeds the tile's list length
    st = out["start"]
    tx, ty, _, _ = oracle.grid(cam)
    lens = (st[1:] - st[:-1]).reshape(ty, tx)
    cap = np.kron(lens, np.ones((16, 16), np.int64))[: cam.height, : cam.width]
    assert (out["neval"] <= cap).all()
    assert out["e_pix"] == int(out["neval"].sum())


def test_permutation_invariance():
    sc, cam = scenes.small_camera_space(n=512, seed=7)
    base = oracle.render(sc, cam)
    perm = np.random.default_rng(3).permutation(sc.n)
    out = oracle.render(sc.subset(perm), cam)
    assert len(np.unique(base["records"]["depth"])) == sc.n
    assert np.array_equal(base["image"], out["image"])
    assert np.array_equal(base["tfinal"], out["tfinal"])


def test_lists_sorted_by_depth_then_index():
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    start, ids, _ = oracle.lists(rec, cam, 1)
    tx, ty, _, _ = oracle.grid(cam)
    vis = np.nonzero(rec["visible"])[0]
    for t in range(tx * ty):
        x, y = t % tx, t // tx
        r = rec["rect"][vis]
        members = vis[(r[:, 0] <= x) & (x < r[:, 2]) & (r[:, 1] <= y) & (y < r[:, 3])]
        want = members[np.lexsort((members, rec["depth"][members]))]
        assert np.array_equal(ids[start[t]:start[t + 1]], want)


def test_tile_lists_equal_full_lists_on_their_tiles():
    # the numpy per-tile builder against the C list builder: every tile of the small workload,
    # and sampled tiles of a world-space scene (all other tiles empty)
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    start, ids, _ = oracle.lists(rec, cam, 1)
    tx, ty, _, _ = oracle.grid(cam)
    s2, i2 = oracle.tile_lists(rec, cam, np.arange(tx * ty))
    assert np.array_equal(start, s2) and np.array_equal(ids, i2)
    sc = scenes.clustered_scene(60_000, seed=31, clusters=16)
    cam = scenes.look_at([3.0, -2.0, 1.0], 640, 360)
    rec = oracle.preprocess(sc, cam)
    start, ids, _ = oracle.lists(rec, cam, 1)
    tx, ty, _, _ = oracle.grid(cam)
    tiles = np.random.default_rng(5).choice(tx * ty, 60, replace=False)
    s2, i2 = oracle.tile_lists(rec, cam, tiles)
    assert int(s2[-1]) > 1000
    for t in range(tx * ty):
        seg = i2[s2[t]:s2[t + 1]]
        if t in set(tiles.tolist()):
            assert np.array_equal(seg, ids[start[t]:start[t + 1]])
        else:
            assert seg.size == 0


@pytest.mark.parametrize("G", [2, 4, 8])
def test_group_lists_filter_to_tile_lists(G):
    # Filtering a depth-sorted group list by a member tile's mask bit gives that tile's list.
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    st1, ids1, _ = oracle.lists(rec, cam, 1)
    stg, idsg, masks = oracle.lists(rec, cam, G)
    tx, ty, gx, gy = oracle.grid(cam, G)
    assert int(masks.max()) < (1 << (G * G))
    for u in range(gx * gy):
        ux, uy = u % gx, u // gx
        seg = idsg[stg[u]:stg[u + 1]]
        mseg = masks[stg[u]:stg[u + 1]]
        assert (mseg != 0).all()
        assert len(set(seg.tolist())) == len(seg)
        for ly in range(G):
            for lx in range(G):
                txx, tyy = ux * G + lx, uy * G + ly
                bit = 1 << (ly * G + lx)
                filt = seg[(mseg & bit) != 0]
                if txx >= tx or tyy >= ty:
                    assert filt.size == 0
                    continue
                t = tyy * tx + txx
                assert np.array_equal(filt, ids1[st1[t]:st1[t + 1]])


def test_load_reduction_counts_by_brute_force():
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    n_total, n_group, lr = oracle.load_reduction(rec, cam, 2)
    vis = np.nonzero(rec["visible"])[0]
    r = rec["rect"][vis]
    tiles = ((r[:, 2] - r[:, 0]) * (r[:, 3] - r[:, 1])).sum()
    groups = 0
    for x0, y0, x1, y1 in r:
        gxs = set(range(x0 // 2, (x1 - 1) // 2 + 1))
        gys = set(range(y0 // 2, (y1 - 1) // 2 + 1))
        groups += len(gxs) * len(gys)
    assert n_total == tiles and n_group == groups
    assert lr == pytest.approx(1 - groups / tiles)


# ------------------------------------------- independent brute-force render ---

def brute_render(sc, cam, bg=(0.0, 0.0, 0.0)):
    """Numpy FP64 render along a different route: complex-step Jacobian, scipy rotation,
    scipy spherical harmonics, global depth sort, direct tile-overlap test per pixel."""
    W, H = cam.width, cam.height
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)
    campos = np.linalg.solve(R, -t)    # the world point that maps to the camera origin
    n = sc.n
    recs = []
    for g in range(n):
        m = sc.mean[:, g].astype(np.float64)
        pc = R @ m + t
        if pc[2] <= cam.znear:
            continue
        w, x, y, z = sc.quat[:, g].astype(np.float64)
        M = Rotation.from_quat([x, y, z, w]).as_matrix()
        V = R @ M @ np.diag(np.exp(2.0 * sc.log_scale[:, g].astype(np.float64))) @ M.T @ R.T
        J = np.zeros((2, 3))
        h = 1e-30
        for k in range(3):
            e = np.zeros(3, complex)
            e[k] = 1j * h
            pz = pc + e
            J[:, k] = np.imag(np.array([cam.fx * pz[0] / pz[2], cam.fy * pz[1] / pz[2]])) / h
        S = J @ V @ J.T + 0.3 * np.eye(2)
        mu = np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])
        r = 3.0 * math.sqrt(np.linalg.eigvalsh(S).max())
        d = m - campos
        d /= np.linalg.norm(d)
        col = np.zeros(3)
        for l in range(sc.sh_degree + 1):
            for mm in range(-l, l + 1):
                col += sc.sh[l * l + l + mm, :, g].astype(np.float64) * real_sh_scipy(l, mm, d)
        col = np.maximum(col + 0.5, 0.0)
        recs.append((pc[2], g, mu, np.linalg.inv(S), float(sc.opacity[g]), col, r))
    recs.sort(key=lambda e: (e[0], e[1]))
    img = np.zeros((3, H, W))
    T_out = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            tx, ty = px // 16, py // 16
            T, C = 1.0, np.zeros(3)
            p = np.array([px + 0.5, py + 0.5])
            for z, g, mu, Q, o, col, r in recs:
                if not (16 * tx <= mu[0] + r and 16 * tx + 16 > mu[0] - r and
                        16 * ty <= mu[1] + r and 16 * ty + 16 > mu[1] - r):
                    continue
                d = p - mu
                a = min(0.99, o * math.exp(-0.5 * d @ Q @ d))
                if a < 1 / 255:
                    continue
                Tn = T * (1 - a)
                if Tn < 1e-4:
                    break
                C += a * T * col
                T = Tn
            img[:, py, px] = C + T * np.asarray(bg)
            T_out[py, px] = T
    return img, T_out


@pytest.mark.parametrize("deg,seed,world", [(0, 11, False), (3, 12, False), (3, 13, True)])
def test_oracle_matches_independent_brute_force(deg, seed, world):
    rng = np.random.default_rng(seed)
    n = 48
    W = H = 32
    if world:
        # world-space Gaussians around the origin seen from a posed camera: exercises the
        # world-to-camera transform and the SH view direction from the camera centre
        cam = scenes.look_at(scenes.sphere_position(rng, 4.0), W, H)
        mean = rng.uniform(-0.8, 0.8, (3, n))
    else:
        cam = scenes.pinhole(W, H, 60.0)
        mean = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(1.0, 3.0, n)])
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0)
    nb = (deg + 1) ** 2
    sh = rng.normal(0, 0.5, (nb, 3, n))
    sc = one_scene(mean, rng.normal(math.log(0.05), 0.4, (3, n)), q,
                   1 / (1 + np.exp(-rng.normal(1.0, 1.0, n))), sh, deg)
    out = oracle.render(sc, cam, bg=(0.05, 0.1, 0.2))
    img, T = brute_render(sc, cam, bg=(0.05, 0.1, 0.2))
    ok = out["ambiguous"] == 0
    assert ok.mean() > 0.95
    assert (out["tfinal"] < 0.9).mean() > 0.1          # the Gaussians actually cover the image
    # The oracle takes the camera centre as -R^T t; the brute force solves R c = -t.  For a
    # float32-rounded rotation the two differ by ~1e-7, which moves the SH view direction.
    tol = 1e-6 if world else 1e-10
    assert np.abs(out["image"] - img)[:, ok].max() < tol
    assert np.abs(out["tfinal"] - T)[ok].max() < 1e-10


# ------------------------------------------------- ambiguity (guard bands) ---

def test_ambiguity_flag_on_alpha_cut():
    # a Gaussian whose alpha at the centre pixel sits just above 1/255 is flagged;
    # one comfortably above is not.
    W = H = 16
    cam = scenes.pinhole(W, H, 60.0)
    for o, flagged in ((np.float32(1 / 255 * (1 + 3e-5)), True), (np.float32(1 / 255 * 1.05), False)):
        z = 2.0
        x = 0.5 * z / cam.fx
        sc = one_scene([x, x, z], [math.log(0.02)] * 3, [1, 0, 0, 0], [o], [0.0, 0.0, 0.0])
        out = oracle.render(sc, cam)
        assert bool(out["ambiguous"][8, 8] & oracle.PIX_ALPHA) == flagged


def test_small_workload_ambiguity_fraction():
    sc, cam = scenes.small_camera_space()
    out = oracle.render(sc, cam)
    assert (out["ambiguous"] != 0).mean() < 1e-3


# --------------------------------------------- the tensorized power (R13) ---

def test_separable_power_expansion_is_exact():
    """The Gaussian-side row k and pixel-side column phi = [x^2, xy, y^2, x, y, 1] (tile-local
    frame) reproduce -1/2 d^T Q d + ln o exactly in rational arithmetic; zero-padding the
    inner dimension (Padding the Inner Dimension) adds only exact zeros."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, c = (Fraction(int(v), 97) + 1 for v in rng.integers(0, 500, 2))
        b = Fraction(int(rng.integers(-50, 50)), 113)
        u, v = (Fraction(int(w), 37) for w in rng.integers(-400, 400, 2))
        lno = Fraction(int(rng.integers(-300, 0)), 59)
        k = [-a / 2, -b, -c / 2, a * u + b * v, b * u + c * v,
             -(a * u * u + 2 * b * u * v + c * v * v) / 2 + lno] + [Fraction(0)] * 10
        for _ in range(5):
            x, y = (int(w) for w in rng.integers(-8, 8, 2))
            phi = [x * x, x * y, y * y, x, y, 1] + [Fraction(0)] * 10
            dx, dy = x - u, y - v
            want = -(a * dx * dx + 2 * b * dx * dy + c * dy * dy) / 2 + lno
            assert sum(p * q for p, q in zip(k, phi)) == want


# ------------------------------------------- opacity-aware tile culling ---

def test_tight_qmin_is_the_rectangle_minimum():
    """tile_qmin against a bounded numerical minimiser of the same quadratic over the
    rectangle of the tile's pixel centres."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(11)
    n = 60
    L = rng.normal(0, 1, (n, 2, 2)) * rng.uniform(0.02, 0.5, (n, 1, 1))
    conic = np.einsum("nij,nkj->nik", L, L) + 1e-3 * np.eye(2)
    rec = {"conic": np.stack([conic[:, 0, 0], conic[:, 0, 1], conic[:, 1, 1]], 1),
           "xy": rng.uniform(-20, 84, (n, 2))}
    cam = scenes.pinhole(64, 64, 60.0)
    tiles = rng.integers(0, 16, n)
    q = oracle.tile_qmin(rec, np.arange(n), tiles, cam)
    for i in range(n):
        x0, y0 = (tiles[i] % 4) * 16 + 0.5, (tiles[i] // 4) * 16 + 0.5
        a, b, c = rec["conic"][i]
        f = lambda p: a * (p[0] - rec["xy"][i, 0]) ** 2 + 2 * b * (p[0] - rec["xy"][i, 0]) * (p[1] - rec["xy"][i, 1]) \
            + c * (p[1] - rec["xy"][i, 1]) ** 2
        best = min(minimize(f, s, bounds=[(x0, x0 + 15), (y0, y0 + 15)], method="L-BFGS-B",
                            options=dict(ftol=1e-15, gtol=1e-12)).fun
                   for s in ([x0, y0], [x0 + 15, y0 + 15], [x0 + 7.5, y0 + 7.5]))
        assert q[i] <= best + 1e-9 * (1 + best)
        assert best - q[i] <= 1e-6 * (1 + best)


def test_tight_culling_drops_only_pairs_below_the_cut_everywhere():
    """Every dropped (Gaussian, tile) pair has alpha < 1/255 at all 256 pixel centres (the
    compositing would skip each of them), and every kept pair is close to the cut somewhere."""
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    start, ids, _ = oracle.lists(rec, cam, 1)
    tx, _, _, _ = oracle.grid(cam)
    tiles = np.repeat(np.arange(len(start) - 1), np.diff(start))
    keep, _ = oracle.tight_keep(rec, ids, tiles, cam)
    assert 0.2 < keep.mean() < 0.95
    px, py = np.meshgrid(np.arange(16) + 0.5, np.arange(16) + 0.5)
    for g, t, k in zip(ids, tiles, keep):
        dx = (t % tx) * 16 + px - rec["xy"][g, 0]
        dy = (t // tx) * 16 + py - rec["xy"][g, 1]
        a, b, c = rec["conic"][g]
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        alpha = np.minimum(0.99, rec["opacity"][g] * np.exp(-0.5 * q))
        if not k:
            assert alpha.max() < 1.0 / 255.0
        else:
            assert q.min() <= 2 * np.log(255 * rec["opacity"][g]) + oracle.TIGHT_MARGIN + 2 * (abs(a) + abs(b) + abs(c)) * 16


def test_tight_lists_leave_the_image_unchanged():
    sc, cam = scenes.small_camera_space()
    rec = oracle.preprocess(sc, cam)
    start, ids, _ = oracle.lists(rec, cam, 1)
    full = oracle.composite(rec, cam, start, ids, nthreads=4)
    st2, ids2, _, keep = oracle.tight_lists(rec, cam, start, ids)
    assert ids2.size < 0.9 * ids.size
    tight = oracle.composite(rec, cam, st2, ids2, nthreads=4)
    for k in ("image", "tfinal", "wsum"):
        assert np.array_equal(full[k], tight[k])
    assert (tight["neval"] <= full["neval"]).all() and tight["neval"].sum() < full["neval"].sum()


def test_tight_isotropic_closed_form():
    """An isotropic Gaussian keeps exactly the tiles whose pixel-centre rectangle lies within
    rho = sigma sqrt(2 ln(255 o) + margin) of its centre (distance from a point to a box)."""
    sigma, o = 9.0, 0.6
    cam = scenes.pinhole(160, 128, 60.0)
    rec = {"conic": np.array([[1 / sigma ** 2, 0.0, 1 / sigma ** 2]]), "xy": np.array([[70.3, 57.9]]),
           "opacity": np.array([o])}
    tiles = np.arange(10 * 8)
    keep, _ = oracle.tight_keep(rec, np.zeros(tiles.size, np.int64), tiles, cam)
    rho = sigma * np.sqrt(2 * np.log(255 * o) + oracle.TIGHT_MARGIN)
    x0, y0 = (tiles % 10) * 16 + 0.5, (tiles // 10) * 16 + 0.5
    ddx = np.maximum(np.maximum(x0 - 70.3, 70.3 - (x0 + 15)), 0)
    ddy = np.maximum(np.maximum(y0 - 57.9, 57.9 - (y0 + 15)), 0)
    assert np.array_equal(keep, np.hypot(ddx, ddy) <= rho)
    assert 4 < keep.sum() < 40


@pytest.mark.parametrize("G", [1, 2, 4, 8])
def test_tight_group_lists_filter_to_tight_tile_lists(G):
    """Opacity-aware culling decides each member tile of a group on its own: filtering the
    culled group lists by a member tile's mask bit gives that tile's culled list, in order,
    and no kept entry has an empty mask."""
    sc = scenes.camera_box_scene(3000, seed=41, log_scale_mu=math.log(0.03), log_scale_sigma=0.9)
    cam = scenes.pinhole(200, 136, 60.0)
    rec = oracle.preprocess(sc, cam)
    st1, ids1, _ = oracle.lists(rec, cam, 1)
    tst1, tids1, _, _ = oracle.tight_lists(rec, cam, st1, ids1)
    stg, idsg, masks, _ = oracle.tight_group_lists(rec, cam, G)
    tx, ty, gx, gy = oracle.grid(cam, G)
    assert (masks != 0).all()
    assert idsg.size < oracle.lists(rec, cam, G)[0][-1]
    seen = 0
    for u in range(gx * gy):
        seg, mseg = idsg[stg[u]:stg[u + 1]], masks[stg[u]:stg[u + 1]]
        for ly in range(G):
            for lx in range(G):
                txx, tyy = (u % gx) * G + lx, (u // gx) * G + ly
                if txx >= tx or tyy >= ty:
                    continue
                t = tyy * tx + txx
                filt = seg[(mseg & np.uint64(1 << (ly * G + lx))) != 0]
                assert np.array_equal(filt, tids1[tst1[t]:tst1[t + 1]]), (G, u, lx, ly)
                seen += filt.size
    assert seen == tids1.size
