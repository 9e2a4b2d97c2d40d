"""Pins of the oracle's per-pixel forward pass: colour and transmission
(Eq. 1-3), opaque-disc depth (Eq. 4-5), index map, and binning (supp. B)."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests.scenes_small import (all_pixels, edge_on_surfels, identity_pose, random_pose, random_scene, scene_from,
                                small_cam)

CAM = small_cam()
W, H = CAM["width"], CAM["height"]


def _render_all(sc, pose=None, cam=CAM, **kw):
    P = orc.make_params(cam, **kw)
    poses = identity_pose() if pose is None else np.asarray(pose).reshape(-1, 12)
    recs = orc.project(P, sc, poses)
    pix = all_pixels(poses.shape[0], cam["height"], cam["width"])
    out = orc.render(P, recs, sc, pix)
    shp = (poses.shape[0], cam["height"], cam["width"])
    return {k: (v.reshape(shp + (3,)) if k == "color" else v.reshape(shp)) for k, v in out.items()}, recs


def _f_closed(alpha, mu, sig2, xs, ys):
    """alpha exp(-1/2 d^2) for an axis-aligned Sigma_2D = diag(sig2)."""
    d2 = (xs + 0.5 - mu[0]) ** 2 / sig2[0] + (ys + 0.5 - mu[1]) ** 2 / sig2[1]
    return alpha * np.exp(-0.5 * d2), d2


def test_single_gaussian_closed_form():
    """One Gaussian: C = c f, T = 1 - f inside the cut-off, nothing outside."""
    Z, s = 2.0, 0.06
    a = float(np.float32(0.8))
    c = np.array([0.2, 0.5, 0.9], np.float32)
    # on the optical axis J is diagonal, so Sigma_2D = diag((f sx/Z)^2, (f sy/Z)^2)
    sc = scene_from([[0.0, 0.0, Z]], [[s, s / 2, s / 10]], [[1, 0, 0, 0]], [a], [c])
    out, recs = _render_all(sc)
    s32 = np.float64(np.float32(s))
    sig2 = ((100 * s32 / Z) ** 2, (100 * np.float64(np.float32(s / 2)) / Z) ** 2)
    mu = (64.0, 48.0)
    ys, xs = np.mgrid[0:H, 0:W]
    f, d2 = _f_closed(a, mu, sig2, xs, ys)
    inside = out["nlist"][0] == 1
    assert inside.sum() > 100
    # the cut-off region matches d^2 <= 9 away from its boundary
    assert (inside[d2 < 9 - 1e-4]).all() and not (inside[d2 > 9 + 1e-4]).any()
    np.testing.assert_allclose(out["trans"][0][inside], 1 - f[inside], rtol=1e-12)
    for ch in range(3):
        np.testing.assert_allclose(out["color"][0][..., ch][inside], np.float64(c[ch]) * f[inside], rtol=1e-12)
    assert (out["trans"][0][~inside] == 1.0).all() and (out["color"][0][~inside] == 0.0).all()
    assert (out["depth"][0][~inside] == -1.0).all() and (out["index"][0][~inside] == -1).all()


def test_two_gaussians_front_to_back_and_swap():
    """C = c1 f1 + c2 f2 (1 - f1) with 1 in front; swapping depths swaps roles."""
    c1, c2 = np.array([1.0, 0, 0], np.float32), np.array([0, 0, 1.0], np.float32)
    a1, a2 = float(np.float32(0.5)), float(np.float32(0.7))

    def scene(z1, z2):
        return scene_from([[0, 0, z1], [0.0, 0, z2]],
                          [[0.05 * z1 / 2, 0.05 * z1 / 2, 0.002], [0.05 * z2 / 2, 0.05 * z2 / 2, 0.002]],
                          [[1, 0, 0, 0], [1, 0, 0, 0]], [a1, a2], [c1, c2])
    o12, r12 = _render_all(scene(2.0, 3.0))
    o21, r21 = _render_all(scene(3.0, 2.0))
    ys, xs = np.mgrid[0:H, 0:W]

    def f_of(recs, i):
        r = recs[0, i]
        sig2 = (r["cov"][0], r["cov"][2])
        return _f_closed([a1, a2][i], r["mu"], sig2, xs, ys)[0]
    f1, f2 = f_of(r12, 0), f_of(r12, 1)
    both = o12["nlist"][0] == 2
    assert both.sum() > 50
    expect = np.float64(c1)[None] * f1[both][:, None] + np.float64(c2)[None] * (f2 * (1 - f1))[both][:, None]
    np.testing.assert_allclose(o12["color"][0][both], expect, rtol=1e-12, atol=1e-15)
    g1, g2 = f_of(r21, 0), f_of(r21, 1)
    both2 = o21["nlist"][0] == 2
    expect2 = np.float64(c2)[None] * g2[both2][:, None] + np.float64(c1)[None] * (g1 * (1 - g2))[both2][:, None]
    np.testing.assert_allclose(o21["color"][0][both2], expect2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(o12["trans"][0][both], ((1 - f1) * (1 - f2))[both], rtol=1e-12)


def test_opaque_disc_normal_incidence():
    """An opaque disc facing the camera: depth is exactly Z0 on the pixels
    where f > e^-1/2, i.e. (dx^2 + dy^2)/sigma^2 < 1 + 2 ln alpha, else -1."""
    Z0, a = 2.0, 0.2
    alpha = float(np.float32(0.99))
    sc = scene_from([[0, 0, Z0]], [[a, a, 0.1 * a]], [[1, 0, 0, 0]], [alpha], [[1, 1, 1]])
    out, _ = _render_all(sc)
    ys, xs = np.mgrid[0:H, 0:W]
    sig = 100 * np.float64(np.float32(a)) / Z0
    rho2 = ((xs + 0.5 - 64) ** 2 + (ys + 0.5 - 48) ** 2) / sig ** 2
    tau = 1 + 2 * np.log(alpha)
    hit = out["index"][0] == 0
    assert hit.sum() > 100
    assert (hit[rho2 < tau - 1e-5]).all() and not hit[rho2 > tau + 1e-5].any()
    assert (out["depth"][0][hit] == Z0).all()
    assert (out["depth"][0][~hit] == -1.0).all()
    assert (out["branch"][0][hit] == 1).all()


@pytest.mark.parametrize("seed", [0, 1])
def test_tilted_disc_against_world_ray_plane(seed):
    """A tilted opaque disc seen by a randomly posed camera: on hit pixels
    whose ray is within 60 degrees of the disc normal, the depth equals the
    camera z of the world-space ray/plane intersection; elsewhere it is the
    centre depth (Eq. 5)."""
    rng = np.random.default_rng(seed)
    pose, Rg, tg = random_pose(rng)
    phi = np.radians(62.0)
    n_cam = np.array([np.sin(phi), 0.0, np.cos(phi)])
    # disc centre 2.5 m ahead of the camera, thin axis along n_cam
    pc = np.array([0.05, -0.02, 2.5])
    from scipy.spatial.transform import Rotation
    t1 = np.cross(n_cam, [0.0, 1.0, 0.0])
    t1 /= np.linalg.norm(t1)
    t2 = np.cross(n_cam, t1)
    R_cam = np.stack([t1, t2, n_cam], 1)
    R_world = Rg @ R_cam
    q = Rotation.from_matrix(R_world).as_quat()
    p_world = Rg @ pc + tg
    sc = scene_from([p_world], [[1.0, 1.0, 0.1]], [[q[3], q[0], q[1], q[2]]], [0.99], [[1, 1, 1]])
    out, recs = _render_all(sc, pose=pose)
    hit = out["index"][0] == 0
    assert hit.sum() > 500
    ys, xs = np.mgrid[0:H, 0:W]
    d_cam = np.stack([(xs + 0.5 - 64) / 100.0, (ys + 0.5 - 48) / 100.0, np.ones_like(xs, float)], -1)
    d_world = d_cam @ Rg.T
    p32 = sc["pos"][0].astype(np.float64)
    n_world = R_world[:, 2]
    # the disc's normal as the oracle sees it (from the float32 quaternion)
    qq = sc["rot"][0].astype(np.float64)
    n_world = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()[:, 2]
    theta = ((p32 - tg) @ n_world) / (d_world @ n_world)
    cosang = np.abs(d_world @ n_world) / np.linalg.norm(d_world, axis=-1)
    plane = hit & (cosang > 0.5 + 1e-6)
    centre = hit & (cosang < 0.5 - 1e-6)
    assert plane.sum() > 50 and centre.sum() > 50
    np.testing.assert_allclose(out["depth"][0][plane], theta[plane], rtol=1e-10)
    assert (out["branch"][0][plane] == 1).all()
    assert (out["branch"][0][centre] == 2).all()
    zc = (Rg.T @ (p32 - tg))[2]
    np.testing.assert_allclose(out["depth"][0][centre], zc, rtol=1e-14)


def test_transparent_only_scene_has_no_depth():
    rng = np.random.default_rng(3)
    sc = random_scene(rng, 300, opaque_frac=0.0)
    out, _ = _render_all(sc)
    assert (out["nlist"] > 0).sum() > 1000
    assert (out["depth"] == -1).all() and (out["index"] == -1).all()


def test_invariants_random_scene():
    """T in [0,1]; colour inside the convex hull of the Gaussian colours:
    C = sum w_i c_i with w_i >= 0 and sum w_i = 1 - T."""
    rng = np.random.default_rng(4)
    sc = random_scene(rng, 1500, spread=0.7)
    sc["color"] = rng.uniform(0.3, 0.6, (1500, 3)).astype(np.float32)
    out, _ = _render_all(sc)
    T, C = out["trans"][0], out["color"][0]
    assert (T >= 0).all() and (T <= 1).all()
    cov = 1 - T > 1e-9
    ratio = C[cov] / (1 - T[cov])[:, None]
    assert ratio.min() >= 0.3 - 1e-9 and ratio.max() <= 0.6 + 1e-9
    assert (out["nlist"] > 3).mean() > 0.5


def test_adding_a_gaussian_behind():
    """Appending a Gaussian behind everything multiplies T by (1 - f) and
    adds c f T_old to the colour; T never increases."""
    rng = np.random.default_rng(6)
    sc = random_scene(rng, 400, spread=0.4, centre=(0, 0, 2.0))
    out0, _ = _render_all(sc)
    extra = scene_from([[0.05, 0.0, 4.0]], [[0.3, 0.2, 0.03]], [[0.9, 0.1, 0.2, 0.3]], [0.6], [[0.3, 0.7, 0.1]])
    sc2 = {k: np.concatenate([sc[k], extra[k]]) for k in sc}
    out1, recs1 = _render_all(sc2)
    assert (out1["trans"] <= out0["trans"] + 1e-15).all()
    r = recs1[0, 400]
    ys, xs = np.mgrid[0:H, 0:W]
    dx, dy = xs + 0.5 - r["mu"][0], ys + 0.5 - r["mu"][1]
    dd = r["conic"][0] * dx * dx + 2 * r["conic"][1] * dx * dy + r["conic"][2] * dy * dy
    f = np.float64(np.float32(0.6)) * np.exp(-0.5 * dd)
    touched = out1["nlist"][0] == out0["nlist"][0] + 1
    assert touched.sum() > 200
    np.testing.assert_allclose(out1["trans"][0][touched], (out0["trans"][0] * (1 - f))[touched], rtol=1e-11)
    dC = out1["color"][0] - out0["color"][0]
    np.testing.assert_allclose(dC[touched], (extra["color"][0].astype(np.float64)[None] *
                                             (f * out0["trans"][0])[touched][:, None]), rtol=1e-9, atol=1e-14)


def test_permutation_invariance():
    rng = np.random.default_rng(8)
    sc = random_scene(rng, 500)
    out0, _ = _render_all(sc)
    perm = rng.permutation(500)
    sc2 = {k: v[perm] for k, v in sc.items()}
    out1, _ = _render_all(sc2)
    np.testing.assert_allclose(out1["color"], out0["color"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(out1["depth"], out0["depth"], rtol=1e-13)
    hit = out0["index"] >= 0
    assert (perm[out1["index"][hit]] == out0["index"][hit]).all()


def test_subset_of_pixels_equals_full_render():
    rng = np.random.default_rng(9)
    sc = random_scene(rng, 300)
    P = orc.make_params(CAM)
    recs = orc.project(P, sc, identity_pose())
    full = orc.render(P, recs, sc, all_pixels(1, H, W))
    idx = rng.choice(H * W, 500, replace=False)
    sub = orc.render(P, recs, sc, all_pixels(1, H, W)[idx])
    for k in full:
        assert np.array_equal(full[k][idx], sub[k])


# ---------------------------------------------------------------- binning

def _box(P, a, mux):
    xe = min(a * P.tile_w + P.tile_w, P.width)
    return (a * P.tile_w + 0.5) - mux, (xe - 0.5) - mux


def _row_interval(P, r, b):
    """The pair thinning rule of the binning spec, restated (binary64, fixed
    order): the x-range (xl, xh) of the margin-inflated decision ellipse
    inside tile row b's band of pixel centres, None when the band misses
    it, the whole line when the binary32 conic is not positive definite."""
    tw, th, H = P.tile_w, P.tile_h, P.height
    a0, a1 = int(r["rect"][0]) // tw, int(r["rect"][1]) // tw
    qa, qb, qc = (float(np.float64(v)) for v in r["conic32"])
    det = qa * qc - qb * qb
    if not (qa > 0.0 and det > 0.0):
        return -np.inf, np.inf
    mux, muy = float(np.float64(r["mu32"][0])), float(np.float64(r["mu32"][1]))
    ly, hy = (b * th + 0.5) - muy, (min(b * th + th, H) - 0.5) - muy
    X = max(-_box(P, a0, mux)[0], _box(P, a1, mux)[1])
    Y = max(-ly, hy)
    M = ((qa * X) * X + ((2.0 * abs(qb)) * X) * Y) + (qc * Y) * Y
    c = (float(np.float32(P.cutoff2)) * 1.001 + 1e-3) + 1e-6 * M
    xt = math.sqrt((c * qc) / det)
    yt = -(qb * xt) / qc
    ends = []
    for yp, sign in ((yt, 1.0), (-yt, -1.0)):
        if ly <= yp <= hy:
            ends.append(sign * xt)
            continue
        ye = ly if yp < ly else hy
        D = qa * c - det * (ye * ye)
        if D < 0.0:
            return None
        ends.append((-(qb * ye) + sign * math.sqrt(D)) / qa)
    return ends[1], ends[0]


def _tile_keeps(P, r, a, b):
    iv = _row_interval(P, r, b)
    if iv is None:
        return False
    lo, hi = _box(P, a, float(np.float64(r["mu32"][0])))
    return lo <= iv[1] and hi >= iv[0]


def _brute_pairs(P, recs, mask):
    F, N = recs.shape
    tw, th = P.tile_w, P.tile_h
    tx = (P.width + tw - 1) // tw
    ty = (P.height + th - 1) // th
    out = []
    for f in range(F):
        for t in range(tx * ty):
            a, b = t % tx, t // tx
            if not mask[f, b * th:(b + 1) * th, a * tw:(a + 1) * tw].any():
                continue
            lst = []
            for i in range(N):
                r = recs[f, i]
                if not r["visible"]:
                    continue
                x0, x1, y0, y1 = r["rect"]
                if x0 // tw <= a <= x1 // tw and y0 // th <= b <= y1 // th and _tile_keeps(P, r, a, b):
                    lst.append((np.float32(r["z32"]), i))
            lst.sort()
            out += [(f, t, i) for _, i in lst]
    return out


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_binning_brute_force(tile):
    rng = np.random.default_rng(10)
    sc = random_scene(rng, 120, spread=0.8)
    pose2, _, _ = random_pose(rng)
    poses = np.stack([identity_pose()[0], identity_pose()[0]])
    P = orc.make_params(CAM, tile=tile)
    recs = orc.project(P, sc, poses)
    mask = (rng.random((2, H, W)) < 0.02).astype(np.uint8)
    mask[1] = 0
    mask[1, 10:40, 20:90] = 1
    b = orc.bin_pairs(P, recs, mask)
    brute = _brute_pairs(P, recs, mask)
    assert b["K"] == len(brute) and b["K"] > 100
    got = list(zip(b["frame"].tolist(), b["tile"].tolist(), b["gid"].tolist()))
    assert got == brute


def test_binning_covers_every_contributing_pixel():
    """No pixel can receive a Gaussian that has no pair with the pixel's
    tile: every (pixel, Gaussian) with d^2 <= 9 is backed by a pair."""
    rng = np.random.default_rng(11)
    sc = random_scene(rng, 150, spread=0.8, smin=0.003, smax=0.15)
    P = orc.make_params(CAM, tile=(16, 16))
    recs = orc.project(P, sc, identity_pose())
    b = orc.bin_pairs(P, recs, np.ones((1, H, W), np.uint8))
    pairs = set(zip(b["tile"].tolist(), b["gid"].tolist()))
    ys, xs = np.mgrid[0:H, 0:W]
    tiles = (ys // 16) * 8 + xs // 16
    for i in range(150):
        r = recs[0, i]
        if r["culled"]:
            continue
        dx = xs + 0.5 - np.float64(r["mu32"][0])
        dy = ys + 0.5 - np.float64(r["mu32"][1])
        a, bb, c = (np.float64(v) for v in r["conic32"])
        inside = a * dx * dx + 2 * bb * dx * dy + c * dy * dy <= 9.0 * (1 + 1e-5)
        for t in np.unique(tiles[inside]):
            assert (int(t), i) in pairs


def test_pair_thinning_drops_only_unreachable_tiles():
    """Every rectangle tile the thinning rule drops has d^2 > cut-off at all
    of its pixel centres (exact quadratic form), and the rule drops a real
    share of the rectangle pairs of thin, tilted surfels."""
    rng = np.random.default_rng(12)
    sc = random_scene(rng, 200, spread=0.8, smin=0.005, smax=0.12)
    sc["scale"][:, 2] = sc["scale"][:, 0] * 0.05
    P = orc.make_params(CAM, tile=(8, 8))
    recs = orc.project(P, sc, identity_pose())
    ys, xs = np.mgrid[0:H, 0:W]
    rect_pairs = dropped = 0
    for i in range(200):
        r = recs[0, i]
        if not r["visible"]:
            continue
        x0, x1, y0, y1 = r["rect"]
        for b in range(y0 // 8, y1 // 8 + 1):
            for a in range(x0 // 8, x1 // 8 + 1):
                rect_pairs += 1
                if _tile_keeps(P, r, a, b):
                    continue
                dropped += 1
                tx, ty = xs[b * 8:(b + 1) * 8, a * 8:(a + 1) * 8], ys[b * 8:(b + 1) * 8, a * 8:(a + 1) * 8]
                dx = tx + 0.5 - np.float64(r["mu32"][0])
                dy = ty + 0.5 - np.float64(r["mu32"][1])
                qa, qb, qc = (np.float64(v) for v in r["conic32"])
                assert (qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy > 9.0).all()
    assert rect_pairs > 500 and dropped > 0.2 * rect_pairs


def _decision32(mu, q32, xs, ys):
    """The per-pixel binary32 form of the decision layer: offsets from the
    binary32 centre, two products, then two fused multiply-adds (each fused
    step evaluated exactly in binary64 products and rounded to binary32 after
    one binary64 addition, which differs from a single rounding only on a
    binary32 tie)."""
    f32 = np.float32
    dx = (xs.astype(f32) + f32(0.5)) - f32(mu[0])
    dy = (ys.astype(f32) + f32(0.5)) - f32(mu[1])
    qa, qb, qc = (f32(v) for v in q32)
    t0 = (qa * dx) * dx
    t1 = ((f32(2.0) * qb * dx).astype(np.float64) * dy + t0).astype(f32)
    return ((qc * dy).astype(np.float64) * dy + t1).astype(f32)


def _needles(rng, n):
    """Records of thin, long footprints in the small camera: minor-axis
    eigenvalue 10^1 .. 10^6 (edge-on surfels), major sigma 3 .. 40 px, any
    orientation; rectangles from the exact extent plus two pixels."""
    recs = np.zeros((1, n), dtype=orc.REC_DTYPE)
    for i in range(n):
        lam1 = 10 ** rng.uniform(1.0, 6.0)
        lam2 = 1.0 / rng.uniform(3.0, 40.0) ** 2
        th = rng.uniform(0.0, np.pi)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        Q = (R * [lam1, lam2]) @ R.T
        q32 = np.array([Q[0, 0], Q[0, 1], Q[1, 1]], np.float32)
        mu = np.array([rng.uniform(0, W), rng.uniform(0, H)], np.float32)
        ex, ey = 3.0 * np.sqrt(1.0 / lam2), 3.0 * np.sqrt(1.0 / lam2)
        r = recs[0, i]
        r["visible"] = 1
        r["mu32"] = mu
        r["conic32"] = q32
        r["z32"] = np.float32(rng.uniform(1.0, 5.0))
        r["rect"] = [max(0, int(np.floor(mu[0] - ex)) - 2), min(W - 1, int(np.ceil(mu[0] + ex)) + 2),
                     max(0, int(np.floor(mu[1] - ey)) - 2), min(H - 1, int(np.ceil(mu[1] + ey)) + 2)]
    return recs


def test_pair_thinning_conservative_on_needle_footprints():
    """Needle footprints, where the binary32 rounding of the per-pixel form
    is large against the cut-off (up to several units at the tips): every
    rectangle pixel that passes the binary32 decision (d^2 <= 9), and every
    one whose exact q is within 9 plus the binary32 evaluation bound
    7 * 2^-24 * (qa dx^2 + |2 qb dx dy| + qc dy^2), lies in a kept tile; the
    rule drops a large share of the rectangle tiles; and the reference
    binning keeps exactly the tiles the rule names."""
    rng = np.random.default_rng(21)
    n = 700
    P = orc.make_params(CAM, tile=(8, 8))
    recs = _needles(rng, n)
    ys, xs = np.mgrid[0:H, 0:W]
    u = 2.0 ** -24
    rect_pairs = dropped = tips = 0
    for i in range(n):
        r = recs[0, i]
        x0, x1, y0, y1 = r["rect"]
        kept = {(a, b) for b in range(y0 // 8, y1 // 8 + 1) for a in range(x0 // 8, x1 // 8 + 1)
                if _tile_keeps(P, r, a, b)}
        nr = (x1 // 8 - x0 // 8 + 1) * (y1 // 8 - y0 // 8 + 1)
        rect_pairs += nr
        dropped += nr - len(kept)
        dx = xs + 0.5 - np.float64(r["mu32"][0])
        dy = ys + 0.5 - np.float64(r["mu32"][1])
        qa, qb, qc = (np.float64(v) for v in r["conic32"])
        q = qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy
        mag = qa * dx * dx + np.abs(2 * qb * dx * dy) + qc * dy * dy
        inrect = (xs >= x0) & (xs <= x1) & (ys >= y0) & (ys <= y1)
        passes = inrect & (_decision32(r["mu32"], r["conic32"], xs, ys) <= np.float32(9.0))
        tips += int((passes & (q > 9.0 * 1.001 + 1e-3)).sum())
        for yy, xx in zip(*np.nonzero(passes | (inrect & (q <= 9.0 + 7.0 * u * mag)))):
            assert (xx // 8, yy // 8) in kept, (i, xx, yy)
    assert dropped > 0.3 * rect_pairs
    assert tips > 0          # pixels only the magnitude term of the margin covers
    sub = recs[:, :120].copy()
    b = orc.bin_pairs(P, sub, np.ones((1, H, W), np.uint8))
    got = list(zip(b["frame"].tolist(), b["tile"].tolist(), b["gid"].tolist()))
    assert got == _brute_pairs(P, sub, np.ones((1, H, W), np.uint8))


def _plain_range(mu, r2):
    """Pixel range of the rectangle rule with the bare cut-off (no allowance
    for binary32 rounding): E the least integer with E^2 >= r2."""
    e = math.ceil(math.sqrt(r2))
    while e > 0 and (e - 1) ** 2 >= r2:
        e -= 1
    while e * e < r2:
        e += 1
    c = math.floor(mu)
    return c - e - 2, c + e + 1


def test_rect_and_pairs_cover_binary32_decisions_of_edge_on_surfels():
    """Needle footprints of surfels seen edge-on: the binary32 decision
    admits pixels beyond the rho^2 ellipse of the binary64 covariance (some
    even beyond the rectangle of the bare cut-off); every pixel it admits
    lies in the record's rectangle and its tile holds the pair, so the
    binning loses no pixel that the per-pixel definition renders."""
    rng = np.random.default_rng(5)
    n = 400
    sc = edge_on_surfels(rng, n)
    P = orc.make_params(CAM, tile=(8, 8))
    recs = orc.project(P, sc, identity_pose())
    b = orc.bin_pairs(P, recs, np.ones((1, H, W), np.uint8))
    pairs = set(zip(b["tile"].tolist(), b["gid"].tolist()))
    ys, xs = np.mgrid[0:H, 0:W]
    tx = (W + 7) // 8
    hits = beyond = 0
    for i in range(n):
        r = recs[0, i]
        if r["culled"]:
            continue
        passes = _decision32(r["mu32"], r["conic32"], xs, ys) <= np.float32(9.0)
        if not passes.any():
            continue
        assert r["visible"], i
        x0, x1, y0, y1 = r["rect"]
        py, px = np.nonzero(passes)
        assert px.min() >= x0 and px.max() <= x1 and py.min() >= y0 and py.max() <= y1, i
        for t in np.unique((py // 8) * tx + px // 8):
            assert (int(t), i) in pairs, (i, t)
        ax = _plain_range(float(r["mu"][0]), 9.0 * float(r["cov"][0]))
        ay = _plain_range(float(r["mu"][1]), 9.0 * float(r["cov"][2]))
        beyond += int(((px < ax[0]) | (px > ax[1]) | (py < ay[0]) | (py > ay[1])).sum())
        hits += len(px)
    assert hits > 500 and beyond > 0


def test_filter50_against_block_counts():
    rng = np.random.default_rng(12)
    cam = small_cam(100, 70)
    P = orc.make_params(cam)
    mask = (rng.random((2, 70, 100)) < rng.uniform(0.2, 0.8, (2, 1, 1))).astype(np.uint8)
    out = orc.filter50(P, mask)
    pad = np.zeros((2, 80, 112), np.uint8)
    pad[:, :70, :100] = mask
    valid = np.zeros((80, 112), np.uint8)
    valid[:70, :100] = 1
    cnt = pad.reshape(2, 5, 16, 7, 16).sum(axis=(2, 4))
    area = valid.reshape(5, 16, 7, 16).sum(axis=(1, 3))
    keep = (2 * cnt >= area[None]).astype(np.uint8)
    expect = (pad * np.repeat(np.repeat(keep, 16, 1), 16, 2))[:, :70, :100]
    assert np.array_equal(out, expect)


def test_unstable_mask_is_transmission_below_one():
    """M_unstable = {T_unstable < 1}: render with the unstable Gaussians
    alone and compare with the coverage helper."""
    rng = np.random.default_rng(13)
    sc = random_scene(rng, 400, unstable_frac=0.3)
    P = orc.make_params(CAM)
    recs = orc.project(P, sc, identity_pose())
    m = orc.unstable_mask_image(P, recs, sc["unstable"])
    keep = sc["unstable"] != 0
    sub = {k: v[keep] for k, v in sc.items()}
    out, _ = _render_all(sub)
    assert 0.05 < m.mean() < 0.95
    assert np.array_equal(m[0] != 0, out["trans"][0] < 1.0)


def test_opacity_clamp_closed_form_and_zero_gradient():
    """alpha = 1 at the centre of a single Gaussian: f = min(alpha g, 0.99) =
    0.99, so C = 0.99 c and T = 0.01 there; the clamp makes f (and C, T)
    locally constant in alpha, so the opacity gradient of that pixel is 0
    (central difference agrees), while an off-centre pixel where alpha g <
    0.99 keeps the unclamped gradient c g."""
    Z, s = 2.0, 0.2
    c = np.array([0.2, 0.5, 0.9], np.float32)
    sc = scene_from([[0.0, 0.0, Z]], [[s, s, s / 10]], [[1, 0, 0, 0]], [1.0], [c])
    P = orc.make_params(CAM)
    poses = identity_pose()
    recs = orc.project(P, sc, poses)
    centre = np.array([[0, 63, 47]], np.int32)          # pixel centre (63.5, 47.5) at ~0.5 px from mu
    off = np.array([[0, 66, 47]], np.int32)
    out = orc.render(P, recs, sc, centre)
    sig = 100 * np.float64(np.float32(s)) / Z
    g = math.exp(-0.5 * (0.5 ** 2 + 0.5 ** 2) / sig ** 2)
    assert g > 0.99
    np.testing.assert_allclose(out["color"][0], 0.99 * c.astype(np.float64), rtol=1e-15)
    np.testing.assert_allclose(out["trans"][0], 0.01, rtol=1e-12)
    for pix, clamped in ((centre, True), (off, False)):
        gC = np.array([[1.0, -2.0, 0.5]])
        gD = np.zeros(1)
        grads = orc.backward(P, recs, sc, poses, pix, gC, gD)
        ref = orc.render(P, recs, sc, pix)
        if clamped:
            assert grads["opacity"][0] == 0.0
        else:
            gi = math.exp(-0.5 * (2.5 ** 2 + 0.5 ** 2) / sig ** 2)   # centre (66.5, 47.5), mu (64, 48)
            np.testing.assert_allclose(grads["opacity"][0], float((gC[0] * c).sum()) * gi, rtol=1e-9)
        # central difference in alpha (float32 steps of 1e-3 below 1)
        vals = []
        for a in (np.float32(0.999), np.float32(0.998)):
            sc2 = dict(sc)
            sc2["opacity"] = np.array([a], np.float32)
            o = orc.render(P, orc.project(P, sc2, poses), sc2, pix)
            vals.append(float((o["color"][0] * gC[0]).sum()))
        fd = (vals[0] - vals[1]) / float(np.float32(0.999) - np.float32(0.998))
        if clamped:
            assert fd == 0.0
        else:
            np.testing.assert_allclose(fd, grads["opacity"][0], rtol=1e-5)
        assert ref["trans"][0] < 1.0


@pytest.mark.parametrize("alpha", [0.7, 0.9, 0.99])
def test_depth_hit_is_the_opacity_threshold(alpha):
    """The depth hit of Eq. 4 is the first Gaussian whose per-pixel opacity
    alpha exp(-d^2 / 2) exceeds e^-1/2, tested here from that definition in
    binary64 on the value-layer distance, not through tau: on every pixel of
    a single Gaussian the oracle hits exactly there, except within 1e-6 of
    the threshold (where the binary32 decision distance may fall either
    side)."""
    a = float(np.float32(alpha))
    sc = scene_from([[0.05, -0.03, 2.0]], [[0.3, 0.2, 0.03]], [[0.9, 0.1, 0.3, 0.2]], [a], [[0.5, 0.5, 0.5]])
    out, recs = _render_all(sc)
    r = recs[0, 0]
    ys, xs = np.mgrid[0:H, 0:W]
    dx, dy = xs + 0.5 - r["mu"][0], ys + 0.5 - r["mu"][1]
    qa, qb, qc = r["conic"]
    f = a * np.exp(-0.5 * (qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy))
    want = f > math.exp(-0.5)
    hit = out["index"][0] == 0
    near = np.abs(f - math.exp(-0.5)) < 1e-6
    assert want.sum() > 20
    assert np.array_equal(hit[~near], want[~near])
    assert near.sum() <= 2
