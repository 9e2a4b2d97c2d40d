"""Pins of the SH colour oracle (oracle/sh.py) against what the mathematics
fixes: orthonormality of the basis on the sphere (exact quadrature), the
addition theorem per band (Legendre polynomials), the gradient table against
finite differences of the basis, the reduction of a DC-only SH colour to the
RGB render, and the chain rule of the SH backward against central finite
differences of the SH render."""
import numpy as np
import pytest
from numpy.polynomial import legendre

from oracle import oracle as orc
from oracle import sh
from tests.scenes_small import all_pixels, identity_pose, random_pose, random_scene, small_cam


def _sphere_quadrature(nz=8, nphi=16):
    """Gauss-Legendre in z = cos(theta) times uniform phi: exact for
    polynomials on the sphere of degree < min(2 nz, nphi)."""
    z, wz = legendre.leggauss(nz)
    phi = 2.0 * np.pi * np.arange(nphi) / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    s = np.sqrt(1.0 - Z * Z)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z], -1).reshape(-1, 3)
    w = np.repeat(wz, nphi) * (2.0 * np.pi / nphi)
    return d, w


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_basis_is_orthonormal_on_the_sphere(degree):
    d, w = _sphere_quadrature()
    Y = sh.basis(d, degree)
    assert Y.shape == (len(d), (degree + 1) ** 2)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(G.shape[0]), atol=1e-12)


def test_addition_theorem_per_band():
    """sum_m Y_lm(a) Y_lm(b) = (2l + 1) / (4 pi) P_l(a . b): fixes every
    function of a band up to a common rotation of the band, including the
    relative signs a wrong table would break."""
    rng = np.random.default_rng(0)
    a = rng.standard_normal((200, 3))
    b = rng.standard_normal((200, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    Ya, Yb = sh.basis(a, 3), sh.basis(b, 3)
    cos = (a * b).sum(1)
    for l in range(4):
        band = slice(l * l, (l + 1) * (l + 1))
        lhs = (Ya[:, band] * Yb[:, band]).sum(1)
        c = np.zeros(l + 1)
        c[l] = 1.0
        rhs = (2 * l + 1) / (4.0 * np.pi) * legendre.legval(cos, c)
        np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_low_bands_match_their_definition():
    """l = 0 is the constant 1 / (2 sqrt(pi)); l = 1 is sqrt(3 / (4 pi)) times
    (y, z, x), the real forms without the Condon-Shortley sign."""
    d = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0], [0.48, 0.6, 0.64]])
    Y = sh.basis(d, 1)
    np.testing.assert_allclose(Y[:, 0], 0.28209479177387814, rtol=1e-15)
    np.testing.assert_allclose(Y[:, 1:], 0.4886025119029199 * d[:, [1, 2, 0]], rtol=1e-15)


def test_basis_grad_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = rng.uniform(-1.2, 1.2, (50, 3))     # the polynomial forms, off the sphere too
    G = sh.basis_grad(p, 3)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (sh.basis(p + e, 3) - sh.basis(p - e, 3)) / (2 * h)
        np.testing.assert_allclose(G[..., a], fd, atol=1e-8)


def _scene(seed, n=20, degree=3):
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, n, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    K = sh.n_coef(degree)
    coef = rng.standard_normal((n, K, 3)).astype(np.float32) * 0.3
    coef[:, 0, :] = (sc["color"] / 0.28209479177387814).astype(np.float32)
    sc["color"] = coef
    return sc


def test_dc_only_sh_renders_like_rgb():
    """Coefficients with only the band-0 term give c = Y_00 SH_0: the SH render
    equals the RGB render of those colours, and dL/dSH_0 = Y_00 dL/dc."""
    cam = small_cam(40, 30, 40.0)
    rng = np.random.default_rng(2)
    sc = random_scene(rng, 25, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    coef = np.zeros((25, 4, 3))
    coef[:, 0, :] = sc["color"].astype(np.float64) / 0.28209479177387814
    sc_sh = dict(sc)
    sc_sh["color"] = coef
    P = orc.make_params(cam)
    poses = identity_pose()
    recs = orc.project(P, sc, poses)
    pix = all_pixels(1, 30, 40)
    ref = orc.render(P, recs, sc, pix)
    got = sh.render(P, recs, sc_sh, poses, pix, 1)
    np.testing.assert_allclose(got["color"], ref["color"], rtol=1e-12, atol=1e-15)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    gr = orc.backward(P, recs, sc, poses, pix, gC, gD)
    gs = sh.backward(P, recs, sc_sh, poses, pix, gC, gD, 1)
    np.testing.assert_allclose(gs["color"][:, 0, :], 0.28209479177387814 * gr["color"], rtol=1e-12, atol=1e-15)
    for k in ("pos", "scale", "rot", "opacity"):
        np.testing.assert_allclose(gs[k], gr[k], rtol=1e-12, atol=1e-15)


def _loss(P, sc, poses, pix, gC, gD, degree):
    recs = orc.project(P, sc, poses)
    out = sh.render(P, recs, sc, poses, pix, degree)
    return float((out["color"] * gC).sum() + (out["depth"] * gD).sum()), out["sig"]


@pytest.mark.parametrize("degree", [1, 3])
def test_sh_backward_matches_finite_differences(degree):
    """Central differences of the SH render (two frames with different view
    directions) against the SH backward, on SH coefficients of every band and
    on positions (which move both the footprint and the view direction);
    perturbations that flip a discrete decision are skipped."""
    cam = small_cam(40, 30, 40.0)
    rng = np.random.default_rng(3 + degree)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    pose_b = look_at(tg + 0.3 * Rg[:, 0], target, up=-Rg[:, 1])
    poses = np.stack([pose_a, pose_b])
    sc = random_scene(rng, 20, centre=target, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    K = sh.n_coef(degree)
    coef = (rng.standard_normal((20, K, 3)) * 0.3).astype(np.float32)
    sc["color"] = coef
    P = orc.make_params(cam)
    pix = all_pixels(2, 30, 40)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    recs = orc.project(P, sc, poses)
    grads = sh.backward(P, recs, sc, poses, pix, gC, gD, degree)
    checked = {"color": 0, "pos": 0}
    scale = {k: np.abs(grads[k]).max() for k in checked}
    for name in checked:
        idx = [i for i in range(20) if sc["unstable"][i]]
        rng.shuffle(idx)
        for i in idx:
            if checked[name] >= 12:
                break
            if name == "color":
                j = (int(rng.integers(K)), int(rng.integers(3)))
            else:
                j = (int(rng.integers(3)),)
            p = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in sc.items()}
            x0 = p[name][(i,) + j]
            h = 1e-5 * max(1.0, abs(x0))
            vals = []
            for sgn in (+1, -1):
                q = {k: v.copy() for k, v in p.items()}
                q[name][(i,) + j] = x0 + sgn * h
                q32 = {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in q.items()}
                vals.append((_loss(P, q32, poses, pix, gC, gD, degree), float(q32[name][(i,) + j])))
            if not np.array_equal(vals[0][0][1], vals[1][0][1]):
                continue
            fd = (vals[0][0][0] - vals[1][0][0]) / (vals[0][1] - vals[1][1])
            an = grads[name][(i,) + j]
            assert abs(fd - an) <= 2e-6 * (abs(an) + 1e-2 * scale[name] + 1e-12), (name, i, j, fd, an)
            checked[name] += 1
    assert min(checked.values()) >= 8, checked


def test_sh_bound_covers_a_binary32_recomputation():
    """The error bound of the SH backward covers the difference between the
    binary64 gradients and the same chain with every colour rounded to
    binary32 and every SH product formed in binary32."""
    cam = small_cam(40, 30, 40.0)
    sc = _scene(7, degree=2)
    rng = np.random.default_rng(8)
    poses = identity_pose()
    P = orc.make_params(cam)
    recs = orc.project(P, sc, poses)
    pix = all_pixels(1, 30, 40)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    g, b = sh.backward(P, recs, sc, poses, pix, gC, gD, 2, bound=(64 * 2.0 ** -24, 0.0, 256.0))
    d, r = sh.directions(sc["pos"], poses)
    Y32 = sh.basis(d, 2).astype(np.float32)
    gcol = orc.backward(P, recs, dict(sc, color64=sh.colors(sc["color"], sc["pos"], poses, 2)[0]), poses, pix,
                        gC, gD)["color"].astype(np.float32)
    approx = (Y32[0][:, :, None] * gcol[:, None, :]).astype(np.float64)
    un = sc["unstable"] != 0
    assert (np.abs(approx - g["color"])[un] <= b["color"][un] + 1e-30).all()
