"""Plain reference of view-dependent colour from spherical-harmonic (SH)
coefficients (Sec. 3.1: the colour c_i of Eq. 1 comes from the Gaussian's
SH coefficients and the view direction), and of its gradients.

TEST INFRASTRUCTURE ONLY (the tests may import it; the product library
never does).  Binary64 numpy; the render and the backward of the C oracle
(oracle.py) are reused frame by frame with that frame's colours.

Readings (the paper names SH coefficients, as in the splatting work it
builds on, but gives no degree, basis or formula):
  * degree D in 1..3 (D = 0 is the plain RGB colour of the hot path);
    K = (D + 1)^2 coefficients per channel, index k = l^2 + l + m for band l
    and order m in -l..l, stored [N][K][3];
  * basis: the orthonormal real spherical harmonics in their Cartesian form
    on the unit sphere, without the Condon-Shortley sign (real forms
    proportional to y, z, x for l = 1), i.e. the table below;
  * view direction of Gaussian i in frame f: the unit vector from the
    camera centre t_g to the Gaussian's centre, d = (p - t_g) / |p - t_g|;
  * c = sum_k SH_k Y_k(d) per channel: no offset and no clamp (the blend of
    Eq. 1 is linear in c, so negative values pass through and the colour is
    differentiable everywhere);
  * the colours are passed to the render oracle in binary64.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc

# normalisation constants of the real SH, from their closed forms
_C0 = 0.5 * np.sqrt(1.0 / np.pi)
_C1 = np.sqrt(3.0 / (4.0 * np.pi))
_C2A = 0.5 * np.sqrt(15.0 / np.pi)
_C2B = 0.25 * np.sqrt(5.0 / np.pi)
_C2C = 0.25 * np.sqrt(15.0 / np.pi)
_C3A = 0.25 * np.sqrt(35.0 / (2.0 * np.pi))
_C3B = 0.5 * np.sqrt(105.0 / np.pi)
_C3C = 0.25 * np.sqrt(21.0 / (2.0 * np.pi))
_C3D = 0.25 * np.sqrt(7.0 / np.pi)
_C3E = 0.25 * np.sqrt(105.0 / np.pi)


def n_coef(degree):
    return (int(degree) + 1) ** 2


def basis(d, degree):
    """Y_k(d) for k < (degree + 1)^2 of unit vectors d (..., 3): (..., K)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    one = np.ones_like(x)
    Y = [_C0 * one]
    if degree >= 1:
        Y += [_C1 * y, _C1 * z, _C1 * x]
    if degree >= 2:
        Y += [_C2A * x * y, _C2A * y * z, _C2B * (3.0 * z * z - 1.0), _C2A * x * z, _C2C * (x * x - y * y)]
    if degree >= 3:
        Y += [_C3A * y * (3.0 * x * x - y * y), _C3B * x * y * z, _C3C * y * (5.0 * z * z - 1.0),
              _C3D * z * (5.0 * z * z - 3.0), _C3C * x * (5.0 * z * z - 1.0), _C3E * z * (x * x - y * y),
              _C3A * x * (x * x - 3.0 * y * y)]
    return np.stack(Y, axis=-1)


def basis_grad(d, degree):
    """Gradient of the polynomial forms of basis() with respect to (x, y, z):
    (..., K, 3).  Only its part tangent to the sphere is used."""
    d = np.asarray(d, np.float64)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    G = [(zero, zero, zero)]
    if degree >= 1:
        G += [(zero, _C1 + zero, zero), (zero, zero, _C1 + zero), (_C1 + zero, zero, zero)]
    if degree >= 2:
        G += [(_C2A * y, _C2A * x, zero), (zero, _C2A * z, _C2A * y), (zero, zero, 6.0 * _C2B * z),
              (_C2A * z, zero, _C2A * x), (2.0 * _C2C * x, -2.0 * _C2C * y, zero)]
    if degree >= 3:
        G += [(6.0 * _C3A * x * y, _C3A * (3.0 * x * x - 3.0 * y * y), zero),
              (_C3B * y * z, _C3B * x * z, _C3B * x * y),
              (zero, _C3C * (5.0 * z * z - 1.0), 10.0 * _C3C * y * z),
              (zero, zero, _C3D * (15.0 * z * z - 3.0)),
              (_C3C * (5.0 * z * z - 1.0), zero, 10.0 * _C3C * x * z),
              (2.0 * _C3E * x * z, -2.0 * _C3E * y * z, _C3E * (x * x - y * y)),
              (_C3A * (3.0 * x * x - 3.0 * y * y), -6.0 * _C3A * x * y, zero)]
    return np.stack([np.stack(g, axis=-1) for g in G], axis=-2)


def directions(pos, poses):
    """Unit view directions (F, N, 3) and distances (F, N) from each frame's
    camera centre (pose rows: rotation, then centre) to each Gaussian."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    poses = np.asarray(poses, np.float64).reshape(-1, 12)
    v = pos[None, :, :] - poses[:, None, 9:12]
    r = np.sqrt((v * v).sum(-1))
    return v / r[..., None], r


def colors(coef, pos, poses, degree):
    """(F, N, 3) colours c = sum_k SH_k Y_k(d) of coefficients (N, K, 3)."""
    K = n_coef(degree)
    coef = np.asarray(coef, np.float64).reshape(-1, K, 3)
    d, _ = directions(pos, poses)
    return np.einsum("fnk,nkc->fnc", basis(d, degree), coef)


def _frame_scene(scene, col):
    s = dict(scene)
    s["color64"] = np.asarray(col, np.float64)
    return s


def render(params, recs, scene, poses, pix, degree, absolute=False):
    """The C oracle's render (oracle.render) with each frame's SH colours;
    scene["color"] holds the coefficients (N, K, 3).  With absolute=True the
    colours are replaced by their magnitudes |c|: the rendered "colour" is
    then sum |c_i| f_i T_i, the magnitude of the terms a binary32 blend adds
    up (SH colours can be negative, so the blend can cancel)."""
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    col = colors(scene["color"], scene["pos"], poses, degree)
    if absolute:
        col = np.abs(col)
    out = None
    for f in np.unique(pix[:, 0]):
        sel = np.nonzero(pix[:, 0] == f)[0]
        r = orc.render(params, recs, _frame_scene(scene, col[f]), pix[sel])
        if out is None:
            out = {k: np.zeros((len(pix),) + v.shape[1:], v.dtype) for k, v in r.items()}
        for k, v in r.items():
            out[k][sel] = v
    if out is None:
        out = orc.render(params, recs, _frame_scene(scene, np.zeros((len(scene["pos"]), 3))), pix)
    return out


def backward(params, recs, scene, poses, pix, gC, gD, degree, bound=None):
    """Parameter gradients of sum(gC . C) + sum(gD . D) with SH colours
    (rows of stable Gaussians zero): the C oracle's backward frame by frame
    with that frame's colours gives the geometric gradients (summed) and
    dL/dc per frame; then dL/dSH_k = sum_f dL/dc_f Y_k(d_f) and the view
    direction adds dL/dp = sum_f (I - d d^T) / |p - t_g| sum_k
    (dL/dc_f . SH_k) grad Y_k(d_f).  With bound=(gamma, t_eps, kappa_thr),
    also returns per-entry error bounds of a binary32 evaluation: the C
    oracle's per frame, carried through the SH sums, plus gamma times the
    sums of absolute terms."""
    K = n_coef(degree)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    gC = np.asarray(gC, np.float64).reshape(-1, 3)
    gD = np.asarray(gD, np.float64).reshape(-1)
    coef = np.asarray(scene["color"], np.float64).reshape(-1, K, 3)
    N = coef.shape[0]
    col = colors(coef, scene["pos"], poses, degree)
    d, r = directions(scene["pos"], poses)
    Y, dY = basis(d, degree), basis_grad(d, degree)
    un = np.asarray(scene["unstable"]).reshape(N) != 0
    tot = {"pos": np.zeros((N, 3)), "scale": np.zeros((N, 3)), "rot": np.zeros((N, 4)),
           "opacity": np.zeros(N), "color": np.zeros((N, K, 3))}
    bnd = {k: np.zeros_like(v) for k, v in tot.items()} if bound is not None else None
    for f in np.unique(pix[:, 0]):
        sel = np.nonzero(pix[:, 0] == f)[0]
        sc_f = _frame_scene(scene, col[f])
        if bound is None:
            g = orc.backward(params, recs, sc_f, poses, pix[sel], gC[sel], gD[sel])
        else:
            g, b = orc.backward(params, recs, sc_f, poses, pix[sel], gC[sel], gD[sel], bound=bound)
        for k in ("pos", "scale", "rot", "opacity"):
            tot[k] += g[k]
        gc = g["color"]                                   # dL/dc_f (N, 3)
        tot["color"] += Y[f][:, :, None] * gc[:, None, :]
        # dL/dd (N, 3) = sum_k (gc . SH_k) grad Y_k, then the tangent part / |v|
        s = np.einsum("nc,nkc->nk", gc, coef)
        u = np.einsum("nk,nka->na", s, dY[f])
        dp = (u - d[f] * (d[f] * u).sum(-1, keepdims=True)) / r[f][:, None]
        tot["pos"] += np.where(un[:, None], dp, 0.0)
        if bound is not None:
            gam = float(bound[0])
            for k in ("pos", "scale", "rot", "opacity"):
                bnd[k] += b[k]
            bc = b["color"]
            aY = np.abs(Y[f])
            bnd["color"] += aY[:, :, None] * bc[:, None, :] + gam * aY[:, :, None] * np.abs(gc)[:, None, :]
            sa = np.einsum("nc,nkc->nk", bc + gam * np.abs(gc), np.abs(coef))
            ua = np.einsum("nk,nka->na", sa + gam * np.abs(s), np.abs(dY[f]))
            bp = (ua + np.abs(d[f]) * (np.abs(d[f]) * ua).sum(-1, keepdims=True)) / r[f][:, None]
            bnd["pos"] += np.where(un[:, None], bp + gam * np.abs(dp), 0.0)
    tot["color"] = np.where(un[:, None, None], tot["color"], 0.0)
    if bound is None:
        return tot
    return tot, bnd
