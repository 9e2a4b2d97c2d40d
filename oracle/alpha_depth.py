"""Plain reference of the alpha-blended depth used in the paper's ablation of
its depth rendering (supplementary, "Ablation study on depth rendering":
the opaque-disc depth of Eq. 4-5 replaced by alpha blending for the
optimisation, while adding and state management keep the disc depth).

TEST INFRASTRUCTURE ONLY (the tests may import it; the product library
never does).  Binary64; the C oracle (oracle.py) is reused frame by frame
with the Gaussians' camera depths in place of a colour channel.

Readings (the ablation names alpha blending, as in the splatting SLAM work
it compares with, but gives no formula):
  * D(u) = sum_i z_i f_i(u) prod_{j<i} (1 - f_j(u)): Eq. 1 with the colour
    replaced by z_i, the camera-frame depth of Gaussian i's centre, over the
    same list and blending as the colour (not normalised by the pixel's
    total opacity);
  * a pixel where no Gaussian blends (T = 1) has no depth (-1) and no depth
    loss, like a pixel without a hit in the disc mode;
  * the index map keeps the disc rule of Eq. 5 (adding and state
    management use it), so only the depth values and their gradients
    change.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc


def _depth_scene(scene, recs, f):
    s = dict(scene)
    z = np.where(recs["visible"][f] != 0, recs["pc"][f][:, 2], 0.0)
    c = np.zeros((len(z), 3))
    c[:, 0] = z
    s["color64"] = c
    return s


def render(params, recs, scene, pix):
    """The C oracle's render with the depth replaced by the alpha-blended
    depth (colour, transmission and the disc-rule index map unchanged)."""
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    out = orc.render(params, recs, scene, pix)
    out["depth"] = np.full(len(pix), -1.0)
    for f in np.unique(pix[:, 0]):
        sel = np.nonzero(pix[:, 0] == f)[0]
        r = orc.render(params, recs, _depth_scene(scene, recs, f), pix[sel])
        out["depth"][sel] = np.where(r["trans"] < 1.0, r["color"][:, 0], -1.0)
    return out


def backward(params, recs, scene, poses, pix, gC, gD, bound=None):
    """Parameter gradients of sum(gC . C) + sum(gD . D) with the
    alpha-blended depth (rows of stable Gaussians zero): the colour part is
    the C oracle's backward with no disc-depth upstream; the depth part is
    the C oracle's backward of a render whose first colour channel is z with
    upstream gD, whose colour gradient dL/dz then reaches the position
    through z = (R_g^T (p - t_g))_z, i.e. dz/dp = the third column of R_g.
    With bound=(gamma, t_eps, kappa_thr), also returns per-entry error bounds
    (the C oracle's bounds of both parts, the dL/dz one carried through
    |dz/dp|)."""
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    gC = np.asarray(gC, np.float64).reshape(-1, 3)
    gD = np.asarray(gD, np.float64).reshape(-1)
    poses = np.asarray(poses, np.float64).reshape(-1, 12)
    N = len(scene["pos"])
    zero = np.zeros(len(pix))
    if bound is None:
        tot = orc.backward(params, recs, scene, poses, pix, gC, zero)
    else:
        tot, bnd = orc.backward(params, recs, scene, poses, pix, gC, zero, bound=bound)
    tot = {k: v.copy() for k, v in tot.items()}
    un = np.asarray(scene["unstable"]).reshape(N) != 0
    for f in np.unique(pix[:, 0]):
        sel = np.nonzero(pix[:, 0] == f)[0]
        gz = np.zeros((len(sel), 3))
        gz[:, 0] = gD[sel]
        args = (params, recs, _depth_scene(scene, recs, f), poses, pix[sel], gz, np.zeros(len(sel)))
        if bound is None:
            g = orc.backward(*args)
        else:
            g, b = orc.backward(*args, bound=bound)
        col_z = poses[f, :9].reshape(3, 3)[:, 2]          # dz/dp
        for k in ("pos", "scale", "rot", "opacity"):
            tot[k] += g[k]
        tot["pos"] += np.where(un[:, None], g["color"][:, :1] * col_z[None, :], 0.0)
        if bound is not None:
            for k in ("pos", "scale", "rot", "opacity"):
                bnd[k] = bnd[k] + b[k]
            bnd["pos"] = bnd["pos"] + np.where(un[:, None], b["color"][:, :1] * np.abs(col_z)[None, :], 0.0)
    if bound is None:
        return tot
    return tot, bnd
