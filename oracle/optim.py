"""Plain reference of the steps of the mapping iteration either side of the
backward (Sec. 3.2 "Gaussian optimization", Eq. 8-9, and "Keyframes and
global optimization"): the L2 regulariser of transparent Gaussians, the
confidence-weighted fusion of a window's result, and the selection of the
pixels with the largest colour errors of a keyframe.

TEST INFRASTRUCTURE ONLY (the tests may import it; the product library
never does).  The fusion and the selection follow fixed binary32
sequences, so their outputs can be compared bit for bit; the regulariser is
binary64.

Readings (where the paper leaves the choice open):
  * L_reg = sum over transparent Gaussians of |p - p0|^2 + |q - q0|^2 +
    |s - s0|^2 (raw quaternion q, activated scale s; p0, q0, s0 the values
    the Gaussian was added with), weighted by w_reg = 1000 in the loss of
    Eq. 8; its gradient 2 w_reg (x - x0) is added to the gradient rows of
    unstable transparent Gaussians (stable rows are not optimised);
  * fusion (Eq. 9) of every Gaussian property that the optimisation updates
    (position, raw quaternion, scale, colour or SH coefficients; the
    opacity is fixed): w = (eta' - eta_prev) / eta' as a binary32 division
    of the two counts (w = 1 when eta' = 0), then
    G = fl32(fl32((1 - w) G_prev) + fl32(w G')) per value; eta keeps eta';
  * "the pixels with the top 40 % colour errors" of a keyframe: with the
    colour error e = (|dC0| + |dC1|) + |dC2| in binary32 (as in Eq. 6) over
    all H W pixels and k = floor(0.4 H W) (binary64 product), the pixels
    whose error is at least the k-th largest error (ties at that value are
    all selected; none when k = 0).
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def reg_l2(w_reg, transparent, unstable, cur, init):
    """L_reg of the transparent Gaussians and its gradients: cur / init are
    dicts of (N, w) arrays for "pos", "rot", "scale".  Returns (w_reg L_reg,
    {name: gradient (N, w)}) with gradient rows only for unstable
    transparent Gaussians (zero elsewhere)."""
    tr = np.asarray(transparent) != 0
    un = np.asarray(unstable) != 0
    loss = 0.0
    grads = {}
    for k in ("pos", "rot", "scale"):
        d = np.asarray(cur[k], np.float64) - np.asarray(init[k], np.float64)
        loss += float((d[tr] ** 2).sum())
        grads[k] = np.where((tr & un)[:, None], 2.0 * w_reg * d, 0.0)
    return w_reg * loss, grads


def fuse(eta_prev, eta_cur, prev, cur):
    """Eq. 9 per Gaussian, in binary32: returns {name: fused (N, ...)} for the
    arrays of `cur` (the window's optimised values G'), with `prev` the
    values before the window (G_{o-1})."""
    ep = np.asarray(eta_prev, np.int64)
    ec = np.asarray(eta_cur, np.int64)
    num = (ec - ep).astype(F32)
    den = ec.astype(F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(ec != 0, num / np.where(ec != 0, den, F32(1)), F32(1)).astype(F32)
    out = {}
    for k, g1 in cur.items():
        g1 = np.asarray(g1, F32)
        g0 = np.asarray(prev[k], F32)
        ww = w.reshape((-1,) + (1,) * (g1.ndim - 1))
        out[k] = ((F32(1) - ww) * g0).astype(F32) + (ww * g1).astype(F32)
    return out


def color_error(color_r, color_in):
    d = np.abs(np.asarray(color_r, F32) - np.asarray(color_in, F32))
    return (d[..., 0] + d[..., 1]) + d[..., 2]


def select_top_error(color_r, color_in, frac):
    """uint8 mask [F][H][W] of the pixels of each frame whose colour error is
    at least the k-th largest, k = floor(frac H W)."""
    e = color_error(color_r, color_in)
    F, H, W = e.shape
    k = int(np.floor(float(frac) * (H * W)))
    out = np.zeros((F, H, W), np.uint8)
    if k <= 0:
        return out
    for f in range(F):
        t = np.sort(e[f].ravel())[::-1][k - 1]
        out[f] = e[f] >= t
    return out
