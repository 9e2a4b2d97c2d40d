"""Plain reference of the steps around the render in the mapping loop:
Gaussian adding (Sec. 3.2 "Gaussians adding", Eq. 6) and state management
(Sec. 3.2 "Gaussian optimization", last paragraph, and "State management").

TEST INFRASTRUCTURE ONLY (the tests may import it; the product library
never does).  Float values in binary64 (numpy); every threshold decision is
taken in binary32 by the written sequence that the GPU kernels follow too,
so the discrete outputs (masks, which pixels add a Gaussian, in which order,
state changes, removals) can be compared exactly.

Readings (where the paper leaves the choice open):
  * pixel centre (x + 0.5, y + 0.5); input depth D <= 0 is invalid, and an
    invalid pixel is in neither adding mask (no vertex can be placed);
  * the colour error of a pixel is the L1 difference summed over the three
    channels compared with 3 delta_c (the mean-channel L1 error against
    delta_c), ec = (|dC0| + |dC1|) + |dC2| > fl32(3 delta_c);
  * no hit (rendered depth -1) counts as a depth error when D is valid;
  * "uniformly sample 5 %": a pixel of M_s or M_c is sampled when its
    uniform random number (an input, one per pixel) is below the rate;
  * vertex V = D K^-1 (x + 0.5, y + 0.5, 1); normal from the vertex map by
    the cross product of the forward differences to the right and lower
    neighbours (none on the last row or column or with an invalid
    neighbour), turned to face the camera;
  * disc radius: the paper's nearest-neighbour formula (supplementary A) is
    not followed; the disc covers the sampled pixel's share of the image,
    r = sqrt(1 / (pi rate)) pixels at depth D, r_world = r D / f with
    f = (fx + fy) / 2; scales (r, r, 0.1 r), thin axis last, rotated so the
    thin axis is the normal; transparent discs capped at 0.01 m;
  * state: a stable Gaussian whose pixel (through the index map) has a
    colour or depth error gets its error count raised once per frame; a
    stable Gaussian with e > delta_e becomes unstable (e = 0, eta = 0,
    t = k); an unstable one with eta > delta_eta becomes stable; an unstable
    one with k - t > delta_t is removed; eta grows by one per optimisation
    step in which the Gaussian's colour gradient is non-zero.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def params(delta_T=0.5, delta_d=0.1, delta_c=0.1, rate=0.05, alpha_opaque=0.99, alpha_transparent=0.1,
           r_transparent=0.01, thickness=0.1, delta_eta=100, delta_e=5, delta_t=200, sh_degree=0):
    """Thresholds of Eq. 6 and the paper's adding constants (delta_T 0.5,
    delta_d 0.1, delta_c 0.1, 5 % sampling, opacities 0.99 / 0.1, 0.01 m,
    axis ratio 1:1:0.1, delta_eta 100 for Replica); delta_e and delta_t are
    not stated in the paper.  sh_degree > 0: new Gaussians carry SH
    coefficients, the band-0 one reproducing the pixel colour in every
    direction (c / Y_00) and the higher bands zero."""
    return dict(delta_T=delta_T, delta_d=delta_d, delta_c=delta_c, rate=rate, alpha_opaque=alpha_opaque,
                alpha_transparent=alpha_transparent, r_transparent=r_transparent, thickness=thickness,
                delta_eta=delta_eta, delta_e=delta_e, delta_t=delta_t, sh_degree=sh_degree)


def color_error(color_r, color_in):
    """Per-pixel L1 colour error (|dC0| + |dC1|) + |dC2| in binary32."""
    d = np.abs(np.asarray(color_r, F32) - np.asarray(color_in, F32))
    return (d[..., 0] + d[..., 1]) + d[..., 2]


def adding_masks(P, color_r, depth_r, trans_r, color_in, depth_in):
    """Eq. 6: M_s = {T > delta_T or |D_r - D| > delta_d}, M_c = {colour error
    > delta_c and not M_s}, on pixels with valid input depth.  Returns a
    uint8 image: 1 for M_s, 2 for M_c, 0 otherwise."""
    D = np.asarray(depth_in, F32)
    valid = D > F32(0)
    ms = valid & ((np.asarray(trans_r, F32) > F32(P["delta_T"])) |
                  (np.abs(np.asarray(depth_r, F32) - D) > F32(P["delta_d"])))
    mc = valid & ~ms & (color_error(color_r, color_in) > F32(3) * F32(P["delta_c"]))
    out = np.zeros(D.shape, np.uint8)
    out[ms] = 1
    out[mc] = 2
    return out


def vertex_map(cam, depth):
    """V(x, y) = D (x + 0.5 - cx) / fx, D (y + 0.5 - cy) / fy, D) in the
    camera frame (binary64)."""
    H, W = depth.shape
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    D = np.asarray(depth, np.float64)
    V = np.empty((H, W, 3))
    V[..., 0] = D * ((x[None, :] - cam["cx"]) / cam["fx"])
    V[..., 1] = D * ((y[:, None] - cam["cy"]) / cam["fy"])
    V[..., 2] = D
    return V


def normal_map(cam, depth):
    """Unit normals (camera frame) from the vertex map: the cross product of
    the differences to the right and lower neighbours, turned towards the
    camera; valid where the pixel and both neighbours have valid depth."""
    D = np.asarray(depth, F32)
    H, W = D.shape
    V = vertex_map(cam, depth)
    N = np.zeros((H, W, 3))
    ok = np.zeros((H, W), bool)
    a = V[:-1, 1:] - V[:-1, :-1]
    b = V[1:, :-1] - V[:-1, :-1]
    n = np.cross(a, b)
    ln = np.linalg.norm(n, axis=-1)
    good = (D[:-1, :-1] > 0) & (D[:-1, 1:] > 0) & (D[1:, :-1] > 0) & (ln > 0)
    n = n / np.where(ln > 0, ln, 1.0)[..., None]
    flip = (n * V[:-1, :-1]).sum(-1) > 0
    n[flip] *= -1.0
    N[:-1, :-1] = n
    ok[:-1, :-1] = good
    return N, ok


def quat_z_to(n):
    """Unit quaternion (w, x, y, z) of the shortest rotation taking e_z to the
    unit vector n (a half-turn about x when n = -e_z)."""
    n = np.asarray(n, np.float64)
    w = 1.0 + n[..., 2]
    q = np.stack([w, -n[..., 1], n[..., 0], np.zeros_like(w)], -1)
    small = w < 1e-12
    q[small] = [0.0, 1.0, 0.0, 0.0]
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def add_gaussians(cam, P, pose, color_in, depth_in, color_r, depth_r, trans_r, index_r, unstable, rand, frame_k,
                  n_cur, capacity):
    """Gaussians added for one frame (Sec. 3.2): the sampled pixels of M_s
    with a valid normal get an opaque disc; the sampled pixels of M_c whose
    depth-hit Gaussian (index map) is stable get a transparent one.  New
    rows follow the existing n_cur in raster order of their pixels, up to
    `capacity` rows in all.  Returns the mask image, the candidate pixels
    (y, x) in order, and the new rows (at most capacity - n_cur)."""
    code = adding_masks(P, color_r, depth_r, trans_r, color_in, depth_in)
    sampled = np.asarray(rand, F32) < F32(P["rate"])
    N, nok = normal_map(cam, depth_in)
    idx = np.asarray(index_r)
    un = np.asarray(unstable) != 0
    hit_stable = (idx >= 0) & ~un[np.clip(idx, 0, None)]
    opaque = (code == 1) & sampled & nok
    transp = (code == 2) & sampled & nok & hit_stable
    cand = opaque | transp
    ys, xs = np.nonzero(cand)                       # raster order
    n_new = int(min(len(ys), max(capacity - n_cur, 0)))
    ys, xs = ys[:n_new], xs[:n_new]
    Rg = np.asarray(pose, np.float64)[:9].reshape(3, 3)
    tg = np.asarray(pose, np.float64)[9:12]
    V = vertex_map(cam, depth_in)[ys, xs]
    pos = V @ Rg.T + tg
    nrm = N[ys, xs] @ Rg.T
    D = np.asarray(depth_in, np.float64)[ys, xs]
    f = 0.5 * (cam["fx"] + cam["fy"])
    r = np.sqrt(1.0 / (np.pi * P["rate"])) * D / f
    is_t = transp[ys, xs]
    r = np.where(is_t, np.minimum(r, P["r_transparent"]), r)
    scale = np.stack([r, r, P["thickness"] * r], -1)
    col = np.asarray(color_in, np.float64)[ys, xs]
    deg = int(P.get("sh_degree", 0))
    if deg:
        coef = np.zeros((n_new, (deg + 1) ** 2, 3))
        coef[:, 0, :] = col / (0.5 * np.sqrt(1.0 / np.pi))
        col = coef
    rows = {"pos": pos, "scale": scale, "rot": quat_z_to(nrm), "normal": nrm,
            "opacity": np.where(is_t, P["alpha_transparent"], P["alpha_opaque"]),
            "color": col, "tstamp": np.full(n_new, frame_k, np.int64),
            "transparent": is_t}
    cy, cx = np.nonzero(cand)
    return {"mask": code, "candidates": np.stack([cy, cx], 1), "n_added": n_new, "rows": rows}


def confidence_count(unstable, d_color, eta):
    """eta + 1 for unstable Gaussians whose colour gradient row is non-zero
    (the colour, the SH band 0, was updated)."""
    g = np.asarray(d_color).reshape(len(eta), -1)
    upd = (np.asarray(unstable) != 0) & np.any(g != 0, axis=1)
    return np.asarray(eta) + upd.astype(np.asarray(eta).dtype)


def state_update(P, color_r, depth_r, index_r, color_in, depth_in, unstable, eta, err, tstamp, frame_k):
    """State management of Sec. 3.2 after a frame's optimisation: error
    counts of the stable Gaussians that a pixel with a colour or depth error
    hits (once per frame), stable -> unstable when e > delta_e, unstable ->
    stable when eta > delta_eta, removal of unstable ones older than
    delta_t.  Returns (unstable, eta, err, tstamp, keep) as new arrays."""
    D = np.asarray(depth_in, F32)
    Dr = np.asarray(depth_r, F32)
    valid = D > F32(0)
    bad = valid & ((color_error(color_r, color_in) > F32(3) * F32(P["delta_c"])) |
                   ((Dr != F32(-1)) & (np.abs(Dr - D) > F32(P["delta_d"]))))
    idx = np.asarray(index_r)
    un = np.asarray(unstable).astype(np.uint8).copy()
    eta = np.asarray(eta).copy()
    err = np.asarray(err).copy()
    ts = np.asarray(tstamp).copy()
    flag = np.zeros(len(un), bool)
    sel = bad & (idx >= 0)
    j = idx[sel]
    flag[j[un[j] == 0]] = True
    err = err + flag.astype(err.dtype)
    was_unstable = un != 0
    to_unstable = ~was_unstable & (err > P["delta_e"])
    to_stable = was_unstable & (eta > P["delta_eta"])
    remove = was_unstable & ~to_stable & (frame_k - ts > P["delta_t"])
    un[to_unstable] = 1
    err[to_unstable] = 0
    eta[to_unstable] = 0
    ts[to_unstable] = frame_k
    un[to_stable] = 0
    keep = ~remove
    return un, eta, err, ts, keep


def compact(keep, *arrays):
    """Rows with keep set, in order (np boolean indexing)."""
    k = np.asarray(keep, bool)
    return tuple(np.asarray(a)[k] for a in arrays)
