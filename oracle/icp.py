"""Plain reference of the frame-to-model tracking of Sec. 3.2 ("Camera
tracking", Eq. 10) on the rasterizer's outputs: the rendered normal map N
(Sec. 3.1: the hit Gaussian's normal per pixel), and a multi-level
point-to-plane ICP of an input depth frame against the rendered depth and
normal maps of the model.

TEST INFRASTRUCTURE ONLY (the tests may import it; the product library
never does).  Binary64 numpy with every per-pixel value computed by the
same written operation sequence the GPU kernels use, so the data
association (which pixels take part) can be compared exactly for a given
pose.

Readings (the paper points to KinectFusion for the details):
  * normal map: the hit Gaussian's binary32 camera-frame normal n^c (the
    smallest-scale axis), turned to face the camera: flipped when
    n . ((x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1) > 0 (binary64); 0 on
    pixels without a hit;
  * pyramid: level l has floor(W / 2^l) x floor(H / 2^l) pixels and
    intrinsics fx / 2^l, fy / 2^l, cx / 2^l, cy / 2^l; a depth of level l+1
    is the binary32 mean of the valid (> 0) depths of its 2 x 2 block at
    level l, ((d00 + d01) + d10) + d11 over the valid ones divided by their
    count (0 when none); a model normal of level l+1 is the normal of the
    first pixel of its block, in raster order, with a valid depth;
  * vertex V(u) = D (x + 0.5 - cx) / fx, D (y + 0.5 - cy) / fy, D) and, for
    the input frame, normal from the cross product of the forward
    differences to the right and lower neighbours (needs all three valid),
    not normalised (only its direction is used);
  * association (projective, as KinectFusion): the input vertex p = R V + t
    under the current estimate T = (R, t) of the input frame's
    camera-to-world pose, into the model camera pm = R_m^T (p - t_m),
    pixel (floor(fx pm.x / pm.z + cx), floor(fy pm.y / pm.z + cy)) when
    pm.z > 0 and inside the level's image; the model vertex q = R_m V_m +
    t_m and normal n = R_m N_m there need a valid model depth and normal;
    a pair is kept when |p - q|^2 <= dist^2 and the input normal
    m = R N turned into the world has |m x n|^2 <= sin^2(angle) |m|^2 |n|^2;
  * residual r = (p - q) . n, Jacobian J = [p x n, n] for the
    left-multiplied update T <- exp(xi) T, xi = (omega, v); normal equations
    A = sum J^T J, b = sum J^T r, xi = -A^{-1} b (Cholesky, binary64; no
    update with fewer than 6 pairs or a non-positive pivot);
  * exp(xi): rotation by Rodrigues' formula, translation V(omega) v;
  * levels run coarse to fine, iters[l] iterations at level l.
"""
from __future__ import annotations

import numpy as np

F32 = np.float32


def normal_map(params, recs, out, pix, H, W):
    """[F][H][W][3] binary64 normals of the render out at the listed pixels
    (oracle.render's index map), oriented to face the camera; 0 elsewhere."""
    F = recs.shape[0]
    N = np.zeros((F, H, W, 3))
    idx = np.asarray(out["index"])
    for p in np.nonzero(idx >= 0)[0]:
        f, x, y = (int(v) for v in pix[p])
        n = recs["nc32"][f, idx[p]].astype(np.float64)
        rx = (x + 0.5 - params.cx) / params.fx
        ry = (y + 0.5 - params.cy) / params.fy
        s = (n[0] * rx + n[1] * ry) + n[2]
        N[f, y, x] = -n if s > 0 else n
    return N


def _down_depth(D):
    H, W = D.shape[0] // 2, D.shape[1] // 2
    out = np.zeros((H, W), F32)
    d = [D[0:2 * H:2, 0:2 * W:2], D[0:2 * H:2, 1:2 * W:2], D[1:2 * H:2, 0:2 * W:2], D[1:2 * H:2, 1:2 * W:2]]
    s = np.zeros((H, W), F32)
    c = np.zeros((H, W), F32)
    for q in d:
        v = q > 0
        s = (s + np.where(v, q, F32(0))).astype(F32)
        c = c + v
    ok = c > 0
    out[ok] = (s[ok] / c[ok].astype(F32)).astype(F32)
    return out


def _down_normal(Dm, Nm):
    H, W = Dm.shape[0] // 2, Dm.shape[1] // 2
    out = np.zeros((H, W, 3))
    got = np.zeros((H, W), bool)
    for dy in (0, 1):
        for dx in (0, 1):
            d = Dm[dy:2 * H:2, dx:2 * W:2][:H, :W]
            n = Nm[dy:2 * H:2, dx:2 * W:2][:H, :W]
            take = (d > 0) & ~got
            out[take] = n[take]
            got |= take
    return out


def pyramid(D, levels):
    P = [np.asarray(D, F32)]
    for _ in range(1, levels):
        P.append(_down_depth(P[-1]))
    return P


def vertex(D, fx, fy, cx, cy):
    H, W = D.shape
    x = np.arange(W) + 0.5
    y = np.arange(H) + 0.5
    Dd = D.astype(np.float64)
    V = np.zeros((H, W, 3))
    V[..., 0] = Dd * ((x[None, :] - cx) / fx)
    V[..., 1] = Dd * ((y[:, None] - cy) / fy)
    V[..., 2] = Dd
    return V


def input_normal(V, D):
    H, W = D.shape
    N = np.zeros((H, W, 3))
    ok = np.zeros((H, W), bool)
    a = V[:-1, 1:] - V[:-1, :-1]
    b = V[1:, :-1] - V[:-1, :-1]
    n = np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                  a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                  a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)
    ok[:-1, :-1] = (D[:-1, :-1] > 0) & (D[:-1, 1:] > 0) & (D[1:, :-1] > 0)
    N[:-1, :-1] = n
    return N, ok


def _rt(T):
    T = np.asarray(T, np.float64).reshape(12)
    return T[:9].reshape(3, 3), T[9:12]


def _mat_vec(R, v):
    """R v with the fixed order ((R0 v0 + R1 v1) + R2 v2) per row."""
    return np.stack([(R[i, 0] * v[..., 0] + R[i, 1] * v[..., 1]) + R[i, 2] * v[..., 2] for i in range(3)], -1)


def _matT_vec(R, v):
    return np.stack([(R[0, i] * v[..., 0] + R[1, i] * v[..., 1]) + R[2, i] * v[..., 2] for i in range(3)], -1)


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def associate(level_in, level_model, K, T, Tm, dist, sin_angle):
    """One level's pairs for the estimate T: returns (keep mask (H, W), p, q,
    n) with p, q, n the world points and model normal per input pixel."""
    D, V, Nn, okn = level_in
    Dm, Vm, Nm = level_model
    fx, fy, cx, cy = K
    R, t = _rt(T)
    Rm, tm = _rt(Tm)
    H, W = D.shape
    Hm, Wm = Dm.shape
    p = _mat_vec(R, V) + t
    pm = _matT_vec(Rm, p - tm)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.floor(fx * pm[..., 0] / pm[..., 2] + cx)
        v = np.floor(fy * pm[..., 1] / pm[..., 2] + cy)
    ok = (D > 0) & okn & (pm[..., 2] > 0) & (u >= 0) & (u < Wm) & (v >= 0) & (v < Hm)
    ui = np.where(ok, u, 0).astype(np.int64)
    vi = np.where(ok, v, 0).astype(np.int64)
    ok &= Dm[vi, ui] > 0
    nm = Nm[vi, ui]
    ok &= _dot(nm, nm) > 0
    q = _mat_vec(Rm, Vm[vi, ui]) + tm
    n = _mat_vec(Rm, nm)
    m = _mat_vec(R, Nn)
    d = p - q
    ok &= _dot(d, d) <= dist * dist
    cr = _cross(m, n)
    ok &= _dot(cr, cr) <= (sin_angle * sin_angle) * (_dot(m, m) * _dot(n, n))
    return ok, p, q, n


def normal_equations(ok, p, q, n):
    """A (6, 6), b (6,), sum r^2 and the pair count of the kept pairs."""
    r = _dot(p - q, n)[ok]
    J = np.concatenate([_cross(p, n), n], -1)[ok]
    return J.T @ J, J.T @ r, float((r * r).sum()), int(ok.sum())


def se3_exp(xi):
    w, v = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = np.sqrt(w @ w)
    Wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        R = np.eye(3) + Wx
        Vm = np.eye(3) + 0.5 * Wx
    else:
        a = np.sin(th) / th
        b = (1 - np.cos(th)) / (th * th)
        c = (th - np.sin(th)) / (th ** 3)
        R = np.eye(3) + a * Wx + b * (Wx @ Wx)
        Vm = np.eye(3) + b * Wx + c * (Wx @ Wx)
    return R, Vm @ v


def solve(A, b, count):
    if count < 6:
        return np.zeros(6)
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return np.zeros(6)
    return -np.linalg.solve(L.T, np.linalg.solve(L, b))


def update(T, xi):
    R, t = _rt(T)
    dR, dt = se3_exp(xi)
    return np.concatenate([(dR @ R).ravel(), dR @ t + dt])


def levels_of(cam, depth_in, depth_model, normal_model, levels):
    """Per level: input (D, V, N, normal-valid) and model (D, V, N) maps and
    intrinsics."""
    Din = pyramid(depth_in, levels)
    Dmo = pyramid(depth_model, levels)
    Nmo = [np.asarray(normal_model, np.float64)]
    for l in range(1, levels):
        Nmo.append(_down_normal(Dmo[l - 1], Nmo[-1]))
    out = []
    for l in range(levels):
        s = 2.0 ** l
        K = (cam["fx"] / s, cam["fy"] / s, cam["cx"] / s, cam["cy"] / s)
        V = vertex(Din[l], *K)
        Nn, okn = input_normal(V, Din[l])
        Vm = vertex(Dmo[l], *K)
        out.append(((Din[l], V, Nn, okn), (Dmo[l], Vm, Nmo[l]), K))
    return out


def icp(cam, depth_in, depth_model, normal_model, pose_model, pose_init, iters=(10, 5, 4), dist=0.1,
        sin_angle=np.sin(np.deg2rad(20.0))):
    """The refined camera-to-world pose of the input frame and the trace
    [(pose used, sum r^2, pairs), ...] of every iteration, coarse to fine."""
    L = len(iters)
    lv = levels_of(cam, depth_in, depth_model, normal_model, L)
    T = np.asarray(pose_init, np.float64).reshape(12)
    trace = []
    for l in reversed(range(L)):
        lin, lmo, K = lv[l]
        for _ in range(iters[l]):
            ok, p, q, n = associate(lin, lmo, K, T, pose_model, dist, sin_angle)
            A, b, err, cnt = normal_equations(ok, p, q, n)
            trace.append((T.copy(), err, cnt, A, b))
            T = update(T, solve(A, b, cnt))
    return T, trace
