"""Seeded synthetic scenes in the shape of the RTG-SLAM mapping workload.

Everything here is input construction (geometry sampling, random poses,
masks, random upstream gradients).  The rasterizer's own arithmetic lives in
the HIP library and, independently, in the CPU oracle; neither is imported
here.

Conventions shared by both consumers:
* world frame z up; camera frame x right, y down, z forward (camera looks
  along +z); a pose is 12 float64 values: the camera-to-world rotation R_g
  row-major, then the camera centre t_g.
* Gaussian parameters (float32): pos (N,3) metres, scale (N,3) metres
  (activated), rot (N,4) raw quaternion (w,x,y,z), opacity (N,) in (0,1),
  color (N,3) RGB, unstable (N,) uint8.

Workloads (sizes of the paper's mapping setting; the real datasets are not
used -- these synthetic scenes stand in for them):
* c1: 2,000 Gaussians uniform in a 1 m cube 2 m ahead, 128x96, fx=fy=100.
* c2: 100k surface Gaussians on the 6 faces of a 5x5x3 m room plus 4
  boxes, 640x480, fx=fy=525, one frame, full mask, all unstable.
* c3: 500k surface Gaussians in a 10x8x3 m two-wall multi-room layout,
  1200x680, fx=fy=600, 20 % unstable in spatial patches, mask = pixels
  covered by unstable Gaussians.
* c4: 1M Gaussians, layout scaled to 14x11x3 m, 8 poses on a random walk,
  per-frame unstable patches sized for 5..60 % of the image.
* c5: 5M Gaussians over a 30x20x3 m floor (walls, boxes, cylinders),
  16 poses, per-frame unstable patches as c4.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

CONFIGS = ("c1", "c2", "c3", "c4", "c5")


def camera(width, height, fx, fy, cx=None, cy=None):
    return {"width": int(width), "height": int(height), "fx": float(fx), "fy": float(fy),
            "cx": float(width) / 2.0 if cx is None else float(cx),
            "cy": float(height) / 2.0 if cy is None else float(cy)}


def look_at(eye, target, up=(0.0, 0.0, 1.0)):
    """Pose (12 float64) of a camera at eye looking at target."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], axis=1)
    return np.concatenate([R.reshape(-1), eye])


def _opacity(rng, n):
    """70 % opaque U[0.95, 0.99], 30 % transparent U[0.02, 0.1]."""
    op = np.where(rng.random(n) < 0.7, rng.uniform(0.95, 0.99, n), rng.uniform(0.02, 0.1, n))
    return op.astype(np.float32)


def _log_uniform(rng, n, lo=0.01, hi=0.05):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def _quat_wxyz(R):
    q = Rotation.from_matrix(R).as_quat()  # x, y, z, w
    return np.concatenate([q[:, 3:4], q[:, :3]], axis=1)


def _cube_scene(rng, n):
    pos = rng.uniform(-0.5, 0.5, (n, 3)) + np.array([0.0, 0.0, 2.0])
    scale = np.stack([_log_uniform(rng, n) for _ in range(3)], axis=1)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return pos, scale, q


# --- surfaces -------------------------------------------------------------

def _rect(origin, u, v):
    return ("rect", np.asarray(origin, float), np.asarray(u, float), np.asarray(v, float))


def _box(x0, y0, x1, y1, h):
    """Top and four sides of an axis-aligned box standing on the floor."""
    return [
        _rect((x0, y0, h), (x1 - x0, 0, 0), (0, y1 - y0, 0)),
        _rect((x0, y0, 0), (x1 - x0, 0, 0), (0, 0, h)),
        _rect((x0, y1, 0), (x1 - x0, 0, 0), (0, 0, h)),
        _rect((x0, y0, 0), (0, y1 - y0, 0), (0, 0, h)),
        _rect((x1, y0, 0), (0, y1 - y0, 0), (0, 0, h)),
    ]


def _room_shell(X, Y, Z):
    return [
        _rect((0, 0, 0), (X, 0, 0), (0, Y, 0)),      # floor
        _rect((0, 0, Z), (0, Y, 0), (X, 0, 0)),      # ceiling
        _rect((0, 0, 0), (0, Y, 0), (0, 0, Z)),      # wall x = 0
        _rect((X, 0, 0), (0, Y, 0), (0, 0, Z)),      # wall x = X
        _rect((0, 0, 0), (X, 0, 0), (0, 0, Z)),      # wall y = 0
        _rect((0, Y, 0), (X, 0, 0), (0, 0, Z)),      # wall y = Y
    ]


def _wall_with_door(axis, c, a0, a1, door_at, Z, door_w=1.0, door_h=2.1):
    """Interior wall on plane axis=c spanning [a0, a1] along the other
    horizontal axis, with a door gap [door_at, door_at + door_w]."""
    def piece(b0, b1, z0, z1):
        if axis == "x":
            return _rect((c, b0, z0), (0, b1 - b0, 0), (0, 0, z1 - z0))
        return _rect((b0, c, z0), (b1 - b0, 0, 0), (0, 0, z1 - z0))
    return [piece(a0, door_at, 0, Z), piece(door_at + door_w, a1, 0, Z),
            piece(door_at, door_at + door_w, door_h, Z)]


def _cylinder(cx, cy, r, h):
    return ("cyl", np.array([cx, cy], float), float(r), float(h))


def _area(s):
    if s[0] == "rect":
        return float(np.linalg.norm(np.cross(s[2], s[3])))
    return 2.0 * np.pi * s[2] * s[3]


def _sample_surfaces(rng, surfaces, n):
    """Surface Gaussians: uniform by area, thin axis along the surface normal,
    random in-plane angle, scales (s, s, 0.1 s) with s log-uniform 1-5 cm."""
    areas = np.array([_area(s) for s in surfaces])
    counts = rng.multinomial(n, areas / areas.sum())
    P, T1, NRM = [], [], []
    for s, k in zip(surfaces, counts):
        if k == 0:
            continue
        if s[0] == "rect":
            _, o, u, v = s
            a, b = rng.random(k), rng.random(k)
            P.append(o + a[:, None] * u + b[:, None] * v)
            nrm = np.cross(u, v)
            nrm /= np.linalg.norm(nrm)
            t1 = u / np.linalg.norm(u)
            NRM.append(np.repeat(nrm[None], k, 0))
            T1.append(np.repeat(t1[None], k, 0))
        else:
            _, c, r, h = s
            ph = rng.uniform(0, 2 * np.pi, k)
            z = rng.uniform(0, h, k)
            P.append(np.stack([c[0] + r * np.cos(ph), c[1] + r * np.sin(ph), z], 1))
            NRM.append(np.stack([np.cos(ph), np.sin(ph), np.zeros(k)], 1))
            T1.append(np.stack([-np.sin(ph), np.cos(ph), np.zeros(k)], 1))
    pos = np.concatenate(P)
    nrm = np.concatenate(NRM)
    t1 = np.concatenate(T1)
    t2 = np.cross(nrm, t1)
    th = rng.uniform(0, 2 * np.pi, n)[:, None]
    a1 = np.cos(th) * t1 + np.sin(th) * t2
    a2 = np.cross(nrm, a1)
    R = np.stack([a1, a2, nrm], axis=2)        # columns: axes of the Gaussian
    q = _quat_wxyz(R)
    s = _log_uniform(rng, n)
    scale = np.stack([s, s, 0.1 * s], axis=1)
    perm = rng.permutation(n)
    return pos[perm], scale[perm], q[perm]


def _random_boxes(rng, k, X, Y, margin=0.6):
    out = []
    for _ in range(k):
        w, d = rng.uniform(0.4, 1.2, 2)
        h = rng.uniform(0.4, 1.5)
        x0 = rng.uniform(margin, X - margin - w)
        y0 = rng.uniform(margin, Y - margin - d)
        out += _box(x0, y0, x0 + w, y0 + d, h)
    return out


def _layout(kind, rng):
    if kind == "room":
        X, Y, Z = 5.0, 5.0, 3.0
        return (X, Y, Z), _room_shell(X, Y, Z) + _random_boxes(rng, 4, X, Y)
    if kind in ("multi", "multi_l"):
        s = 1.0 if kind == "multi" else 1.4
        X, Y, Z = 10.0 * s, 8.0 * s, 3.0
        surf = _room_shell(X, Y, Z)
        surf += _wall_with_door("x", 0.4 * X, 0.0, Y, rng.uniform(0.5, Y / 2 - 1.5), Z)
        surf += _wall_with_door("y", 0.5 * Y, 0.4 * X, X, rng.uniform(0.4 * X + 0.5, X - 1.5), Z)
        surf += _random_boxes(rng, 6 if kind == "multi" else 10, X, Y)
        return (X, Y, Z), surf
    if kind == "floor":
        X, Y, Z = 30.0, 20.0, 3.0
        surf = _room_shell(X, Y, Z)
        for xw in (6.0, 12.0, 18.0, 24.0):
            surf += _wall_with_door("x", xw, 0.0, 10.0, rng.uniform(1.0, 8.0), Z)
        for yw in (10.0,):
            surf += _wall_with_door("y", yw, 0.0, X, rng.uniform(1.0, X - 2.0), Z)
        surf += _random_boxes(rng, 30, X, Y)
        for _ in range(10):
            surf.append(_cylinder(rng.uniform(1, X - 1), rng.uniform(11, Y - 1), rng.uniform(0.15, 0.4), Z))
        return (X, Y, Z), surf
    raise ValueError(kind)


def _random_walk(rng, start, yaw0, F, X, Y, step=(0.1, 0.3), dyaw=np.radians(30.0), margin=0.7):
    """F poses: each step moves <= 0.3 m and turns <= 30 degrees (the
    keyframe thresholds of the paper's global optimisation)."""
    eye = np.array(start, float)
    yaw = yaw0
    poses = []
    for k in range(F):
        if k > 0:
            for _ in range(100):
                ang = rng.uniform(0, 2 * np.pi)
                d = rng.uniform(*step)
                cand = eye + np.array([d * np.cos(ang), d * np.sin(ang), 0.0])
                if margin < cand[0] < X - margin and margin < cand[1] < Y - margin:
                    eye = cand
                    break
            yaw += rng.uniform(-dyaw, dyaw)
        pitch = rng.uniform(-np.radians(10), np.radians(10))
        fwd = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        poses.append(look_at(eye, eye + fwd))
    return np.stack(poses)


def _keyframe_batch(rng, start, yaw0, F, X, Y, margin=0.7, walk_factor=4):
    """A batch of F keyframes drawn from a keyframe list along a random
    walk.  The list follows the paper's keyframe rule: a new keyframe once
    the camera has turned more than 30 degrees or moved more than 0.3 m since
    the last one, so each step is either a turn of 30-40 degrees (with a move
    below 0.3 m) or a move of 0.3-0.4 m (with a turn below 30 degrees).  The
    batch is F keyframes of a list walk_factor * F long, drawn at random and
    kept in walk order, as the global optimisation draws random keyframes."""
    L = walk_factor * F
    eye = np.array(start, float)
    yaw = yaw0
    poses = []
    for k in range(L):
        if k > 0:
            turn = rng.random() < 0.5
            if turn:
                d = rng.uniform(0.0, 0.3)
                yaw += rng.choice([-1.0, 1.0]) * np.radians(rng.uniform(30.0, 40.0))
            else:
                d = rng.uniform(0.3, 0.4)
                yaw += np.radians(rng.uniform(-30.0, 30.0))
            for _ in range(100):
                ang = yaw + rng.uniform(-np.pi / 2, np.pi / 2)
                cand = eye + np.array([d * np.cos(ang), d * np.sin(ang), 0.0])
                if margin < cand[0] < X - margin and margin < cand[1] < Y - margin:
                    eye = cand
                    break
        pitch = rng.uniform(-np.radians(10), np.radians(10))
        fwd = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        poses.append(look_at(eye, eye + fwd))
    pick = np.sort(rng.choice(L, F, replace=False))
    return np.stack(poses)[pick]


def _project_centres(pos, pose, cam):
    """Pixel coordinates and depth of points (pinhole; used only to place
    unstable patches in view)."""
    R = pose[:9].reshape(3, 3)
    pc = (pos - pose[9:]) @ R
    z = pc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = cam["fx"] * pc[:, 0] / z + cam["cx"]
        v = cam["fy"] * pc[:, 1] / z + cam["cy"]
    return u, v, z


class _Coverage:
    """Approximate per-frame image coverage of groups of Gaussians, used
    only to place unstable patches: each Gaussian's footprint is taken as a
    disc of radius 3 s_max f / z pixels (an upper bound of its cut-off
    ellipse), evaluated on a grid of sample pixels every `step` pixels.  The
    realised masks are computed afterwards by the rasterizer (or the oracle)
    and reported; this estimate only steers the choice of patches."""

    def __init__(self, pos, scale, poses, cam, step=8, z_near=0.2):
        self.pos, self.smax = pos, scale.max(axis=1)
        self.poses, self.cam, self.step, self.z_near = poses, cam, step, z_near
        self.gw = (cam["width"] + step - 1) // step
        self.gh = (cam["height"] + step - 1) // step
        self._discs = {}

    def _disc(self, r):
        if r not in self._discs:
            o = np.arange(-r, r + 1)
            dx, dy = np.meshgrid(o, o)
            k = dx * dx + dy * dy <= r * r
            self._discs[r] = (dx[k], dy[k])
        return self._discs[r]

    def cover(self, idx, f):
        """Boolean sample grid (gh, gw) of frame f covered by Gaussians idx."""
        out = np.zeros(self.gh * self.gw, bool)
        if len(idx) == 0:
            return out.reshape(self.gh, self.gw)
        u, v, z = _project_centres(self.pos[idx], self.poses[f], self.cam)
        ok = z > self.z_near
        u, v, z, sm = u[ok], v[ok], z[ok], self.smax[idx][ok]
        st = self.step
        r = 3.0 * sm * self.cam["fx"] / z / st             # radius in grid cells
        gu, gv = (u - 0.5 * st) / st, (v - 0.5 * st) / st   # grid coordinates of the centres
        inb = (gu + r >= 0) & (gu - r <= self.gw - 1) & (gv + r >= 0) & (gv - r <= self.gh - 1)
        gu, gv, r = gu[inb], gv[inb], r[inb]
        ri = np.minimum(np.ceil(r).astype(np.int64), max(self.gw, self.gh))
        cu, cv = np.rint(gu).astype(np.int64), np.rint(gv).astype(np.int64)
        for rr in np.unique(ri):
            sel = ri == rr
            dx, dy = self._disc(int(rr))
            X = cu[sel, None] + dx[None]
            Y = cv[sel, None] + dy[None]
            # exact disc test against the unrounded centre and radius
            keep = ((X - gu[sel, None]) ** 2 + (Y - gv[sel, None]) ** 2 <= r[sel, None] ** 2) & \
                   (X >= 0) & (X < self.gw) & (Y >= 0) & (Y < self.gh)
            out[(Y[keep] * self.gw + X[keep])] = True
        return out.reshape(self.gh, self.gw)


def _place_unstable(rng, pos, scale, tree, poses, cam, targets, iters=None, per_iter=8, max_members=800,
                    radius=(0.1, 1.5), overshoot=2.0, tol=0.02, by_rank=False):
    """Unstable Gaussians as a union of world-space spherical patches chosen
    so that each frame's covered fraction approaches its target.

    Each round takes the frame furthest below its target (relative to the
    target), draws `per_iter` candidate balls around surface points that
    frame sees (the nearest Gaussian along a random pixel ray, radius
    log-uniform), and adds the candidate with the best score: the sum over
    frames of the newly covered samples up to each frame's remaining deficit,
    minus `overshoot` times those beyond it.  A frame whose best candidate
    does not score above zero is not drawn again.  With `by_rank`, the
    targets are a set of fractions rather than one per frame: before each
    round they are re-assigned to the frames in the order of the frames'
    current coverage (the most covered frame takes the largest target), since
    frames that see the same region cannot take very different fractions.
    Returns (indices, estimated per-frame fractions, targets as assigned)."""
    F = len(poses)
    targets = np.asarray(targets, np.float64)
    tsorted = np.sort(targets)
    iters = 4 * F + 8 if iters is None else iters
    cov = _Coverage(pos, scale, poses, cam, step=16)
    W, H = cam["width"], cam["height"]
    proj = [_project_centres(pos, poses[f], cam) for f in range(F)]
    # frustum test of a ball: its centre within the half-angles (plus the
    # angle the ball subtends) and in front of the near plane
    tx, ty = (0.5 * W) / cam["fx"], (0.5 * H) / cam["fy"]
    cx_, cy_ = 1.0 / np.sqrt(1 + tx * tx), 1.0 / np.sqrt(1 + ty * ty)

    def in_frustum(c, rad, f):
        R = poses[f][:9].reshape(3, 3)
        p = (c - poses[f][9:]) @ R
        # distance of the ball centre to the four side planes (inward normals)
        d = [(-p[0] + tx * p[2]) * cx_, (p[0] + tx * p[2]) * cx_, (-p[1] + ty * p[2]) * cy_,
             (p[1] + ty * p[2]) * cy_]
        return p[2] + rad > 0.2 and min(d) > -rad

    ncell = cov.gw * cov.gh
    cur = np.zeros((F, cov.gh * cov.gw), bool)
    deficit = targets * ncell
    stuck = np.zeros(F, bool)
    members = []
    for _ in range(iters):
        if by_rank:
            covered = cur.sum(1) + 1e-3 * np.arange(F)
            targets = np.empty(F)
            targets[np.argsort(covered, kind="stable")] = tsorted
            deficit = targets * ncell - cur.sum(1)
        rel = np.where(stuck, -np.inf, deficit / (targets * ncell))
        f = int(np.argmax(rel))
        if not rel[f] > tol / max(targets[f], 1e-9):
            break
        u, v, z = proj[f]
        best, best_score = None, 0.0
        for _ in range(per_iter):
            px, py = rng.uniform(0.0, W), rng.uniform(0.0, H)
            near = np.nonzero((z > 0.3) & (np.abs(u - px) < 8) & (np.abs(v - py) < 8))[0]
            if near.size == 0:
                continue
            c = near[np.argmin(z[near])]
            rad = float(np.exp(rng.uniform(np.log(radius[0]), np.log(radius[1]))))
            mem = np.asarray(tree.query_ball_point(pos[c], rad), np.int64)
            if mem.size == 0:
                continue
            sub = mem if mem.size <= max_members else rng.choice(mem, max_members, replace=False)
            grid = np.zeros((F, ncell), bool)
            for g in range(F):
                if in_frustum(pos[c], rad + 0.2, g):
                    grid[g] = cov.cover(sub, g).reshape(-1)
            new = (grid & ~cur).sum(1).astype(np.float64)
            gain = np.minimum(new, np.maximum(deficit, 0.0))
            score = float((gain - overshoot * (new - gain)).sum())
            if score > best_score:
                best, best_score = (mem, grid, new), score
        if best is None:
            stuck[f] = True
            continue
        mem, grid, new = best
        members.append(mem)
        deficit -= new
        cur |= grid
    idx = np.unique(np.concatenate(members)) if members else np.zeros(0, np.int64)
    return idx, cur.mean(1), targets


def make_config(name, seed=None):
    """Seeded workload dict: scene, cam, poses (F,12), mask ('full' or
    'unstable'), and metadata."""
    idx = CONFIGS.index(name)
    seed = idx if seed is None else seed
    rng = np.random.default_rng(seed)
    meta = {"name": name, "seed": seed}
    if name == "c1":
        n = 2000
        pos, scale, rot = _cube_scene(rng, n)
        cam = camera(128, 96, 100.0, 100.0)
        poses = np.concatenate([np.eye(3).reshape(-1), np.zeros(3)])[None]
        unstable = np.ones(n, np.uint8)
        mask = "full"
    elif name == "c2":
        n = 100_000
        (X, Y, Z), surf = _layout("room", rng)
        pos, scale, rot = _sample_surfaces(rng, surf, n)
        cam = camera(640, 480, 525.0, 525.0)
        eye = np.array([rng.uniform(2.0, 3.0), rng.uniform(1.0, 1.5), 1.5])
        yaw = np.radians(90.0 + rng.uniform(-20, 20))
        pitch = np.radians(rng.uniform(-10, 10))
        fwd = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        poses = look_at(eye, eye + fwd)[None]
        unstable = np.ones(n, np.uint8)
        mask = "full"
    else:
        kind, n, F = {"c3": ("multi", 500_000, 1), "c4": ("multi_l", 1_000_000, 8),
                      "c5": ("floor", 5_000_000, 16)}[name]
        (X, Y, Z), surf = _layout(kind, rng)
        pos, scale, rot = _sample_surfaces(rng, surf, n)
        cam = camera(1200, 680, 600.0, 600.0)
        start = np.array([rng.uniform(1.0, 0.4 * X - 1.0), rng.uniform(1.0, 0.5 * Y - 1.0), 1.5])
        yaw0 = rng.uniform(0, 2 * np.pi)
        if name == "c3":
            # a single view into the layout, not at a wall in front of the
            # camera: the heading (of 24) with the deepest median view depth
            sub = pos[rng.choice(len(pos), min(len(pos), 50_000), replace=False)]
            best = -1.0
            for yaw in yaw0 + np.arange(24) * (2 * np.pi / 24):
                fwd = np.array([np.cos(yaw), np.sin(yaw), 0.0])
                u, v, z = _project_centres(sub, look_at(start, start + fwd), cam)
                seen = (z > 0.2) & (u >= 0) & (u < cam["width"]) & (v >= 0) & (v < cam["height"])
                score = float(np.median(z[seen])) if seen.sum() > 100 else 0.0
                if score > best:
                    best, yaw_best = score, yaw
            yaw0 = yaw_best
        if name == "c3":
            poses = _random_walk(rng, start, yaw0, F, X, Y)
        else:
            poses = _keyframe_batch(rng, start, yaw0, F, X, Y)
        tree = cKDTree(pos)
        unstable = np.zeros(n, np.uint8)
        if name == "c3":
            # 20 % of the Gaussians in spatial patches: those in view of the
            # camera chosen to cover about a quarter of the image, the rest
            # out of its view (footprint included)
            sel, est, _ = _place_unstable(rng, pos, scale, tree, poses, cam, [0.25])
            unstable[sel] = 1
            u, v, z = _project_centres(pos, poses[0], cam)
            marg = 3.0 * scale.max(axis=1) * cam["fx"] / np.maximum(z, 1e-6)
            seen = (z > 0.0) & (u + marg > 0) & (u - marg < cam["width"]) & (v + marg > 0) & \
                (v - marg < cam["height"])
            away = np.nonzero(~seen)[0]
            while unstable.mean() < 0.2:
                c = away[rng.integers(len(away))]
                ball = np.asarray(tree.query_ball_point(pos[c], 0.5), np.int64)
                unstable[ball[~seen[ball]]] = 1
            meta["unstable_frac"] = float(unstable.mean())
            meta["target_mask_fracs"] = [0.25]
            meta["estimated_mask_fracs"] = [float(x) for x in est]
        else:
            # per-frame coverage spread over 5-60 % (evenly spaced targets,
            # assigned to the frames as the placement goes)
            sel, est, fracs = _place_unstable(rng, pos, scale, tree, poses, cam, np.linspace(0.05, 0.60, F),
                                              by_rank=True)
            unstable[sel] = 1
            meta["target_mask_fracs"] = [float(x) for x in fracs]
            meta["estimated_mask_fracs"] = [float(x) for x in est]
        mask = "unstable"
    scene = {"pos": pos.astype(np.float32), "scale": scale.astype(np.float32),
             "rot": rot.astype(np.float32), "opacity": _opacity(rng, n),
             "color": rng.random((n, 3)).astype(np.float32), "unstable": unstable}
    return {"scene": scene, "cam": cam, "poses": np.asarray(poses, np.float64), "mask": mask,
            "meta": meta}


def jitter_means(scene, sigma=0.01, seed=1000):
    """Copy of scene with positions jittered by N(0, sigma) (targets of the
    single-frame fwd+bwd workload are a render of such a copy)."""
    rng = np.random.default_rng(seed)
    out = dict(scene)
    out["pos"] = (scene["pos"] + rng.normal(0.0, sigma, scene["pos"].shape)).astype(np.float32)
    return out


def random_upstream(mask, seed=7, scale=1.0):
    """Seeded upstream gradients (gC (F,H,W,3), gD (F,H,W)), float32, zero
    outside the mask: the same arrays are fed to the oracle and the GPU."""
    rng = np.random.default_rng(seed)
    m = np.asarray(mask) != 0
    gC = (rng.standard_normal(m.shape + (3,)) * scale).astype(np.float32) * m[..., None]
    gD = (rng.standard_normal(m.shape) * scale).astype(np.float32) * m
    return gC.astype(np.float32), gD.astype(np.float32)
