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


def _patches_in_view(rng, pos, tree, pose, cam, frac, n_patch=6):
    """Indices of Gaussians in n_patch world-space spherical patches centred
    on near-surface points seen by this camera, sized so the patches cover
    roughly frac of the image."""
    u, v, z = _project_centres(pos, pose, cam)
    W, H = cam["width"], cam["height"]
    inview = np.nonzero((z > 0.5) & (u > 0.1 * W) & (u < 0.9 * W) & (v > 0.1 * H) & (v < 0.9 * H))[0]
    if inview.size == 0:
        return np.zeros(0, np.int64)
    sel = []
    for _ in range(n_patch):
        # nearest surface along a random in-view direction: smallest depth
        # among the in-view Gaussians projecting close to a random pixel
        px, py = rng.uniform(0.15 * W, 0.85 * W), rng.uniform(0.15 * H, 0.85 * H)
        near = inview[(np.abs(u[inview] - px) < 6) & (np.abs(v[inview] - py) < 6)]
        if near.size == 0:
            continue
        c = near[np.argmin(z[near])]
        d = z[c]
        r = d / cam["fx"] * np.sqrt(frac * W * H / (n_patch * np.pi))
        sel.append(np.asarray(tree.query_ball_point(pos[c], r), np.int64))
    return np.unique(np.concatenate(sel)) if sel else np.zeros(0, np.int64)


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
        poses = _random_walk(rng, start, yaw0, F, X, Y)
        tree = cKDTree(pos)
        unstable = np.zeros(n, np.uint8)
        if name == "c3":
            # 20 % of the Gaussians in spatial patches: some in view of the
            # camera, the rest out of its view
            sel = _patches_in_view(rng, pos, tree, poses[0], cam, 0.3, n_patch=8)
            unstable[sel] = 1
            u, v, z = _project_centres(pos, poses[0], cam)
            away = np.nonzero(~((z > 0.0) & (u > -0.2 * cam["width"]) & (u < 1.2 * cam["width"]) &
                                (v > -0.2 * cam["height"]) & (v < 1.2 * cam["height"])))[0]
            while unstable.mean() < 0.2:
                c = away[rng.integers(len(away))]
                unstable[np.asarray(tree.query_ball_point(pos[c], 0.5), np.int64)] = 1
            meta["unstable_frac"] = float(unstable.mean())
        else:
            fracs = np.linspace(0.05, 0.60, F)
            rng.shuffle(fracs)
            for f in range(F):
                sel = _patches_in_view(rng, pos, tree, poses[f], cam, 0.6 * fracs[f])
                unstable[sel] = 1
            meta["target_mask_fracs"] = [float(x) for x in fracs]
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
