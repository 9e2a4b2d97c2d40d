"""Hand-built tiny scenes for closed-form and invariant checks."""
import numpy as np

from rtg_synth import camera


def identity_pose():
    return np.concatenate([np.eye(3).reshape(-1), np.zeros(3)])[None]


def random_pose(rng, look_dist=2.0):
    """A random camera-to-world pose (rotation from a random unit quaternion)
    and the world point it looks at look_dist ahead."""
    from scipy.spatial.transform import Rotation
    R = Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
    t = rng.uniform(-1, 1, 3)
    return np.concatenate([R.reshape(-1), t]), R, t


def scene_from(pos, scale, rot, opacity, color, unstable=None):
    n = len(pos)
    return {"pos": np.asarray(pos, np.float32).reshape(n, 3),
            "scale": np.asarray(scale, np.float32).reshape(n, 3),
            "rot": np.asarray(rot, np.float32).reshape(n, 4),
            "opacity": np.asarray(opacity, np.float32).reshape(n),
            "color": np.asarray(color, np.float32).reshape(n, 3),
            "unstable": (np.ones(n, np.uint8) if unstable is None
                         else np.asarray(unstable, np.uint8).reshape(n))}


def small_cam(w=128, h=96, f=100.0):
    return camera(w, h, f, f)


def all_pixels(F, H, W):
    f, y, x = np.meshgrid(np.arange(F), np.arange(H), np.arange(W), indexing="ij")
    return np.stack([f.ravel(), x.ravel(), y.ravel()], 1).astype(np.int32)


def random_scene(rng, n, centre=(0.0, 0.0, 2.0), spread=0.5, smin=0.01, smax=0.08,
                 opaque_frac=0.7, unstable_frac=1.0):
    pos = rng.uniform(-spread, spread, (n, 3)) + np.asarray(centre)
    scale = np.exp(rng.uniform(np.log(smin), np.log(smax), (n, 3)))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q *= rng.uniform(0.5, 2.0, (n, 1))          # raw, non-unit quaternions
    op = np.where(rng.random(n) < opaque_frac, rng.uniform(0.95, 0.99, n), rng.uniform(0.02, 0.1, n))
    col = rng.random((n, 3))
    un = (rng.random(n) < unstable_frac).astype(np.uint8)
    return scene_from(pos, scale, q, op, col, un)


def _quat_of(R):
    """(w, x, y, z) of a proper rotation matrix (all four roots, signs from
    the skew part; exact enough for test scenes)."""
    w = np.sqrt(max(0.0, 1.0 + R[0, 0] + R[1, 1] + R[2, 2])) / 2
    x = np.copysign(np.sqrt(max(0.0, 1.0 + R[0, 0] - R[1, 1] - R[2, 2])) / 2, R[2, 1] - R[1, 2])
    y = np.copysign(np.sqrt(max(0.0, 1.0 - R[0, 0] + R[1, 1] - R[2, 2])) / 2, R[0, 2] - R[2, 0])
    z = np.copysign(np.sqrt(max(0.0, 1.0 - R[0, 0] - R[1, 1] + R[2, 2])) / 2, R[1, 0] - R[0, 1])
    return np.array([w, x, y, z])


def edge_on_surfels(rng, n, unstable_frac=1.0, thick_exp=(-7.0, -4.0), tilt_exp=(-5.0, -2.0)):
    """Surfels seen almost edge-on by the identity camera: centre 1.5-3 m
    ahead inside the view, in-plane scales 5-30 cm at any angle, thickness
    10^thick_exp m (default 1e-7..1e-4), normal perpendicular to the viewing
    ray up to a tilt of 10^tilt_exp rad (default 1e-5..1e-2; None: no
    tilt).  Their footprints are needles with condition numbers 1e2..1e10 by
    default, where binary32 rounding of the decision form matters."""
    pos = np.zeros((n, 3))
    rot = np.zeros((n, 4))
    scale = np.zeros((n, 3))
    for i in range(n):
        z = rng.uniform(1.5, 3.0)
        pos[i] = [rng.uniform(-0.5, 0.5) * z, rng.uniform(-0.4, 0.4) * z, z]
        ang = rng.uniform(0.0, np.pi)
        d = pos[i] / np.linalg.norm(pos[i])
        n0 = np.array([-np.sin(ang), np.cos(ang), 0.0])
        nn = n0 - d * (n0 @ d)
        nn /= np.linalg.norm(nn)
        tilt = 0.0 if tilt_exp is None else 10 ** rng.uniform(*tilt_exp)
        nt = np.cos(tilt) * nn + np.sin(tilt) * d
        e1 = np.array([np.cos(ang), np.sin(ang), 0.0])
        e1 = e1 - nt * (e1 @ nt)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nt, e1)
        rot[i] = _quat_of(np.stack([e1, e2, nt], axis=1))
        scale[i] = [rng.uniform(0.05, 0.3), rng.uniform(0.05, 0.3), 10 ** rng.uniform(*thick_exp)]
    op = rng.uniform(0.5, 0.99, n)
    col = rng.random((n, 3))
    un = (rng.random(n) < unstable_frac).astype(np.uint8)
    return scene_from(pos, scale, rot, op, col, un)


def footprint_condition(recs):
    """Condition number of every visible footprint (binary64 Sigma2D of the
    oracle's records), shape (F, N); inf where culled."""
    cov = recs["cov"]
    a, b, c = cov[..., 0], cov[..., 1], cov[..., 2]
    m, r = 0.5 * (a + c), np.sqrt(0.25 * (a - c) ** 2 + b * b)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = (m + r) / (m - r)
    return np.where(recs["visible"] != 0, k, np.inf)
