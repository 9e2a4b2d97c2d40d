"""Pins of the tracking oracle (oracle/icp.py): the SE(3) exponential against
the matrix exponential of the twist, the point-to-plane Jacobian against
finite differences of the residual, the pyramid and normal-map rules on
small cases, and recovery of a known camera motion from synthetic depth of
a room corner (three planes, so all six degrees of freedom are fixed)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import icp
from oracle import oracle as orc
from tests.scenes_small import identity_pose, scene_from, small_cam


def _hat(xi):
    w, v = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = v
    return M


@pytest.mark.parametrize("scale", [1e-14, 1e-6, 0.3, 2.0])
def test_se3_exp_matches_the_matrix_exponential(scale):
    rng = np.random.default_rng(int(-np.log10(scale)) + 5)
    xi = rng.standard_normal(6) * scale
    R, t = icp.se3_exp(xi)
    E = expm(_hat(xi))
    np.testing.assert_allclose(R, E[:3, :3], atol=1e-13)
    np.testing.assert_allclose(t, E[:3, 3], atol=1e-13)


def test_point_to_plane_jacobian_matches_finite_differences():
    rng = np.random.default_rng(1)
    p, q = rng.standard_normal(3), rng.standard_normal(3)
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    J = np.concatenate([np.cross(p, n), n])
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        rp = [(icp.se3_exp(s * e)[0] @ p + icp.se3_exp(s * e)[1] - q) @ n for s in (1, -1)]
        assert (rp[0] - rp[1]) / (2 * h) == pytest.approx(J[k], abs=1e-8)


def test_depth_pyramid_and_model_normal_rules():
    D = np.array([[1, 2, 0, 4], [3, 0, 0, 0], [5, 5, 5, 5], [5, 5, 5, 0]], np.float32)
    P = icp.pyramid(D, 2)
    assert np.array_equal(P[1], np.array([[2.0, 4.0], [5.0, 5.0]], np.float32))
    N = np.zeros((4, 4, 3))
    N[0, 0] = [1, 0, 0]
    N[0, 2] = [0, 1, 0]
    N[0, 3] = [0, 0, 1]
    N[2:, :] = [0, 0, -1]
    M = icp._down_normal(D, N)
    assert np.array_equal(M[0, 0], [1, 0, 0])          # first valid pixel of the block
    assert np.array_equal(M[0, 1], [0, 0, 1])          # (0, 2) has no depth: (0, 3)
    assert np.array_equal(M[1, 1], [0, 0, -1])


def test_normal_map_faces_the_camera():
    """A surfel seen frontally: its normal (the thin axis, +z or -z) comes out
    as (0, 0, -1) whichever sign the rotation gives it."""
    cam = small_cam(40, 30, 40.0)
    P = orc.make_params(cam)
    for q in ([1, 0, 0, 0], [0, 1, 0, 0]):            # thin axis +z, and turned by pi about x (-z)
        sc = scene_from([[0, 0, 2.0]], [[0.2, 0.2, 0.001]], [q], [0.9], [[1, 1, 1]])
        recs = orc.project(P, sc, identity_pose())
        pix = orc.masked_pixels(np.ones((1, 30, 40), np.uint8))
        out = orc.render(P, recs, sc, pix)
        N = icp.normal_map(P, recs, out, pix, 30, 40)
        hit = out["index"] >= 0
        assert hit.sum() > 30
        f, x, y = pix[hit, 0], pix[hit, 1], pix[hit, 2]
        np.testing.assert_allclose(N[f, y, x], np.tile([0, 0, -1.0], (hit.sum(), 1)), atol=1e-6)


def corner_maps(cam, pose):
    """Depth and camera-frame normal maps of a room corner (floor y = 1,
    walls x = -1.5 and z = 4, world frame) seen from camera-to-world pose
    `pose`: ray-plane intersections, the nearest positive one per pixel."""
    H, W = cam["height"], cam["width"]
    R, t = pose[:9].reshape(3, 3), pose[9:12]
    x = (np.arange(W) + 0.5 - cam["cx"]) / cam["fx"]
    y = (np.arange(H) + 0.5 - cam["cy"]) / cam["fy"]
    d_cam = np.stack(np.broadcast_arrays(x[None, :], y[:, None], np.ones((1, 1))), -1)   # (H, W, 3), z = 1
    d_w = d_cam @ R.T
    planes = [(np.array([0, 1.0, 0]), 1.0), (np.array([1.0, 0, 0]), -1.5), (np.array([0, 0, 1.0]), 4.0)]
    best = np.full((H, W), np.inf)
    nrm = np.zeros((H, W, 3))
    for n, c in planes:
        den = d_w @ n
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (c - t @ n) / den          # depth along the camera z (d_cam has z = 1)
        take = (s > 0) & (s < best)
        best[take] = s[take]
        nc = R.T @ n
        nrm[take] = nc
    D = np.where(np.isfinite(best), best, 0.0).astype(np.float32)
    # orient towards the camera
    flip = (nrm * d_cam).sum(-1) > 0
    nrm[flip] *= -1
    return D, nrm.astype(np.float32)


def test_icp_recovers_a_known_motion():
    cam = small_cam(160, 120, 140.0)
    pose_m = np.concatenate([np.eye(3).ravel(), [0.1, 0.2, 0.0]])
    # the true pose of the input frame: a small rotation and translation away
    xi_true = np.array([0.01, -0.008, 0.006, 0.015, -0.01, 0.012])
    R0, t0 = pose_m[:9].reshape(3, 3), pose_m[9:]
    dR, dt = icp.se3_exp(xi_true)
    pose_true = np.concatenate([(dR @ R0).ravel(), dR @ t0 + dt])
    Dm, Nm = corner_maps(cam, pose_m)
    Din, _ = corner_maps(cam, pose_true)
    T, trace = icp.icp(cam, Din, Dm, Nm, pose_m, pose_m, iters=(10, 5, 4))
    assert np.abs(T - pose_true).max() < 1e-4, np.abs(T - pose_true).max()
    assert trace[-1][2] > 1000 and trace[-1][1] < trace[0][1]
