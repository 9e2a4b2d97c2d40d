"""Pins of the oracle's projection step (Sec. 3.1, Eq. 2) against closed
forms and independent library routines (scipy rotations, numerical
Jacobians of the pinhole map)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import oracle as orc
from tests.scenes_small import identity_pose, random_pose, random_scene, scene_from, small_cam

CAM = small_cam()


def _one(pos, scale, rot, op=0.99, pose=None, **kw):
    sc = scene_from([pos], [scale], [rot], [op], [[0.5, 0.5, 0.5]])
    P = orc.make_params(CAM, **kw)
    return orc.project(P, sc, identity_pose() if pose is None else pose)[0, 0]


def test_closed_form_on_axis():
    """Identity rotation and pose, centre on the optical axis: mu is the
    principal point and Sigma_2D = diag((fx sx/Z)^2, (fy sy/Z)^2)."""
    Z, sx, sy = 2.5, 0.04, 0.02
    r = _one([0, 0, Z], [sx, sy, 0.004], [1, 0, 0, 0])
    sx, sy = float(np.float32(sx)), float(np.float32(sy))   # inputs are float32
    assert r["culled"] == 0 and r["visible"] == 1
    assert r["mu"][0] == CAM["cx"] and r["mu"][1] == CAM["cy"]
    np.testing.assert_allclose(r["cov"], [(100 * sx / Z) ** 2, 0.0, (100 * sy / Z) ** 2], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(r["conic"], [1 / (100 * sx / Z) ** 2, 0.0, 1 / (100 * sy / Z) ** 2], rtol=1e-13)
    assert r["z32"] == np.float32(Z)
    # thin axis is z -> normal along the optical axis, plane offset = Z
    np.testing.assert_allclose(np.abs(r["nc"]), [0, 0, 1], atol=1e-15)
    assert abs(abs(r["h"]) - Z) < 1e-14


def test_rotation_about_view_axis_swaps_axes():
    Z, sx, sy = 2.0, 0.05, 0.01
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)      # 90 degrees about z
    r = _one([0, 0, Z], [sx, sy, 0.003], [c, 0, 0, s])
    sx, sy = float(np.float32(sx)), float(np.float32(sy))
    np.testing.assert_allclose(r["cov"], [(100 * sy / Z) ** 2, 0.0, (100 * sx / Z) ** 2], rtol=1e-12, atol=1e-12)


def _num_jacobian(pc, fx, fy):
    def pi(v):
        return np.array([fx * v[0] / v[2], fy * v[1] / v[2]])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-6 * max(1.0, abs(pc[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (pi(pc + e) - pi(pc - e)) / (2 * h)
    return J


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_against_scipy_rotation_and_numerical_jacobian(seed):
    """Sigma_2D = J W R S^2 R^T W^T J^T with R from scipy (scalar-last
    quaternion convention converted), W = R_g^T, and J the numerical
    Jacobian of the pinhole map; mu = pi(R_g^T (p - t_g))."""
    rng = np.random.default_rng(seed)
    pose, Rg, tg = random_pose(rng)
    sc = random_scene(rng, 200, centre=tg + 2.0 * Rg[:, 2], spread=0.6)
    P = orc.make_params(CAM)
    recs = orc.project(P, sc, pose[None])[0]
    checked = 0
    for i in range(200):
        r = recs[i]
        if r["culled"]:
            continue
        q = sc["rot"][i].astype(np.float64)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S3 = R @ np.diag(sc["scale"][i].astype(np.float64) ** 2) @ R.T
        pc = Rg.T @ (sc["pos"][i].astype(np.float64) - tg)
        J = _num_jacobian(pc, CAM["fx"], CAM["fy"])
        S2 = J @ Rg.T @ S3 @ Rg @ J.T
        np.testing.assert_allclose(r["pc"], pc, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(r["mu"], [CAM["fx"] * pc[0] / pc[2] + CAM["cx"],
                                             CAM["fy"] * pc[1] / pc[2] + CAM["cy"]], rtol=1e-12)
        np.testing.assert_allclose(r["cov"], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7,
                                   atol=1e-9 * np.abs(S2).max())
        Q = np.linalg.inv(np.array([[r["cov"][0], r["cov"][1]], [r["cov"][1], r["cov"][2]]]))
        np.testing.assert_allclose(r["conic"], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-9,
                                   atol=1e-12 * np.abs(Q).max())
        k = int(np.argmin(sc["scale"][i]))
        n = Rg.T @ R[:, k]
        assert abs(abs(np.dot(n, r["nc"])) - 1.0) < 1e-12
        assert abs(np.dot(pc, r["nc"]) - r["h"]) < 1e-12
        # the normal is the eigenvector of Sigma_3D with the smallest eigenvalue
        w, V = np.linalg.eigh(S3)
        assert abs(abs(np.dot(V[:, 0], R[:, k])) - 1.0) < 1e-6
        assert r["tau32"] == np.float32(1.0 + 2.0 * np.log(np.float64(sc["opacity"][i])))
        checked += 1
    assert checked > 100


def test_culling():
    assert _one([0, 0, 0.1], [0.01] * 3, [1, 0, 0, 0])["culled"] == 1       # before near plane
    assert _one([0, 0, -2], [0.01] * 3, [1, 0, 0, 0])["culled"] == 1        # behind camera
    assert _one([0, 0, 2], [0.01] * 3, [0, 0, 0, 0])["culled"] == 1         # zero quaternion
    assert _one([0, 0, 2], [0.0, 0.0, 0.0], [1, 0, 0, 0])["culled"] == 1    # zero area
    assert _one([np.nan, 0, 2], [0.01] * 3, [1, 0, 0, 0])["culled"] == 1
    far = _one([50, 0, 2], [0.01] * 3, [1, 0, 0, 0])
    assert far["culled"] == 0 and far["visible"] == 0                        # off-image
    assert _one([0, 0, 2], [0.01] * 3, [1, 0, 0, 0], z_near=2.5)["culled"] == 1


def test_dilation_adds_to_diagonal():
    a = _one([0.1, -0.2, 2], [0.03, 0.02, 0.01], [0.9, 0.1, 0.3, 0.2])
    b = _one([0.1, -0.2, 2], [0.03, 0.02, 0.01], [0.9, 0.1, 0.3, 0.2], dilation=0.3)
    np.testing.assert_allclose(np.array(b["cov"]) - np.array(a["cov"]), [0.3, 0.0, 0.3], atol=1e-12)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_rect_is_conservative_brute_force(tile):
    """Every pixel whose decision d^2 (from the stored fp32 centre and
    conic, evaluated here in float64 with slack) is within the cut-off lies
    inside the record's pixel rectangle."""
    rng = np.random.default_rng(5)
    sc = random_scene(rng, 300, spread=0.8, smin=0.005, smax=0.2)
    P = orc.make_params(CAM, tile=tile)
    recs = orc.project(P, sc, identity_pose())[0]
    ys, xs = np.mgrid[0:CAM["height"], 0:CAM["width"]]
    ux, uy = xs + 0.5, ys + 0.5
    n_vis = 0
    for r in recs:
        if r["culled"]:
            continue
        dx = ux - np.float64(r["mu32"][0])
        dy = uy - np.float64(r["mu32"][1])
        a, b, c = (np.float64(v) for v in r["conic32"])
        dd = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        inside = dd <= 9.0 * (1 + 1e-5)
        if not r["visible"]:
            assert not inside.any()
            continue
        n_vis += 1
        x0, x1, y0, y1 = r["rect"]
        assert 0 <= x0 <= x1 < CAM["width"] and 0 <= y0 <= y1 < CAM["height"]
        iy, ix = np.nonzero(inside)
        assert (ix >= x0).all() and (ix <= x1).all() and (iy >= y0).all() and (iy <= y1).all()
    assert n_vis > 100
