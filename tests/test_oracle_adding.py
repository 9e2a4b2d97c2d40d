"""Pins of the adding / state-management reference (oracle/adding.py):
hand-made pixels for each clause of Eq. 6, closed forms of the vertex and
normal maps on planes, the disc orientation against scipy's rotation, the
order and capacity of the added rows, and each state-management rule."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import adding as A
from rtg_synth import camera

P = A.params()


def _px(T, Dr, D, dc):
    """One-pixel images: rendered T, depth Dr, input depth D, colour error
    dc per channel (rendered 0.5 + dc, input 0.5)."""
    return (np.full((1, 1, 3), 0.5 + dc, np.float32), np.array([[Dr]], np.float32),
            np.array([[T]], np.float32), np.full((1, 1, 3), 0.5, np.float32), np.array([[D]], np.float32))


@pytest.mark.parametrize("T,Dr,D,dc,code", [
    (0.6, 2.0, 2.0, 0.0, 1),     # light passes: new geometry
    (0.4, 2.2, 2.0, 0.0, 1),     # depth error 0.2 > 0.1
    (0.4, -1.0, 2.0, 0.0, 1),    # no hit, valid input depth
    (0.4, 2.05, 2.0, 0.2, 2),    # geometry right, colour error 0.2 > 0.1
    (0.4, 2.05, 2.0, 0.05, 0),   # both errors small
    (0.6, 2.0, 0.0, 0.5, 0),     # invalid input depth: neither mask
    (0.5, 2.0, 2.0, 0.0, 0),     # T = delta_T exactly: not above it
])
def test_adding_mask_clauses(T, Dr, D, dc, code):
    assert A.adding_masks(P, *_px(T, Dr, D, dc))[0, 0] == code


def test_vertex_map_at_the_principal_point_and_fronto_plane_normals():
    cam = camera(8, 6, 50.0, 60.0)
    D = np.full((6, 8), 2.5)
    V = A.vertex_map(cam, D)
    # pixel (3, 2) has centre (3.5, 2.5); cx = 4, cy = 3
    np.testing.assert_allclose(V[2, 3], [2.5 * (-0.5 / 50.0), 2.5 * (-0.5 / 60.0), 2.5], rtol=0, atol=1e-15)
    N, ok = A.normal_map(cam, D)
    assert ok[:-1, :-1].all() and not ok[-1].any() and not ok[:, -1].any()
    np.testing.assert_allclose(N[:-1, :-1], np.broadcast_to([0.0, 0.0, -1.0], N[:-1, :-1].shape), atol=1e-12)


def test_normal_of_a_tilted_plane():
    """Plane z = z0 + a X in camera coordinates: along the ray of pixel u,
    D = z0 / (1 - a r_x) with r_x = (u_x - cx) / fx; its normal, turned
    towards the camera, is (a, 0, -1) / |(a, 0, -1)|."""
    cam = camera(16, 12, 40.0, 40.0)
    a, z0 = 0.3, 3.0
    x = np.arange(16) + 0.5
    rx = (x - cam["cx"]) / cam["fx"]
    D = np.broadcast_to(z0 / (1.0 - a * rx), (12, 16)).copy()
    N, ok = A.normal_map(cam, D)
    ref = np.array([a, 0.0, -1.0]) / np.hypot(a, 1.0)
    np.testing.assert_allclose(N[ok], np.broadcast_to(ref, N[ok].shape), atol=1e-12)


def test_disc_orientation_maps_the_thin_axis_to_the_normal():
    rng = np.random.default_rng(3)
    n = rng.standard_normal((50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    n = np.vstack([n, [[0, 0, 1.0], [0, 0, -1.0]]])
    q = A.quat_z_to(n)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()   # scipy: (x, y, z, w)
    np.testing.assert_allclose(R[:, :, 2], n, atol=1e-12)


def _frame(seed, H=12, W=16):
    rng = np.random.default_rng(seed)
    cam = camera(W, H, 20.0, 20.0)
    D = rng.uniform(1.0, 3.0, (H, W)).astype(np.float32)
    D[rng.random((H, W)) < 0.1] = 0.0
    C = rng.random((H, W, 3)).astype(np.float32)
    Cr = (C + rng.choice([0.0, 0.3], (H, W, 1))).astype(np.float32)
    Dr = (D + rng.choice([0.0, 0.5], (H, W))).astype(np.float32)
    Tr = rng.choice([0.2, 0.7], (H, W), p=[0.8, 0.2]).astype(np.float32)
    I = rng.integers(-1, 30, (H, W)).astype(np.int32)
    un = (rng.random(30) < 0.5).astype(np.uint8)
    rand = rng.random((H, W)).astype(np.float32)
    return cam, D, C, Cr, Dr, Tr, I, un, rand


def test_added_rows_follow_the_rules_in_raster_order():
    cam, D, C, Cr, Dr, Tr, I, un, rand = _frame(4)
    Pp = A.params(rate=0.5)
    pose = np.concatenate([np.eye(3).ravel(), [0.1, -0.2, 0.3]])
    out = A.add_gaussians(cam, Pp, pose, C, D, Cr, Dr, Tr, I, un, rand, 7, 30, 10 ** 6)
    code = out["mask"]
    N, nok = A.normal_map(cam, D)
    rows = out["rows"]
    ys, xs = out["candidates"][:, 0], out["candidates"][:, 1]
    assert len(ys) == out["n_added"] > 0
    assert np.all(np.diff(ys * 16 + xs) > 0)
    for k, (y, x) in enumerate(zip(ys, xs)):
        assert rand[y, x] < 0.5 and nok[y, x]
        if code[y, x] == 1:
            assert rows["opacity"][k] == 0.99
        else:
            assert code[y, x] == 2 and I[y, x] >= 0 and un[I[y, x]] == 0 and rows["opacity"][k] == 0.1
            assert rows["scale"][k, 0] <= 0.01
        V = A.vertex_map(cam, D)[y, x]
        np.testing.assert_allclose(rows["pos"][k], V + [0.1, -0.2, 0.3], atol=1e-12)
        np.testing.assert_allclose(rows["scale"][k, 2], 0.1 * rows["scale"][k, 0], rtol=1e-15)
    assert np.all(rows["tstamp"] == 7)
    # every pixel that qualifies is listed
    qual = (rand < 0.5) & nok & ((code == 1) | ((code == 2) & (I >= 0) & (un[np.clip(I, 0, None)] == 0)))
    assert qual.sum() == len(ys)
    # capacity: only the first rows fit
    few = A.add_gaussians(cam, Pp, pose, C, D, Cr, Dr, Tr, I, un, rand, 7, 30, 33)
    assert few["n_added"] == 3
    np.testing.assert_array_equal(few["rows"]["pos"], rows["pos"][:3])


def test_state_rules():
    Pp = A.params(delta_eta=10, delta_e=2, delta_t=5)
    # Gaussians: 0 stable hit by error pixels (e 2 -> 3 > 2: becomes unstable)
    # 1 stable hit, e 0 -> 1; 2 unstable, eta 11 > 10: becomes stable;
    # 3 unstable, old (k - t = 6 > 5): removed; 4 unstable, young: kept;
    # 5 stable not hit: unchanged
    un = np.array([0, 0, 1, 1, 1, 0], np.uint8)
    eta = np.array([50, 50, 11, 3, 3, 50])
    err = np.array([2, 0, 0, 0, 0, 1])
    ts = np.array([0, 0, 0, 4, 9, 0])
    k = 10
    H, W = 2, 3
    C = np.full((H, W, 3), 0.5, np.float32)
    Cr = C.copy()
    Cr[0, 0] += 0.5
    Cr[0, 1] += 0.5
    Cr[1, 0] += 0.5
    D = np.full((H, W), 2.0, np.float32)
    Dr = D.copy()
    I = np.array([[0, 0, 5], [1, 2, 3]], np.int32)   # pixels (0,0),(0,1) hit 0 twice: counted once
    u2, e2, r2, t2, keep = A.state_update(Pp, Cr, Dr, I, C, D, un, eta, err, ts, k)
    np.testing.assert_array_equal(r2, [0, 1, 0, 0, 0, 1])
    np.testing.assert_array_equal(u2, [1, 0, 0, 1, 1, 0])
    np.testing.assert_array_equal(e2, [0, 50, 11, 3, 3, 50])
    np.testing.assert_array_equal(t2, [10, 0, 0, 4, 9, 0])
    np.testing.assert_array_equal(keep, [1, 1, 1, 0, 1, 1])


def test_confidence_count_counts_colour_updates_of_unstable_rows():
    un = np.array([1, 1, 0, 1], np.uint8)
    g = np.array([[0, 0, 1e-9], [0, 0, 0], [1, 1, 1], [-2, 0, 0]], np.float32)
    np.testing.assert_array_equal(A.confidence_count(un, g, np.array([0, 5, 7, 1])), [1, 5, 7, 2])
