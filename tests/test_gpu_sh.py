"""GPU parity of the view-dependent SH colour (Sec. 3.1, the colour of Eq. 1
from SH coefficients and the view direction) against the SH oracle
(oracle/sh.py), through the C ABI: the render, the gradients (SH
coefficients of every band, and positions, which also move the view
direction), the fused L1 step against the separate calls, the Adam update
with its band-0 and higher-band rates, and the SH rows of new Gaussians."""
import numpy as np
import pytest
import torch

from oracle import adding as oad
from oracle import oracle as orc
from oracle import sh
from rtg_synth import random_upstream
from tests.gpu_helpers import (EL_MAX_TOL, GRAD_GAMMA, PRECISE_KAPPA, T_EPS, assert_parity, compare_forward,
                               dev_poses, err_stats, fmt_stats, gpu_forward, need_gpu, rel_err)
from tests.scenes_small import random_pose, random_scene, small_cam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _scene(seed, degree, n=1500):
    rng = np.random.default_rng(seed)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    pose_b = look_at(tg + 0.4 * Rg[:, 0], target, up=-Rg[:, 1])
    sc = random_scene(rng, n, centre=target, spread=0.6, unstable_frac=0.6)
    K = sh.n_coef(degree)
    coef = (rng.standard_normal((n, K, 3)) * 0.25).astype(np.float32)
    coef[:, 0, :] = (sc["color"] / 0.28209479177387814).astype(np.float32)
    sc["color"] = coef
    return sc, np.stack([pose_a, pose_b])


def _grad_stats(grads, ref, bnd, unstable):
    out = {}
    un = np.asarray(unstable) != 0
    for k in ("pos", "scale", "rot", "opacity", "color"):
        got = grads[k].cpu().numpy()
        assert (got[~un] == 0).all(), k
        out["d_" + k] = err_stats(got, ref[k], floor=bnd[k] / EL_MAX_TOL)
    return out


@pytest.mark.parametrize("degree,tile", [(1, (16, 16)), (2, (8, 8)), (3, (32, 8))])
def test_sh_render_and_gradients_match_oracle(degree, tile):
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(100, 75, 90.0)
    sc, poses = _scene(20 + degree, degree)
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(30 + degree)
    mask = (rng.random((F, 75, 100)) < 0.5).astype(np.uint8)
    rast = Rasterizer(cam, N, F, tile_w=tile[0], tile_h=tile[1], sh_degree=degree)
    assert rast.color_shape == (N, (degree + 1) ** 2, 3)
    g = gpu_forward(rast, sc, poses, mask)
    assert g["status"]["status"] == 0
    P = orc.make_params(cam, tile=tile)
    recs = orc.project(P, sc, poses)
    pix = orc.masked_pixels(mask)
    out = sh.render(P, recs, sc, poses, pix, degree)
    errs = compare_forward(g, pix, out, recs)
    # SH colours take both signs, so a pixel's blend can cancel: the colour's
    # elementwise floor is the binary32 error bound of its terms,
    # GRAD_GAMMA sum |c_i| f_i T_i (admitted in full by the 1e-4 gate)
    cabs = sh.render(P, recs, sc, poses, pix, degree, absolute=True)["color"]
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    errs["color"] = err_stats(g["color"][f, y, x], out["color"], floor=GRAD_GAMMA * cabs / EL_MAX_TOL)
    # the view direction differs between the frames: the colours do too
    cols = sh.colors(sc["color"], sc["pos"], poses, degree)
    assert np.abs(cols[0] - cols[1]).max() > 1e-3
    gC, gD = random_upstream(mask, seed=40 + degree)
    grads = rast.alloc_grads()
    C, D, T, I = g["tensors"]
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), D, T, I, torch.as_tensor(gC).cuda(),
                       torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    ref, bnd = sh.backward(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x], degree,
                           bound=(GRAD_GAMMA, T_EPS, PRECISE_KAPPA))
    errs.update(_grad_stats(grads, ref, bnd, sc["unstable"]))
    print("SH degree %d" % degree, fmt_stats(errs))
    assert errs["index_mismatch"] == 0
    assert_parity(errs)
    # the higher bands receive gradients
    assert np.abs(grads["color"].cpu().numpy()[:, 1:, :]).max() > 0


def test_sh_fused_l1_step_equals_separate_calls():
    """The fused L1 backward with SH colour equals the L1 loss kernels + the
    plain backward (gradients within float summation order)."""
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(100, 75, 90.0)
    sc, poses = _scene(50, 2)
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(51)
    mask = (rng.random((F, 75, 100)) < 0.6).astype(np.uint8)
    rast = Rasterizer(cam, N, F, sh_degree=2)
    g = gpu_forward(rast, sc, poses, mask)
    C, D, T, I = g["tensors"]
    Cgt = torch.rand_like(C)
    Dgt = torch.where(torch.rand_like(D) < 0.9, torch.rand_like(D) * 3 + 0.5, torch.zeros_like(D))
    dp = dev_poses(poses)
    dC = torch.zeros_like(C)
    dD = torch.zeros_like(D)
    loss_a = torch.zeros(1, device="cuda")
    rast.loss_l1_into(g["ws"], C, D, Cgt, Dgt, dC, dD, loss_a)
    ga = rast.alloc_grads()
    rast.backward_raster(g["ws"], D, T, I, dC, dD)
    rast.backward_project(g["ws"], g["params"], dp, ga)
    gb = rast.alloc_grads()
    loss_b = torch.zeros(1, device="cuda")
    rast.backward_raster_l1(g["ws"], C, D, T, I, Cgt, Dgt)
    rast.backward_project_l1(g["ws"], g["params"], dp, gb, loss_b)
    torch.cuda.synchronize()
    assert abs(loss_a.item() - loss_b.item()) <= 1e-5 * abs(loss_a.item())
    for k in ("pos", "scale", "rot", "opacity", "color"):
        assert torch.count_nonzero(ga[k]) > 0, k
        assert rel_err(gb[k].cpu().numpy(), ga[k].cpu().numpy()) <= 1e-5, k


def test_sh_adam_uses_band_rates():
    """Adam with SH coefficients: band 0 at lr_color, bands 1..3 at
    lr_sh_rest, moments [N][10 + 3K]; against the oracle's Adam."""
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(40, 30, 40.0)
    n, deg = 200, 3
    K = sh.n_coef(deg)
    rng = np.random.default_rng(60)
    sc = random_scene(rng, n, unstable_frac=0.5)
    sc["color"] = rng.standard_normal((n, K, 3)).astype(np.float32)
    rast = Rasterizer(cam, n, 1, sh_degree=deg)
    from tests.gpu_helpers import dev_params
    params = [p.clone() for p in dev_params(sc)]
    m, v, step = rast.alloc_adam_state()
    assert m.shape == (n, 10 + 3 * K)
    lr = (1e-3, 2e-3, 1e-3, 5e-4, 2.5e-5)
    ref = {"pos": sc["pos"].astype(np.float64), "c0": sc["color"][:, 0, :].astype(np.float64),
           "crest": sc["color"][:, 1:, :].reshape(n, -1).astype(np.float64)}
    stt = {k: (np.zeros_like(x), np.zeros_like(x)) for k, x in ref.items()}
    un = sc["unstable"]
    for it in range(1, 4):
        grads = {k: torch.as_tensor(rng.standard_normal(s).astype(np.float32)).cuda()
                 for k, s in (("pos", (n, 3)), ("scale", (n, 3)), ("rot", (n, 4)), ("color", (n, K, 3)))}
        gcol = grads["color"].cpu().numpy()
        rast.adam(params, grads, m, v, step, lr=lr, eps=1e-15)
        for k, lrk, gk in (("pos", lr[0], grads["pos"].cpu().numpy()), ("c0", lr[3], gcol[:, 0, :]),
                           ("crest", lr[4], gcol[:, 1:, :].reshape(n, -1))):
            ref[k], mm, vv = orc.adam_step(ref[k], gk, stt[k][0], stt[k][1], it, lrk, un, eps=1e-15)
            stt[k] = (mm, vv)
    col = params[4].cpu().numpy()
    assert np.allclose(params[0].cpu().numpy(), ref["pos"], rtol=1e-5, atol=1e-6)
    assert np.allclose(col[:, 0, :], ref["c0"], rtol=1e-5, atol=1e-6)
    assert np.allclose(col[:, 1:, :].reshape(n, -1), ref["crest"], rtol=1e-5, atol=1e-7)
    # the higher bands moved by 0.05 of band 0's rate
    moved0 = np.abs(col[:, 0, :] - sc["color"][:, 0, :])[un != 0].max()
    moved1 = np.abs(col[:, 1:, :] - sc["color"][:, 1:, :])[un != 0].max()
    assert 0 < moved1 < 0.2 * moved0


def test_sh_rows_of_added_gaussians():
    """rtg_add_gaussians with sh_degree 2 writes the band-0 coefficient c /
    Y_00 of the pixel colour and zero higher bands (the oracle's rows)."""
    from paper_2404_19706_amd import mapping
    cam = small_cam(64, 48, 60.0)
    H, W = 48, 64
    rng = np.random.default_rng(70)
    D = rng.uniform(1.0, 2.0, (H, W)).astype(np.float32)
    Cin = rng.random((H, W, 3)).astype(np.float32)
    Cr = np.zeros((H, W, 3), np.float32)
    Dr = np.full((H, W), -1.0, np.float32)
    Tr = np.ones((H, W), np.float32)
    Ir = np.full((H, W), -1, np.int32)
    rnd = rng.random((H, W)).astype(np.float32)
    pose = np.concatenate([np.eye(3).ravel(), [0.1, -0.2, 0.3]])
    P = oad.params(sh_degree=2)
    ref = oad.add_gaussians(cam, P, pose, Cin, D, Cr, Dr, Tr, Ir, np.zeros(1, np.uint8), rnd, 3, 0, 10000)
    n_new = ref["n_added"]
    assert n_new > 50
    state = mapping.alloc_state(10000, sh_degree=2)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()  # noqa: E731
    counts = mapping.add_gaussians(cam, mapping.adding_params(sh_degree=2), t(pose), t(Cin), t(D), t(Cr), t(Dr),
                                   t(Tr), t(Ir), t(rnd), 3, 0, state)
    torch.cuda.synchronize()
    assert int(counts[0]) == n_new
    got = state["color"][:n_new].cpu().numpy()
    assert got.shape == (n_new, 9, 3)
    np.testing.assert_allclose(got, ref["rows"]["color"], rtol=1e-6, atol=1e-7)
    assert (got[:, 1:, :] == 0).all()
