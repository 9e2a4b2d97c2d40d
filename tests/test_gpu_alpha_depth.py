"""GPU parity of the alpha-blended depth mode (the depth-rendering ablation:
D = sum_i z_i f_i T_i, index map still by the first hit of Eq. 5) against
oracle/alpha_depth.py, through the C ABI: render (colour, transmission and
index map unchanged; the blended depth), gradients of every parameter, and
the fused L1 step against the separate calls."""
import numpy as np
import pytest
import torch

from oracle import alpha_depth as ad
from oracle import oracle as orc
from rtg_synth import random_upstream
from tests.gpu_helpers import (GRAD_GAMMA, PRECISE_KAPPA, T_EPS, assert_parity, compare_forward,
                               dev_poses, err_stats, fmt_stats, gpu_forward, grad_stats, need_gpu)
from tests.scenes_small import random_pose, random_scene, small_cam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _scene(seed, n=1500):
    rng = np.random.default_rng(seed)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    pose_b = look_at(tg + 0.3 * Rg[:, 0], target, up=-Rg[:, 1])
    sc = random_scene(rng, n, centre=target, spread=0.6, unstable_frac=0.6)
    return sc, np.stack([pose_a, pose_b])


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_alpha_depth_render_and_gradients_match_oracle(tile):
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(100, 75, 90.0)
    sc, poses = _scene(80 + tile[0])
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(81)
    mask = (rng.random((F, 75, 100)) < 0.5).astype(np.uint8)
    rast = Rasterizer(cam, N, F, tile_w=tile[0], tile_h=tile[1], depth_mode=1)
    g = gpu_forward(rast, sc, poses, mask)
    P = orc.make_params(cam, tile=tile)
    recs = orc.project(P, sc, poses)
    pix = orc.masked_pixels(mask)
    out = ad.render(P, recs, sc, pix)
    errs = compare_forward(g, pix, out)
    # pixels that stop compositing below t_eps drop less than t_eps z of depth
    zmax = float(recs["pc"][..., 2][recs["visible"] != 0].max())
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    errs["depth"] = err_stats(g["depth"][f, y, x], out["depth"], floor=2e4 * T_EPS * zmax)
    assert (out["depth"] == -1).sum() > 0 and (out["depth"] > 0).sum() > 0
    assert np.array_equal(g["depth"][f, y, x] == -1, out["depth"] == -1)
    gC, gD = random_upstream(mask, seed=82)
    grads = rast.alloc_grads()
    C, D, T, I = g["tensors"]
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), D, T, I, torch.as_tensor(gC).cuda(),
                       torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    ref, bnd = ad.backward(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x],
                           bound=(GRAD_GAMMA, T_EPS, PRECISE_KAPPA))
    errs.update(grad_stats(grads, ref, sc["unstable"], bnd))
    print("alpha-blended depth", tile, fmt_stats(errs))
    assert errs["index_mismatch"] == 0
    assert_parity(errs)


def test_alpha_depth_l1_step_through_the_separate_calls():
    """With alpha-blended depth the colour and depth paths share the
    footprint and opacity gradients, so the fused L1 backward (which scales
    the two paths' slots apart) reports RTG_E_UNSUPPORTED; the L1 loss
    kernels + the plain backward give the oracle's gradients of the L1 loss
    at its upstream."""
    from paper_2404_19706_amd import Rasterizer
    from paper_2404_19706_amd._lib import RTG_E_UNSUPPORTED, lib
    cam = small_cam(100, 75, 90.0)
    sc, poses = _scene(90)
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(91)
    mask = (rng.random((F, 75, 100)) < 0.6).astype(np.uint8)
    rast = Rasterizer(cam, N, F, depth_mode=1)
    g = gpu_forward(rast, sc, poses, mask)
    C, D, T, I = g["tensors"]
    Cgt = torch.rand_like(C)
    Dgt = torch.where(torch.rand_like(D) < 0.9, torch.rand_like(D) * 3 + 0.5, torch.zeros_like(D))
    import ctypes
    _p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = lib().rtg_backward_raster_l1(rast._plan, _p(g["ws"]), _p(C), _p(D), _p(T), _p(I), _p(Cgt), _p(Dgt), None)
    assert st == RTG_E_UNSUPPORTED
    dp = dev_poses(poses)
    dC, dD = torch.zeros_like(C), torch.zeros_like(D)
    loss = torch.zeros(1, device="cuda")
    rast.loss_l1_into(g["ws"], C, D, Cgt, Dgt, dC, dD, loss)
    grads = rast.alloc_grads()
    rast.backward_raster(g["ws"], D, T, I, dC, dD)
    rast.backward_project(g["ws"], g["params"], dp, grads)
    torch.cuda.synchronize()
    P = orc.make_params(cam)
    recs = orc.project(P, sc, poses)
    pix = orc.masked_pixels(mask)
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    gC = dC.cpu().numpy()[f, y, x]
    gD = dD.cpu().numpy()[f, y, x]
    ref, bnd = ad.backward(P, recs, sc, poses, pix, gC, gD, bound=(GRAD_GAMMA, T_EPS, PRECISE_KAPPA))
    errs = grad_stats(grads, ref, sc["unstable"], bnd)
    print("alpha-blended depth, L1 step", fmt_stats(errs))
    assert_parity(errs)
