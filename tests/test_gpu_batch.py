"""GPU checks of the batched-keyframe form and its autotuner.

A batch of F frames in one pass must give, frame by frame, exactly the
single-frame passes' forward outputs (the frame only selects pairs and
pixels; no arithmetic crosses frames), and the sum over frames of their
gradients for the same upstream (up to FP32 rounding of the per-Gaussian
accumulation).  The batched result is also checked against the oracle.
The autotuner must return one of its candidates, reproduce the candidate's
outputs bit for bit (tile shape and queue mode change no value) and cache
its choice."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from rtg_synth import random_upstream
from tests.gpu_helpers import (assert_parity, compare_forward, dev_mask, dev_params, dev_poses, fmt_stats, grad_stats,
                               need_gpu, oracle_grads, rel_err)
from tests.scenes_small import random_pose, random_scene, small_cam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _scene_and_poses(seed, F=3, n=1800):
    rng = np.random.default_rng(seed)
    from rtg_synth import look_at
    pose0, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    poses = [pose0]
    for k in range(1, F):
        eye = tg + 0.12 * k * Rg[:, 0] - 0.05 * k * Rg[:, 1]
        poses.append(look_at(eye, target, up=-Rg[:, 1]))
    sc = random_scene(rng, n, centre=target, spread=0.6, unstable_frac=0.5)
    return sc, np.stack(poses)


@pytest.mark.parametrize("tile,ipp", [((16, 16), 0), ((8, 8), 1), ((32, 8), 4)])
def test_batched_equals_per_frame_passes(tile, ipp):
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(120, 90, 100.0)
    sc, poses = _scene_and_poses(3)
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(4)
    # uneven masks: 10 %, 50 %, 90 % of the pixels
    mask = np.stack([(rng.random((90, 120)) < p).astype(np.uint8) for p in (0.1, 0.5, 0.9)])
    params, dp, dm = dev_params(sc), dev_poses(poses), dev_mask(mask)
    gC, gD = random_upstream(mask, seed=5)
    tgC, tgD = torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda()

    rb = Rasterizer(cam, N, F, tile_w=tile[0], tile_h=tile[1], items_per_pop=ipp)
    Cb, Db, Tb, Ib, wsb = rb.forward(params, dp, dm)
    gb = rb.backward_into(wsb, params, dp, Db, Tb, Ib, tgC, tgD, rb.alloc_grads())
    torch.cuda.synchronize()
    assert rb.read_status(wsb)["status"] == 0

    sums = {k: torch.zeros_like(v, dtype=torch.float64) for k, v in gb.items()}
    for f in range(F):
        rf = Rasterizer(cam, N, 1, tile_w=tile[0], tile_h=tile[1], items_per_pop=ipp)
        Cf, Df, Tf, If, wsf = rf.forward(params, dp[f:f + 1], dm[f:f + 1])
        gf = rf.backward_into(wsf, params, dp[f:f + 1], Df, Tf, If, tgC[f:f + 1].contiguous(),
                              tgD[f:f + 1].contiguous(), rf.alloc_grads())
        torch.cuda.synchronize()
        for a, b in ((Cf, Cb), (Df, Db), (Tf, Tb), (If, Ib)):
            assert torch.equal(a[0], b[f]), "frame %d differs between batched and single-frame pass" % f
        for k in sums:
            sums[k] += gf[k].double()
    for k in sums:
        assert rel_err(gb[k].cpu().numpy(), sums[k].cpu().numpy()) <= 1e-5, k

    # and the batch against the oracle
    P = orc.make_params(cam, tile=tile)
    recs = orc.project(P, sc, poses)
    pix = orc.masked_pixels(mask)
    out = orc.render(P, recs, sc, pix)
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    g = {"color": Cb.cpu().numpy(), "depth": Db.cpu().numpy(), "trans": Tb.cpu().numpy(), "index": Ib.cpu().numpy()}
    e = compare_forward(g, pix, out, recs)
    assert e["index_mismatch"] == 0
    gref, gbnd = oracle_grads(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x])
    e.update(grad_stats(gb, gref, sc["unstable"], gbnd))
    print("batched vs oracle", tile, ipp, fmt_stats(e))
    assert_parity(e)


def test_fit_rasterizer_grows_capacity():
    from paper_2404_19706_amd.autotune import fit_rasterizer
    cam = small_cam(120, 90, 100.0)
    sc, poses = _scene_and_poses(6, F=2)
    params, dp = dev_params(sc), dev_poses(poses)
    dm = torch.ones((2, 90, 120), dtype=torch.uint8, device="cuda")
    r, ws, st = fit_rasterizer(cam, len(sc["pos"]), 2, params, dp, dm, first_guess=64)
    assert st["status"] == 0 and st["pairs"] > 64
    assert r.max_pairs >= st["pairs"]


def test_fit_rasterizer_shrinks_capacity():
    from paper_2404_19706_amd.autotune import fit_rasterizer
    cam = small_cam(120, 90, 100.0)
    sc, poses = _scene_and_poses(6, F=2)
    params, dp = dev_params(sc), dev_poses(poses)
    dm = torch.ones((2, 90, 120), dtype=torch.uint8, device="cuda")
    r, ws, st = fit_rasterizer(cam, len(sc["pos"]), 2, params, dp, dm, first_guess=1 << 22)
    assert st["status"] == 0 and not st["overflow"]
    assert st["pairs"] <= r.max_pairs == int(st["pairs"] * 1.25) + 4096


def test_autotuner_choice_is_a_candidate_and_cached(tmp_path):
    from paper_2404_19706_amd import Rasterizer
    from paper_2404_19706_amd.autotune import Autotuner
    cam = small_cam(120, 90, 100.0)
    sc, poses = _scene_and_poses(8, F=2)
    F, N = poses.shape[0], len(sc["pos"])
    params, dp = dev_params(sc), dev_poses(poses)
    rng = np.random.default_rng(9)
    dm = dev_mask((rng.random((F, 90, 120)) < 0.4).astype(np.uint8))
    path = str(tmp_path / "tune.json")
    at = Autotuner(cache_path=path, reps=2)
    res = at.tune(cam, params, dp, dm)
    assert not res["cached"]
    assert (res["tile_w"], res["tile_h"]) in ((16, 16), (8, 8), (32, 8))
    assert (res["items_per_pop"], res["static_share"]) in ((0, 0), (4, 30), (2, 50))
    # nine shared schedules, then the forward's own on top of the best
    from paper_2404_19706_amd.autotune import FWD_SCHEDULES
    assert 9 < len(res["table"]) <= 9 + len(FWD_SCHEDULES)
    assert (res["fwd_items_per_pop"], res["fwd_static_share"]) in ((-1, -1),) + FWD_SCHEDULES
    again = Autotuner(cache_path=path).tune(cam, params, dp, dm)
    assert again["cached"] and again["tile_w"] == res["tile_w"] and again["items_per_pop"] == res["items_per_pop"]
    assert again["static_share"] == res["static_share"]
    # the chosen configuration renders exactly what the default one does
    outs = []
    for kw in (dict(tile_w=res["tile_w"], tile_h=res["tile_h"], items_per_pop=res["items_per_pop"],
                    static_share=res["static_share"], fwd_items_per_pop=res["fwd_items_per_pop"],
                    fwd_static_share=res["fwd_static_share"]), {}):
        r = Rasterizer(cam, N, F, **kw)
        C, D, T, I, _ = r.forward(params, dp, dm)
        torch.cuda.synchronize()
        outs.append((C, D, T, I))
    for a, b in zip(*outs):
        assert torch.equal(a, b)
