"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bar: bit-exact projection decisions, pair lists, tile ranges, index map and
M_unstable; <= 1e-4 normwise relative error on colour, depth, transmission
and every gradient tensor."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from rtg_synth import make_config, random_upstream
from tests.gpu_helpers import (assert_parity, compare_forward, dev_mask, dev_params, dev_poses, fmt_stats,
                               gpu_forward, grad_stats, need_gpu, oracle_forward, oracle_grads, rel_err, ws_view)
from tests.scenes_small import (edge_on_surfels, footprint_condition, identity_pose, random_pose, random_scene,
                                small_cam)

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _rast(cam, n, frames=1, **kw):
    from paper_2404_19706_amd import Rasterizer
    return Rasterizer(cam, n, frames, **kw)


def _two_pose_scene(seed, n=1500, cam=None):
    rng = np.random.default_rng(seed)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    pose_b = look_at(tg + 0.15 * Rg[:, 0], target, up=-Rg[:, 1])
    sc = random_scene(rng, n, centre=target, spread=0.6, unstable_frac=0.6)
    return sc, np.stack([pose_a, pose_b])


def _check_pairs(rast, ws, P, recs, mask, F, N, g):
    """Per-tile pair counts, starts and sorted Gaussian lists equal the
    oracle's binning."""
    b = orc.bin_pairs(P, recs, mask)
    nt = b["tile_active"].shape[1]
    tend = ws_view(rast, ws, "tile_end", torch.int32, F * nt).cpu().numpy()
    start = ws_view(rast, ws, "tile_start", torch.int32, F * nt).cpu().numpy()
    npairs = tend - start
    K = int(npairs.sum())
    assert K == b["K"] == g["status"]["pairs"]
    pairs = ws_view(rast, ws, "pairs", torch.int32, K).cpu().numpy().astype(np.int64)
    cnt = np.bincount(b["frame"] * nt + b["tile"], minlength=F * nt)
    assert np.array_equal(cnt, npairs)
    nz = cnt > 0
    assert np.array_equal(start[nz], np.concatenate([[0], np.cumsum(cnt)[:-1]])[nz])
    got_gid = pairs - (np.repeat(np.arange(F * nt), cnt) // nt) * N
    assert np.array_equal(got_gid, b["gid"])


# ------------------------------------------------------------ decisions

@pytest.mark.parametrize("tile,size,flat", [((16, 16), (100, 75), 0.0), ((8, 8), (100, 75), 0.0),
                                            ((32, 8), (100, 75), 0.0), ((8, 8), (1030, 1030), 0.0),
                                            ((8, 8), (100, 75), 1e-6), ((32, 8), (400, 300), 1e-9)])
def test_projection_and_binning_bit_exact(tile, size, flat):
    """Ragged tiles on both axes; the 1030x1030 case has 129 x 129 tiles of
    8x8, more than one binning block's LDS chunk of tiles.  The flat cases
    make every Gaussian a surfel of that thickness, so surfels seen near
    edge-on give needle footprints for the pair thinning (condition numbers
    above 1e5; at 1e-9 one binary32 conic is not positive definite)."""
    W, H = size
    cam = small_cam(W, H, 90.0 * W / 100.0)
    sc, poses = _two_pose_scene(1, n=1200)
    if flat:
        sc["scale"][:, 2] = flat
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(2)
    mask = (rng.random((F, H, W)) < 0.3).astype(np.uint8)
    mask[1, H // 4:H // 2, W // 3:4 * W // 5] = 1
    rast = _rast(cam, N, F, tile_w=tile[0], tile_h=tile[1])
    g = gpu_forward(rast, sc, poses, mask)
    P = orc.make_params(cam, tile=tile)
    recs = orc.project(P, sc, poses)
    ws = g["ws"]
    vis = ws_view(rast, ws, "vis", torch.int32, N).cpu().numpy().view(np.uint32)
    hot = ws_view(rast, ws, "hot", torch.float32, 16 * F * N).cpu().numpy().reshape(F, N, 16)
    zk = ws_view(rast, ws, "zkey", torch.float32, F * N).cpu().numpy().reshape(F, N)
    rect = ws_view(rast, ws, "rect", torch.int16, 4 * F * N).cpu().numpy().reshape(F, N, 4)
    for f in range(F):
        ov = recs["visible"][f] != 0
        gv = ((vis >> f) & 1) != 0
        assert np.array_equal(ov, gv), f
        r = recs[f][ov]
        h = hot[f][ov]
        assert np.array_equal(h[:, 0].view(np.uint32), r["mu32"][:, 0].view(np.uint32))
        assert np.array_equal(h[:, 1].view(np.uint32), r["mu32"][:, 1].view(np.uint32))
        assert np.array_equal(h[:, 2].view(np.uint32), r["conic32"][:, 0].view(np.uint32))
        assert np.array_equal(h[:, 3], 2.0 * r["conic32"][:, 1])
        assert np.array_equal(h[:, 4].view(np.uint32), r["conic32"][:, 2].view(np.uint32))
        assert np.array_equal(h[:, 6].view(np.uint32), r["tau32"].view(np.uint32))
        assert np.array_equal(zk[f][ov].view(np.uint32), r["z32"].view(np.uint32))
        assert np.array_equal(rect[f][ov].astype(np.int32), r["rect"])
    _check_pairs(rast, ws, P, recs, mask, F, N, g)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_edge_on_surfels_bit_exact_decisions(tile):
    """Surfels seen edge-on (needle footprints, condition numbers up to
    1e10): rectangles, visibility, pair lists and the index map bit-exact,
    including the pixels that binary32 rounding of the decision form admits
    beyond the ellipse."""
    cam = small_cam()
    sc = edge_on_surfels(np.random.default_rng(5), 400)
    poses = identity_pose()
    N = len(sc["pos"])
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    rast = _rast(cam, N, 1, tile_w=tile[0], tile_h=tile[1])
    g = gpu_forward(rast, sc, poses, mask)
    P, recs, pix, out = oracle_forward(cam, sc, poses, mask, tile=tile)
    ws = g["ws"]
    vis = ws_view(rast, ws, "vis", torch.int32, N).cpu().numpy().view(np.uint32)
    rect = ws_view(rast, ws, "rect", torch.int16, 4 * N).cpu().numpy().reshape(N, 4)
    ov = recs["visible"][0] != 0
    assert np.array_equal(ov, (vis & 1) != 0)
    assert np.array_equal(rect[ov].astype(np.int32), recs[0]["rect"][ov])
    _check_pairs(rast, ws, P, recs, mask, 1, N, g)
    e = compare_forward(g, pix, out, recs)
    print("edge-on surfels", tile, fmt_stats(e))
    assert e["index_mismatch"] == 0


@pytest.mark.parametrize("band", [2, 3, 4, 6, 8])
def test_needle_footprint_values(band):
    """Value parity on needle footprints: surfels seen exactly edge-on with
    thickness chosen so that the footprint condition number kappa lies in
    about [10^band, 10^(band+1)].  Colour, depth, transmission and the
    gradients of a random upstream against the oracle at every pixel."""
    cam = small_cam()
    lo, hi = -1.0 - (band + 1) / 2.0, -1.0 - band / 2.0
    sc = edge_on_surfels(np.random.default_rng(40 + band), 300, thick_exp=(lo, hi), tilt_exp=None)
    poses = identity_pose()
    N = len(sc["pos"])
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    rast = _rast(cam, N, 1)
    g = gpu_forward(rast, sc, poses, mask)
    P, recs, pix, out = oracle_forward(cam, sc, poses, mask)
    kap = footprint_condition(recs)[0]
    kap = kap[np.isfinite(kap)]
    e = compare_forward(g, pix, out, recs)
    gC, gD = random_upstream(mask, seed=41)
    grads = rast.alloc_grads()
    C, D, T, I = g["tensors"]
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), D, T, I,
                       torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    ref, gbnd = oracle_grads(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x])
    e.update(grad_stats(grads, ref, sc["unstable"], gbnd))
    print("needle band 1e%d: kappa %.1e..%.1e (median %.1e), %d pixels with a list" %
          (band, kap.min(), kap.max(), np.median(kap), int((out["nlist"] > 0).sum())), fmt_stats(e), flush=True)
    assert e["index_mismatch"] == 0
    assert_parity(e)


# ------------------------------------------------------------ forward values

def test_forward_parity_c1():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    rast = _rast(cam, len(sc["pos"]), 1)
    g = gpu_forward(rast, sc, poses, mask)
    _, recs, pix, out = oracle_forward(cam, sc, poses, mask)
    e = compare_forward(g, pix, out, recs)
    print("c1 forward errors", fmt_stats(e))
    assert e["index_mismatch"] == 0
    assert_parity(e)


def test_forward_masked_ragged_two_frames():
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(3, n=2000)
    rng = np.random.default_rng(4)
    mask = (rng.random((2, 75, 100)) < 0.15).astype(np.uint8)
    rast = _rast(cam, len(sc["pos"]), 2)
    g = gpu_forward(rast, sc, poses, mask)
    _, recs, pix, out = oracle_forward(cam, sc, poses, mask)
    e = compare_forward(g, pix, out, recs)
    print("ragged masked errors", fmt_stats(e))
    assert e["index_mismatch"] == 0
    assert_parity(e)
    # unmasked pixels keep the caller's prefill
    off = mask == 0
    assert (g["color"][off] == 0).all() and (g["trans"][off] == 1).all()
    assert (g["depth"][off] == -1).all() and (g["index"][off] == -1).all()


def test_forward_bit_identical_across_tiles_and_queue_granularity():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    rng = np.random.default_rng(5)
    mask = (rng.random((1, cam["height"], cam["width"])) < 0.5).astype(np.uint8)
    ref = None
    for tile in [(16, 16), (8, 8), (32, 8)]:
        # (items_per_pop, static_share, forward's own items_per_pop and share)
        for sched in ((0, 0, -1, -1), (1, 0, -1, -1), (3, 0, -1, -1), (2, 50, 4, 50), (0, 0, 2, 30)):
            rast = _rast(cam, len(sc["pos"]), 1, tile_w=tile[0], tile_h=tile[1], items_per_pop=sched[0],
                         static_share=sched[1], fwd_items_per_pop=sched[2], fwd_static_share=sched[3])
            g = gpu_forward(rast, sc, poses, mask)
            cur = [g[k] for k in ("color", "depth", "trans", "index")]
            if ref is None:
                ref = cur
            else:
                for a, b in zip(cur, ref):
                    assert np.array_equal(a.view(np.uint32) if a.dtype != np.int32 else a,
                                          b.view(np.uint32) if b.dtype != np.int32 else b)


@pytest.mark.parametrize("lanes,tile", [(4, (16, 16)), (32, (16, 16)), (32, (8, 8)), (8, (32, 8))])
def test_straggler_path_is_bit_identical(lanes, tile):
    """The forward compositing kernel switches a pack's last few live
    pixels to the straggler path (each walks the rest of its list alone,
    one entry per lane); with the switch forced early (any remaining entry)
    the render equals that of the pack path bit for bit, the gradients
    (whose backward reads the render's per-pixel list ends) equal its
    gradients up to the order of the float atomic sums, and both match the
    oracle."""
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(41, n=4000)
    rng = np.random.default_rng(42)
    mask = (rng.random((2, 75, 100)) < 0.5).astype(np.uint8)
    N = len(sc["pos"])
    kw = dict(tile_w=tile[0], tile_h=tile[1])
    runs = []
    for sl in (0, lanes):
        rast = _rast(cam, N, 2, straggler_lanes=sl, straggler_rest=1, **kw)
        g = gpu_forward(rast, sc, poses, mask)
        gC, gD = random_upstream(mask, seed=43)
        grads = rast.alloc_grads()
        C, D, T, I = g["tensors"]
        rast.backward_into(g["ws"], g["params"], dev_poses(poses), D, T, I, torch.as_tensor(gC).cuda(),
                           torch.as_tensor(gD).cuda(), grads)
        torch.cuda.synchronize()
        runs.append((g, [grads[k].cpu().numpy() for k in sorted(grads)]))
    (g0, gr0), (g1, gr1) = runs
    for k in ("color", "depth", "trans", "index"):
        a, b = g0[k], g1[k]
        assert np.array_equal(a.view(np.uint32) if a.dtype != np.int32 else a,
                              b.view(np.uint32) if b.dtype != np.int32 else b), k
    for a, b in zip(gr0, gr1):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * (np.abs(a).max() + 1e-30))
    _, recs, pix, out = oracle_forward(cam, sc, poses, mask, tile=tile)
    e = compare_forward(g1, pix, out, recs)
    assert e["index_mismatch"] == 0
    assert_parity(e)
    errs = _grad_parity(cam, sc, poses, mask, seed=43, straggler_lanes=lanes, straggler_rest=1, **kw)
    print("straggler path gradient errors", lanes, tile, fmt_stats(errs))
    assert_parity(errs)


@pytest.mark.parametrize("cap", [64, 1, 200])
def test_long_list_sort_path_matches_lds_path(cap):
    """Lists above sort_cap are sorted in LDS runs of a power of two >= 2 cap
    (>= 64) and merged; the pair lists must equal the one-pass LDS sort's."""
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    r1, r2 = _rast(cam, len(sc["pos"]), 1), _rast(cam, len(sc["pos"]), 1, sort_cap=cap)
    g1 = gpu_forward(r1, sc, poses, mask)
    g2 = gpu_forward(r2, sc, poses, mask)
    assert g2["status"]["big_tiles"] > 0 and g1["status"]["big_tiles"] == 0
    K = g1["status"]["pairs"]
    assert g2["status"]["pairs"] == K
    p1 = ws_view(r1, g1["ws"], "pairs", torch.int32, K).cpu().numpy()
    p2 = ws_view(r2, g2["ws"], "pairs", torch.int32, K).cpu().numpy()
    assert np.array_equal(p1, p2)
    for k in ("color", "depth", "trans", "index"):
        assert np.array_equal(g1[k], g2[k])


def test_long_list_sort_with_tight_capacity():
    """With the pair capacity equal to the pair count the long-list sort runs
    on its smallest grid (capacity / (sort_cap + 1) + 1 workgroups); every
    listed tile is still sorted."""
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    r1 = _rast(cam, len(sc["pos"]), 1)
    g1 = gpu_forward(r1, sc, poses, mask)
    K = g1["status"]["pairs"]
    r2 = _rast(cam, len(sc["pos"]), 1, max_pairs=K, sort_cap=64)
    g2 = gpu_forward(r2, sc, poses, mask)
    assert g2["status"]["big_tiles"] > 0 and not g2["status"]["overflow"] and g2["status"]["pairs"] == K
    p1 = ws_view(r1, g1["ws"], "pairs", torch.int32, K).cpu().numpy()
    p2 = ws_view(r2, g2["ws"], "pairs", torch.int32, K).cpu().numpy()
    assert np.array_equal(p1, p2)
    for k in ("color", "depth", "trans", "index"):
        assert np.array_equal(g1[k], g2[k])


@pytest.mark.parametrize("cap", [0, 100])
def test_sort_paths_bit_exact(cap):
    """Per-tile lists from 1 to ~730 pairs: with the default cap the one-wave
    rank sort (<= 64 and <= 256 keys) and the workgroup LDS bitonic sort
    both run; with cap 100 every list above it takes the run sort (bitonic over 1024
    threads) plus merge rounds.  The lists must equal the oracle's."""
    cam = small_cam(96, 72, 80.0)
    sc, poses = _two_pose_scene(3, n=3000)
    F, N = poses.shape[0], len(sc["pos"])
    mask = np.ones((F, 72, 96), np.uint8)
    rast = _rast(cam, N, F, tile_w=16, tile_h=16, **({"sort_cap": cap} if cap else {}))
    g = gpu_forward(rast, sc, poses, mask)
    P = orc.make_params(cam, tile=(16, 16))
    recs = orc.project(P, sc, poses)
    nt = 6 * 5   # 16x16 tiles over 96x72
    ws = g["ws"]
    tend = ws_view(rast, ws, "tile_end", torch.int32, F * nt).cpu().numpy()
    tstart = ws_view(rast, ws, "tile_start", torch.int32, F * nt).cpu().numpy()
    n = tend - tstart
    if cap:
        assert g["status"]["big_tiles"] > 0 and n.max() > 2 * 256
    else:
        assert g["status"]["big_tiles"] == 0
        assert ((n > 64) & (n <= 256)).any() and (n > 256).any() and ((n > 0) & (n <= 64)).any()
    _check_pairs(rast, ws, P, recs, mask, F, N, g)


@pytest.mark.parametrize("cap", [0, 400, 1000])
def test_register_sort_sizes_bit_exact(cap):
    """A dense two-frame scene, per-tile lists from a few to ~4800 pairs.
    Default cap: the one-wave rank sort, LDS steps at 512 keys, the
    register-resident bitonic sort at 1024, 2048 and 4096 keys, and lists
    above 4096 as 4096-key run sorts plus a merge.  Caps 400 and 1000: run
    sorts of 1024 and 2048 keys (the power of two >= 2 cap) plus merges.
    The lists must equal the oracle's."""
    cam = small_cam(96, 72, 80.0)
    sc, poses = _two_pose_scene(3, n=20000)
    F, N = poses.shape[0], len(sc["pos"])
    mask = np.ones((F, 72, 96), np.uint8)
    rast = _rast(cam, N, F, tile_w=16, tile_h=16, **({"sort_cap": cap} if cap else {}))
    g = gpu_forward(rast, sc, poses, mask)
    P = orc.make_params(cam, tile=(16, 16))
    recs = orc.project(P, sc, poses)
    nt = 6 * 5
    ws = g["ws"]
    tend = ws_view(rast, ws, "tile_end", torch.int32, F * nt).cpu().numpy()
    tstart = ws_view(rast, ws, "tile_start", torch.int32, F * nt).cpu().numpy()
    n = tend - tstart
    for lo, hi in ((0, 256), (256, 512), (512, 1024), (1024, 2048), (2048, 4096), (4096, 1 << 30)):
        assert ((n > lo) & (n <= hi)).any(), (lo, hi)
    assert g["status"]["big_tiles"] > 0
    _check_pairs(rast, ws, P, recs, mask, F, N, g)


@pytest.mark.parametrize("cap", [0, 100])
def test_tile_ranges_over_many_chunks(cap):
    """Eight frames of 40 x 30 tiles (9,600 (frame, tile)s, three chunks of
    4096, so the chunk-parallel range and item pass runs), with and without
    long lists: pair lists equal the oracle's, the item count is that of the
    packs, and the render is bit-identical to the frames rendered one plan
    each (one chunk)."""
    cam = small_cam(320, 240, 280.0)
    rng = np.random.default_rng(33)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    F = 8
    poses = np.stack([look_at(tg + 0.05 * k * Rg[:, 0], target, up=-Rg[:, 1]) for k in range(F)])
    sc = random_scene(rng, 4000, centre=target, spread=0.6)
    N = len(sc["pos"])
    mask = (rng.random((F, 240, 320)) < rng.uniform(0.2, 0.9, (F, 1, 1))).astype(np.uint8)
    kw = dict(tile_w=8, tile_h=8, **({"sort_cap": cap} if cap else {}))
    rast = _rast(cam, N, F, **kw)
    g = gpu_forward(rast, sc, poses, mask)
    P = orc.make_params(cam, tile=(8, 8))
    recs = orc.project(P, sc, poses)
    _check_pairs(rast, g["ws"], P, recs, mask, F, N, g)
    npx = mask.reshape(F, 30, 8, 40, 8).sum((2, 4))
    assert g["status"]["items"] == int(((npx + 63) // 64).sum())
    assert g["status"]["pixels"] == int(mask.sum())
    if cap:
        assert g["status"]["big_tiles"] > 0
    for f in range(F):
        r1 = _rast(cam, N, 1, **kw)
        g1 = gpu_forward(r1, sc, poses[f:f + 1], mask[f:f + 1])
        for k in ("color", "depth", "trans", "index"):
            assert np.array_equal(g[k][f], g1[k][0]), (f, k)


def test_pair_staging_overflow_gives_the_same_lists():
    """The counting pass stages every pair it finds; a binning block whose
    staging region overflows enumerates its pairs a second time instead.
    With the default capacity nothing falls back; with regions of one entry
    every block with a pair does, and with regions of the median block's
    pair count only the blocks above it (both paths in one binning).  The
    pair lists equal the oracle's and the renders are bit-identical.  Here
    every binning block (256 Gaussians of one frame) has a region of its
    own."""
    W, H = 400, 300
    cam = small_cam(W, H, 90.0 * W / 100.0)
    sc, poses = _two_pose_scene(1, n=1200)
    F, N = poses.shape[0], len(sc["pos"])
    rng = np.random.default_rng(2)
    mask = (rng.random((F, H, W)) < 0.3).astype(np.uint8)
    P = orc.make_params(cam, tile=(8, 8))
    recs = orc.project(P, sc, poses)
    b = orc.bin_pairs(P, recs, mask)
    per_block = np.bincount(b["frame"] * 5 + b["gid"] // 256, minlength=F * 5)
    with_pairs = int((per_block > 0).sum())
    med = int(np.median(per_block))
    above = int((per_block > med).sum())
    assert 0 < above < with_pairs
    ref = None
    restaged = {}
    for cap in (0, 1, med):
        rast = _rast(cam, N, F, tile_w=8, tile_h=8, **({"stage_cap": cap} if cap else {}))
        g = gpu_forward(rast, sc, poses, mask)
        restaged[cap] = g["status"]["restaged_blocks"]
        _check_pairs(rast, g["ws"], P, recs, mask, F, N, g)
        if ref is None:
            ref = g
        else:
            for k in ("color", "depth", "trans", "index"):
                assert np.array_equal(ref[k], g[k]), (cap, k)
    assert restaged == {0: 0, 1: with_pairs, med: above}, restaged


# ------------------------------------------------------------ edge cases

def test_empty_mask_and_all_culled():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    rast = _rast(cam, len(sc["pos"]), 1)
    g = gpu_forward(rast, sc, poses, np.zeros((1, cam["height"], cam["width"]), np.uint8))
    assert g["status"]["pixels"] == 0 and g["status"]["pairs"] == 0 and g["status"]["items"] == 0
    assert (g["trans"] == 1).all() and (g["index"] == -1).all()
    behind = dict(sc)
    behind["pos"] = sc["pos"] * np.array([1, 1, -1], np.float32)
    g = gpu_forward(rast, behind, poses, np.ones((1, cam["height"], cam["width"]), np.uint8))
    assert g["status"]["pairs"] == 0 and g["status"]["pixels"] == cam["width"] * cam["height"]
    assert (g["trans"] == 1).all() and (g["depth"] == -1).all() and (g["color"] == 0).all()


def test_zero_gaussians():
    cam = small_cam(40, 30, 40.0)
    from tests.scenes_small import scene_from
    sc = scene_from(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0), np.zeros((0, 3)))
    rast = _rast(cam, 0, 1)
    g = gpu_forward(rast, sc, identity_pose(), np.ones((1, 30, 40), np.uint8))
    assert g["status"]["pairs"] == 0 and (g["trans"] == 1).all()


def test_pair_capacity_overflow_reports_and_renders_nothing():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    rast = _rast(cam, len(sc["pos"]), 1, max_pairs=100)
    g = gpu_forward(rast, sc, poses, np.ones((1, cam["height"], cam["width"]), np.uint8))
    from paper_2404_19706_amd._lib import RTG_E_CAPACITY
    assert g["status"]["status"] == RTG_E_CAPACITY and g["status"]["overflow"] == 1
    assert g["status"]["items"] == 0
    # every tile's pair range is left empty, so the sorts have nothing to do
    tw, th = rast.cfg.tile_w, rast.cfg.tile_h
    nt = -(-cam["width"] // tw) * -(-cam["height"] // th)
    tend = ws_view(rast, g["ws"], "tile_end", torch.int32, nt).cpu().numpy()
    tstart = ws_view(rast, g["ws"], "tile_start", torch.int32, nt).cpu().numpy()
    assert (tend == tstart).all()
    assert (g["trans"] == 1).all() and (g["index"] == -1).all()


def test_invalid_arguments_are_rejected_on_the_host():
    from paper_2404_19706_amd import RtgError
    cam = small_cam(40, 30, 40.0)
    with pytest.raises(RtgError):
        _rast(cam, 10, 1, tile_w=12, tile_h=12)
    with pytest.raises(RtgError):
        _rast(cam, 10, 33)
    rast = _rast(cam, 10, 1)
    ws = rast.new_workspace()
    from paper_2404_19706_amd._lib import lib as L, RTG_E_INVALID
    import ctypes
    assert L().rtg_bin(rast._plan, ctypes.c_void_p(ws.data_ptr() + 1), ctypes.c_void_p(ws.data_ptr()),
                       None) == RTG_E_INVALID
    assert L().rtg_render(rast._plan, ctypes.c_void_p(ws.data_ptr()), None, None, None, None, None) == RTG_E_INVALID


# ------------------------------------------------------------ M_unstable

def test_unstable_mask_bit_exact():
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(6, n=1500)
    rast = _rast(cam, len(sc["pos"]), 2)
    m = rast.unstable_mask(dev_params(sc), dev_poses(poses)).cpu().numpy()
    P = orc.make_params(cam)
    recs = orc.project(P, sc, poses)
    ref = orc.unstable_mask_image(P, recs, sc["unstable"])
    assert 0.05 < ref.mean() < 0.95
    assert np.array_equal(m, ref)


def test_filter50_renders_the_filtered_pixel_set():
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(7, n=800)
    rng = np.random.default_rng(8)
    mask = (rng.random((2, 75, 100)) < rng.uniform(0.3, 0.7, (2, 1, 1))).astype(np.uint8)
    rast = _rast(cam, len(sc["pos"]), 2, tile_filter50=1)
    g = gpu_forward(rast, sc, poses, mask)
    eff = orc.filter50(orc.make_params(cam), mask)
    assert 0 < eff.sum() < mask.sum()
    assert g["status"]["pixels"] == int(eff.sum())
    assert np.array_equal(g["index"] != -1, (g["index"] != -1) & (eff != 0))
    assert (g["trans"][eff == 0] == 1).all()


# ------------------------------------------------------------ backward

def _grad_parity(cam, sc, poses, mask, seed, **kw):
    N, F = len(sc["pos"]), poses.shape[0]
    rast = _rast(cam, N, F, **kw)
    g = gpu_forward(rast, sc, poses, mask)
    gC, gD = random_upstream(mask, seed=seed)
    grads = rast.alloc_grads()
    C, D, T, I = g["tensors"]
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), D, T, I,
                       torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    P, recs, pix, out = oracle_forward(cam, sc, poses, mask)
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    ref, gbnd = oracle_grads(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x])
    return grad_stats(grads, ref, sc["unstable"], gbnd)


def test_backward_parity_single_frame():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], dict(cfg["scene"]), cfg["poses"]
    sc["unstable"] = (np.random.default_rng(9).random(len(sc["pos"])) < 0.5).astype(np.uint8)
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    errs = _grad_parity(cam, sc, poses, mask, seed=10)
    print("c1 gradient errors", fmt_stats(errs))
    assert_parity(errs)


def test_backward_parity_masked_two_frames_ragged():
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(11, n=1500)
    rng = np.random.default_rng(12)
    mask = (rng.random((2, 75, 100)) < 0.4).astype(np.uint8)
    errs = _grad_parity(cam, sc, poses, mask, seed=13, tile_w=8, tile_h=8)
    print("ragged two-frame gradient errors", fmt_stats(errs))
    assert_parity(errs)


def test_autograd_function_matches_direct_calls():
    from paper_2404_19706_amd import rasterize_masked
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    rast = _rast(cam, len(sc["pos"]), 1)
    params = [p.clone().requires_grad_(True) if p.dtype == torch.float32 else p for p in dev_params(sc)]
    C, D, T, I = rasterize_masked(*params, dev_poses(poses), dev_mask(mask), rast)
    gC, gD = random_upstream(mask, seed=14)
    (C * torch.as_tensor(gC).cuda()).sum().add((D * torch.as_tensor(gD).cuda()).sum()).backward()
    g = gpu_forward(rast, sc, poses, mask)
    grads = rast.alloc_grads()
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), *g["tensors"][1:],
                       torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda(), grads)
    for p, k in zip(params[:5], ("pos", "scale", "rot", "opacity", "color")):
        assert rel_err(p.grad.cpu().numpy(), grads[k].cpu().numpy()) < 1e-6


# ------------------------------------------------------------ harness

def test_l1_loss_and_upstream_match_oracle():
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
    rng = np.random.default_rng(15)
    mask = (rng.random((1, cam["height"], cam["width"])) < 0.6).astype(np.uint8)
    rast = _rast(cam, len(sc["pos"]), 1)
    g = gpu_forward(rast, sc, poses, mask)
    C, D, T, I = g["tensors"]
    Cgt = torch.rand_like(C)
    Dgt = torch.where(torch.rand_like(D) < 0.1, torch.zeros_like(D), torch.rand_like(D) * 3)
    dC = torch.zeros_like(C)
    dD = torch.zeros_like(D)
    loss = torch.zeros(1, device="cuda")
    rast.loss_l1_into(g["ws"], C, D, Cgt, Dgt, dC, dD, loss)
    gc_ref, gd_ref, l_ref = orc.l1_upstream(C.cpu().numpy(), D.cpu().numpy(), Cgt.cpu().numpy(),
                                            Dgt.cpu().numpy(), mask)
    assert rel_err(dC.cpu().numpy(), gc_ref) < 1e-6
    assert rel_err(dD.cpu().numpy(), gd_ref) < 1e-6
    assert abs(float(loss) - l_ref) < 1e-5 * max(1.0, l_ref)


@pytest.mark.parametrize("tile,ipp", [((16, 16), 0), ((32, 8), 1)])
def test_fused_l1_backward_equals_separate_calls(tile, ipp):
    """rtg_backward_raster_l1 + rtg_backward_project_l1 give the loss value
    and parameter gradients of rtg_loss_l1 + rtg_backward_raster +
    rtg_backward_project up to float summation order; two frames, ragged
    masks, targets with invalid depths, weights other than one; twice in a
    row on the same projection (the per-wave sums are rewritten)."""
    cam = small_cam(100, 75, 90.0)
    sc, poses = _two_pose_scene(5, n=1500)
    rng = np.random.default_rng(16)
    mask = (rng.random((2, 75, 100)) < 0.5).astype(np.uint8)
    rast = _rast(cam, len(sc["pos"]), 2, tile_w=tile[0], tile_h=tile[1], items_per_pop=ipp)
    g = gpu_forward(rast, sc, poses, mask)
    C, D, T, I = g["tensors"]
    ws, params, dp = g["ws"], g["params"], dev_poses(poses)
    Cgt = torch.rand_like(C)
    Dgt = torch.where(torch.rand_like(D) < 0.1, torch.zeros_like(D), torch.rand_like(D) * 3)
    w_c, w_d = 0.7, 0.3
    dC, dD = torch.zeros_like(C), torch.zeros_like(D)
    loss_a = torch.zeros(1, device="cuda")
    rast.loss_l1_into(ws, C, D, Cgt, Dgt, dC, dD, loss_a, w_c=w_c, w_d=w_d)
    rast.backward_raster(ws, D, T, I, dC, dD)
    ga = rast.alloc_grads()
    rast.backward_project(ws, params, dp, ga)
    for _ in range(2):
        loss_b = torch.zeros(1, device="cuda")
        rast.backward_raster_l1(ws, C, D, T, I, Cgt, Dgt)
        gb = rast.alloc_grads()
        rast.backward_project_l1(ws, params, dp, gb, loss_b, w_c=w_c, w_d=w_d)
        torch.cuda.synchronize()
        assert abs(float(loss_b) - float(loss_a)) <= 1e-6 * abs(float(loss_a))
        # the scales enter after the float accumulation instead of before:
        # a few binary32 roundings per sum
        for k in ga:
            assert torch.count_nonzero(ga[k]) > 0, k
            assert rel_err(gb[k].cpu().numpy(), ga[k].cpu().numpy()) <= 1e-5, k


def test_adam_matches_oracle():
    from paper_2404_19706_amd import Rasterizer
    cam = small_cam(40, 30, 40.0)
    n = 300
    rng = np.random.default_rng(16)
    sc = random_scene(rng, n, unstable_frac=0.5)
    rast = Rasterizer(cam, n, 1)
    params = [p.clone() for p in dev_params(sc)]
    m = torch.zeros((n, 13), device="cuda")
    v = torch.zeros((n, 13), device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    lr = (1e-3, 2e-3, 1e-3, 1e-3)
    ref = {"pos": sc["pos"].astype(np.float64), "logs": np.log(sc["scale"].astype(np.float64)),
           "rot": sc["rot"].astype(np.float64), "color": sc["color"].astype(np.float64)}
    st = {k: (np.zeros_like(x), np.zeros_like(x)) for k, x in ref.items()}
    un = sc["unstable"]
    for it in range(1, 4):
        grads = {k: torch.as_tensor(rng.standard_normal(s).astype(np.float32)).cuda()
                 for k, s in (("pos", (n, 3)), ("scale", (n, 3)), ("rot", (n, 4)), ("color", (n, 3)))}
        s_now = params[1].cpu().numpy().astype(np.float64)
        rast.adam(params, grads, m, v, step, lr=lr, eps=1e-15)
        for k, lrk, gk in (("pos", lr[0], grads["pos"].cpu().numpy()),
                           ("logs", lr[1], s_now * grads["scale"].cpu().numpy()),
                           ("rot", lr[2], grads["rot"].cpu().numpy()),
                           ("color", lr[3], grads["color"].cpu().numpy())):
            ref[k], mm, vv = orc.adam_step(ref[k], gk, st[k][0], st[k][1], it, lrk, un, eps=1e-15)
            st[k] = (mm, vv)
    assert int(step.item()) == 3
    assert np.allclose(params[0].cpu().numpy(), ref["pos"], rtol=1e-5, atol=1e-6)
    assert np.allclose(params[1].cpu().numpy(), np.exp(ref["logs"]), rtol=1e-5, atol=1e-7)
    assert np.allclose(params[2].cpu().numpy(), ref["rot"], rtol=1e-5, atol=1e-6)
    assert np.allclose(params[4].cpu().numpy(), ref["color"], rtol=1e-5, atol=1e-6)
    assert np.array_equal(params[3].cpu().numpy(), sc["opacity"])


# ------------------------------------------------------------ binning bounds

def _gpu_pair_set(rast, ws, F, N, nt, K):
    tend = ws_view(rast, ws, "tile_end", torch.int32, F * nt).cpu().numpy().astype(np.int64)
    start = ws_view(rast, ws, "tile_start", torch.int32, F * nt).cpu().numpy().astype(np.int64)
    pairs = ws_view(rast, ws, "pairs", torch.int32, K).cpu().numpy().astype(np.int64)
    cnt = tend - start
    ft = np.repeat(np.arange(F * nt), cnt)
    pos = np.concatenate([np.arange(s, e) for s, e in zip(start, tend) if e > s]) if K else np.zeros(0, np.int64)
    gid = pairs[pos] - (ft // nt) * N
    return set((ft * N + gid).tolist())


@pytest.mark.parametrize("case,tile", [("c1", (16, 16)), ("ragged", (8, 8)), ("ragged", (32, 8)),
                                       ("edge_on", (16, 16))])
def test_pair_lists_lie_between_the_needed_and_the_plain_pairs(case, tile):
    """Independent of the pair-thinning rule both sides implement: every
    (frame, tile, Gaussian) pair the GPU bins is one the paper's plain rule
    would bin (the Gaussian's rectangle covers the tile, the tile has a
    masked pixel), and every pair a pixel needs (the Gaussian is in the list
    L(u) of a masked pixel u of that tile, from the oracle) is binned."""
    if case == "c1":
        cfg = make_config("c1")
        cam, sc, poses = cfg["cam"], cfg["scene"], cfg["poses"]
        mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    elif case == "ragged":
        cam = small_cam(100, 75, 90.0)
        sc, poses = _two_pose_scene(21, n=1500)
        mask = (np.random.default_rng(22).random((2, 75, 100)) < 0.3).astype(np.uint8)
    else:
        cam = small_cam()
        sc = edge_on_surfels(np.random.default_rng(23), 400)
        poses = identity_pose()
        mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    F, N = poses.shape[0], len(sc["pos"])
    rast = _rast(cam, N, F, tile_w=tile[0], tile_h=tile[1])
    g = gpu_forward(rast, sc, poses, mask)
    tw, th = tile
    tx, ty = -(-cam["width"] // tw), -(-cam["height"] // th)
    nt = tx * ty
    got = _gpu_pair_set(rast, g["ws"], F, N, nt, g["status"]["pairs"])
    P, recs, pix, _ = oracle_forward(cam, sc, poses, mask, tile=tile)
    # plain rule: rectangle tiles with a masked pixel
    act = np.zeros((F, ty, tx), bool)
    f_, x_, y_ = pix[:, 0], pix[:, 1], pix[:, 2]
    act[f_, y_ // th, x_ // tw] = True
    plain = set()
    for f in range(F):
        vis = np.nonzero(recs["visible"][f])[0]
        for i in vis:
            x0, x1, y0, y1 = recs["rect"][f, i]
            for b in range(y0 // th, y1 // th + 1):
                for a in range(x0 // tw, x1 // tw + 1):
                    if act[f, b, a]:
                        plain.add((f * nt + b * tx + a) * N + int(i))
    need = set()
    for (f, x, y), L in zip(pix, orc.pixel_lists(P, recs, pix)):
        base = (int(f) * nt + (int(y) // th) * tx + int(x) // tw) * N
        need.update((base + L.astype(np.int64)).tolist())
    print(case, tile, "needed", len(need), "binned", len(got), "plain", len(plain), flush=True)
    assert need <= got, len(need - got)
    assert got <= plain, len(got - plain)
    assert len(got) < len(plain) or case == "c1"


# ------------------------------------------------------------ FP32 forward sanity

def test_gpu_gradients_against_finite_differences_of_the_gpu_forward():
    """Loose sanity check of the GPU's own FP32 forward: central differences
    (steps of ~1e-3 of each parameter) of sum(gC . C) + sum(gD . D) rendered
    on the GPU against the GPU's analytic gradient, for 60 random parameter
    entries whose perturbation flips no discrete decision (list membership,
    clamp, depth hit, branch: the oracle's per-pixel decision signature is
    compared, as the forward is discontinuous there); within 2e-2 of the
    gradient scale of the parameter group."""
    cfg = make_config("c1")
    cam, sc, poses = cfg["cam"], dict(cfg["scene"]), cfg["poses"]
    N = len(sc["pos"])
    mask = np.ones((1, cam["height"], cam["width"]), np.uint8)
    rast = _rast(cam, N, 1)
    gC, gD = random_upstream(mask, seed=31)
    tgC, tgD = torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda()
    g = gpu_forward(rast, sc, poses, mask)
    grads = rast.alloc_grads()
    rast.backward_into(g["ws"], g["params"], dev_poses(poses), *g["tensors"][1:], tgC, tgD, grads)
    torch.cuda.synchronize()
    gnp = {k: v.cpu().numpy() for k, v in grads.items()}

    P, recs0, pix, out0 = oracle_forward(cam, sc, poses, mask)

    def loss(scn):
        o = gpu_forward(rast, scn, poses, mask)
        Cc, Dd = o["color"].astype(np.float64), o["depth"].astype(np.float64)
        sig = orc.render(P, orc.project(P, scn, poses), scn, pix)["sig"]
        return float((Cc * gC).sum() + (Dd * gD).sum()), sig

    rng = np.random.default_rng(32)
    checked, worst = 0, 0.0
    fields = [("pos", 3), ("scale", 3), ("rot", 4), ("opacity", 1), ("color", 3)]
    for name, w in fields:
        scale_g = float(np.abs(gnp[name]).max())
        tried = 0
        for i in rng.permutation(N):
            if tried >= 12:
                break
            c = int(rng.integers(w))
            x0 = float(sc[name][i] if w == 1 else sc[name][i, c])
            h = 1e-3 * max(abs(x0), 1e-2)
            vals, idxs = [], []
            for sgn in (1, -1):
                s2 = {k: v.copy() for k, v in sc.items()}
                if w == 1:
                    s2[name][i] = np.float32(x0 + sgn * h)
                else:
                    s2[name][i, c] = np.float32(x0 + sgn * h)
                l, ind = loss(s2)
                vals.append(l)
                idxs.append(ind)
            if not (np.array_equal(idxs[0], out0["sig"]) and np.array_equal(idxs[1], out0["sig"])):
                continue
            hp = float(np.float32(x0 + h)) - float(np.float32(x0 - h))
            fd = (vals[0] - vals[1]) / hp
            an = float(gnp[name][i] if w == 1 else gnp[name][i, c])
            worst = max(worst, abs(fd - an) / max(scale_g, 1e-12))
            tried += 1
            checked += 1
    print("GPU FD sanity: %d entries, worst |fd - grad| / group scale %.2e" % (checked, worst), flush=True)
    assert checked >= 40
    assert worst < 2e-2
