"""The no-allocation forward entry point (rtg_forward_static), called
through the C ABI, against the workspace path (rtg_project + rtg_bin +
rtg_render on a caller-allocated workspace) on the same inputs: two calls in
a row on one device, the second with a smaller problem (fewer Gaussians,
frames and pixels), so what the first call left in the shared scratch must
not leak into the second.  Forward outputs must be bit-identical and the
device status must report success."""
import ctypes

import numpy as np
import pytest
import torch

from tests.gpu_helpers import dev_mask, dev_params, dev_poses, need_gpu
from tests.scenes_small import random_pose, random_scene, small_cam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _case(seed, n, frames, w, h, max_pairs):
    from paper_2404_19706_amd import Rasterizer
    from rtg_synth import look_at
    rng = np.random.default_rng(seed)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    poses = [pose_a] + [look_at(tg + 0.1 * k * Rg[:, 0], target, up=-Rg[:, 1]) for k in range(1, frames)]
    sc = random_scene(rng, n, centre=target, spread=0.6, unstable_frac=0.5)
    cam = small_cam(w, h)
    # ragged masks: a random half of the pixels, plus one empty row band
    mask = (rng.random((frames, h, w)) < 0.5).astype(np.uint8)
    mask[:, h // 3:h // 3 + 5] = 0
    rast = Rasterizer(cam, n, frames, max_pairs=max_pairs)
    return rast, dev_params(sc), dev_poses(np.stack(poses)), dev_mask(mask)


def _static_forward(rast, params, poses, mask):
    from paper_2404_19706_amd._lib import lib
    C, D, T, I = rast.alloc_outputs()
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    st = lib().rtg_forward_static(rast._plan, *[_p(t) for t in params], _p(poses), _p(mask), _p(C), _p(D), _p(T),
                                  _p(I), _p(status), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    torch.cuda.synchronize()
    return (C, D, T, I), int(status.item())


def test_static_forward_matches_workspace_path_on_two_calls():
    from paper_2404_19706_amd._lib import STATIC_SCRATCH_BYTES
    cases = [(11, 3000, 3, 160, 120, 400_000), (12, 700, 1, 96, 64, 50_000)]
    for k, (seed, n, frames, w, h, mp) in enumerate(cases):
        rast, params, poses, mask = _case(seed, n, frames, w, h, mp)
        assert rast.ws_bytes <= STATIC_SCRATCH_BYTES
        print("static forward: case %d n=%d frames=%d %dx%d ws=%d B" % (k, n, frames, w, h, rast.ws_bytes), flush=True)
        got, status = _static_forward(rast, params, poses, mask)
        C, D, T, I, ws = rast.forward(params, poses, mask)
        torch.cuda.synchronize()
        st = rast.read_status(ws)
        assert st["status"] == 0 and status == 0, (st, status)
        assert st["pixels"] == int(mask.sum())
        for a, b in zip(got, (C, D, T, I)):
            assert torch.equal(a, b), k
        assert int((I >= 0).sum()) > 0


def test_static_forward_reports_capacity_overflow():
    """A plan whose pair capacity is too small: the call succeeds on the
    host, renders nothing, and writes RTG_E_CAPACITY to status_out."""
    rast, params, poses, mask = _case(13, 2000, 1, 128, 96, 64)
    got, status = _static_forward(rast, params, poses, mask)
    assert status == -2
    C, D, T, I = got
    assert bool((I == -1).all()) and bool((T == 1).all())
