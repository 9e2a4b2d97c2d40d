"""Parity at the benchmark workloads' full sizes, in the launch
configuration the benchmark times.

The step (projection, binning, forward, L1 loss, backward compositing,
projection backward) is built exactly as the benchmark builds it, captured
in a HIP graph and replayed; the forward outputs of the replay are then
compared, at a seeded sample of masked pixels, with the FP64 oracle computed
pixel by pixel, and the gradients of an upstream that is non-zero only at
the sampled pixels (one more backward on the same plan) with the oracle's
gradients of the same upstream.  Bar: index map exact, <= 1e-4 normwise
relative error on colour, depth, transmission and every gradient.  For the
16-keyframe workload the sample is drawn from the first two keyframes and
the oracle projects only those (the other frames get no upstream)."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from tests.gpu_helpers import need_gpu, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


@pytest.mark.parametrize("name,tile,ipp,frames", [("c1", (8, 8), 0, None), ("c2", (32, 8), 0, None),
                                                  ("c2", (16, 16), 0, None), ("c3", (32, 8), 0, None),
                                                  ("c4", (16, 16), 1, None), ("c5", (16, 16), 1, 2)])
def test_full_size_sampled_parity(name, tile, ipp, frames, n_px=1500):
    import bench
    wl = bench.build_workload(name)
    step = bench.Step(wl, tile, ipp)
    step()
    torch.cuda.synchronize()
    graph = bench.capture(step)
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    st = step.rast.read_status(step.ws)
    assert st["status"] == 0, st

    F = wl["F"] if frames is None else frames
    mask = wl["mask"].cpu().numpy()[:F]
    allpix = orc.masked_pixels(mask)
    rng = np.random.default_rng(123)
    pix = allpix[rng.choice(len(allpix), min(n_px, len(allpix)), replace=False)]
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    sc = {k: t.cpu().numpy() for k, t in zip(("pos", "scale", "rot", "opacity", "color", "unstable"),
                                              wl["params"])}
    P = orc.make_params(wl["cam"], tile=tile)
    poses = wl["poses_np"][:F]
    recs = orc.project(P, sc, poses)
    ref = orc.render(P, recs, sc, pix)
    C, D, T, I = (t.cpu().numpy() for t in (step.C, step.D, step.T, step.I))
    err = {"color": rel_err(C[f, y, x], ref["color"]), "depth": rel_err(D[f, y, x], ref["depth"]),
           "trans": rel_err(T[f, y, x], ref["trans"])}
    mism = int((I[f, y, x] != ref["index"]).sum())

    gC = np.zeros(C.shape, np.float32)
    gD = np.zeros(D.shape, np.float32)
    gC[f, y, x] = rng.standard_normal((len(pix), 3)).astype(np.float32)
    gD[f, y, x] = rng.standard_normal(len(pix)).astype(np.float32)
    grads = step.rast.alloc_grads()
    step.rast.backward_into(step.ws, wl["params"], wl["poses"], step.D, step.T, step.I,
                            torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    gref = orc.backward(P, recs, sc, poses, pix, gC[f, y, x], gD[f, y, x])
    for k in ("pos", "scale", "rot", "opacity", "color"):
        err["d_" + k] = rel_err(grads[k].cpu().numpy(), gref[k])
    print(name, tile, ipp, "pixels", len(pix), "index mismatches", mism, err)
    assert mism == 0
    assert max(err.values()) <= TOL, err


def test_captured_step_replays_match_eager():
    """The benchmark's step (projection, binning, forward, the L1 loss folded
    into both backward kernels, projection backward) captured in a HIP graph:
    every replay, with eager work and synchronisations in between, gives the
    eager step's outputs (forward bit for bit; loss and gradients up to the
    order of the float atomic accumulation)."""
    import bench
    wl = bench.build_workload("c2")
    step = bench.Step(wl, (16, 16), 0)
    step()
    torch.cuda.synchronize()
    ref_out = [t.clone() for t in (step.C, step.D, step.T, step.I)]
    ref_loss = float(step.loss)
    ref_g = {k: v.clone() for k, v in step.grads.items()}
    graph = bench.capture(step)
    for rep in range(3):
        for t in (step.C, step.D, step.T, step.I):
            t.fill_(-7)
        for v in step.grads.values():
            v.fill_(3.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(ref_out, (step.C, step.D, step.T, step.I)):
            assert torch.equal(a, b), rep
        assert abs(float(step.loss) - ref_loss) <= 1e-6 * abs(ref_loss), rep
        for k in ref_g:
            assert rel_err(step.grads[k].cpu().numpy(), ref_g[k].cpu().numpy()) <= 1e-5, (rep, k)
        step()   # eager work between the replays
        torch.cuda.synchronize()
