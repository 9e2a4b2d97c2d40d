"""Pins of the oracle's backward pass: central finite differences of its own
FP64 forward (pinned above by closed forms), on every parameter whose
perturbation flips no discrete decision; plus the harness references
(L1 upstream gradients, Adam) against torch's CPU autograd and optimiser."""
import numpy as np
import pytest
import torch

from oracle import oracle as orc
from tests.scenes_small import all_pixels, identity_pose, random_pose, random_scene, small_cam

CAM = small_cam(40, 30, 40.0)
H, W = CAM["height"], CAM["width"]


def _loss(P, sc, poses, pix, gC, gD):
    recs = orc.project(P, sc, poses)
    out = orc.render(P, recs, sc, pix)
    return float((out["color"] * gC).sum() + (out["depth"] * gD).sum()), out["sig"]


def _fd_check(sc, poses, seed, n_check=40, tol=2e-6):
    rng = np.random.default_rng(seed)
    P = orc.make_params(CAM)
    F = poses.shape[0]
    pix = all_pixels(F, H, W)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    recs = orc.project(P, sc, poses)
    grads = orc.backward(P, recs, sc, poses, pix, gC, gD)
    N = len(sc["pos"])
    fields = [("pos", 3), ("scale", 3), ("rot", 4), ("opacity", 1), ("color", 3)]
    checked = {k: 0 for k, _ in fields}
    base_scale = {k: np.abs(grads[k]).max() for k, _ in fields}
    for name, width in fields:
        cand = [(i, c) for i in range(N) for c in range(width) if sc["unstable"][i]]
        rng.shuffle(cand)
        for i, c in cand:
            if checked[name] >= n_check:
                break
            # float64 copies so that +-h is exact
            p = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in sc.items()}
            x0 = p[name][i] if width == 1 else p[name][i, c]
            h = 1e-5 * max(1.0, abs(x0)) if name != "scale" else 1e-5 * abs(x0)
            vals = []
            sigs = []
            for sgn in (+1, -1):
                q = {k: v.copy() for k, v in p.items()}
                if width == 1:
                    q[name][i] = x0 + sgn * h
                else:
                    q[name][i, c] = x0 + sgn * h
                q32 = {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in q.items()}
                # the perturbation must be exactly representable in float32
                xv = q32[name][i] if width == 1 else q32[name][i, c]
                vals.append((_loss(P, q32, poses, pix, gC, gD), float(xv)))
                sigs.append(vals[-1][0][1])
            if not np.array_equal(sigs[0], sigs[1]):
                continue
            (lp, _), xp = vals[0]
            (lm, _), xm = vals[1]
            fd = (lp - lm) / (xp - xm)
            an = grads[name][i] if width == 1 else grads[name][i, c]
            assert abs(fd - an) <= tol * (abs(an) + 1e-2 * base_scale[name] + 1e-12), (name, i, c, fd, an)
            checked[name] += 1
    return checked


def test_fd_single_frame_identity_pose():
    rng = np.random.default_rng(0)
    sc = random_scene(rng, 25, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    checked = _fd_check(sc, identity_pose(), seed=1)
    assert min(checked.values()) >= 15, checked


def test_fd_two_frames_random_poses():
    """Gradients summed over two frames with non-trivial poses."""
    rng = np.random.default_rng(2)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    pose_b = pose_a.copy()
    # second camera shifted 0.1 m sideways, looking at the same point
    from rtg_synth import look_at
    pose_b = look_at(tg + 0.1 * Rg[:, 0], target, up=-Rg[:, 1])
    sc = random_scene(rng, 25, centre=target, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    checked = _fd_check(sc, np.stack([pose_a, pose_b]), seed=3)
    assert min(checked.values()) >= 15, checked


def test_stable_rows_are_zero_and_frames_add():
    rng = np.random.default_rng(4)
    sc = random_scene(rng, 60, spread=0.3, unstable_frac=0.5)
    P = orc.make_params(CAM)
    pose2 = identity_pose()[0].copy()
    pose2[9] = 0.05
    poses = np.stack([identity_pose()[0], pose2])
    recs = orc.project(P, sc, poses)
    pix = all_pixels(2, H, W)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    g = orc.backward(P, recs, sc, poses, pix, gC, gD)
    stable = sc["unstable"] == 0
    for k in g:
        assert (g[k][stable] == 0).all()
    # batch gradient = sum of the single-frame gradients
    half = len(pix) // 2
    g0 = orc.backward(P, recs[:1], sc, poses[:1], pix[:half], gC[:half], gD[:half])
    g1 = orc.backward(P, recs[1:], sc, poses[1:], pix[half:] - np.array([1, 0, 0], np.int32), gC[half:], gD[half:])
    for k in g:
        np.testing.assert_allclose(g[k], g0[k] + g1[k], rtol=1e-10, atol=1e-13)


def test_l1_upstream_matches_torch_autograd():
    rng = np.random.default_rng(5)
    F = 2
    C = rng.random((F, H, W, 3))
    Cgt = rng.random((F, H, W, 3))
    D = np.where(rng.random((F, H, W)) < 0.2, -1.0, rng.uniform(0.5, 3, (F, H, W)))
    Dgt = np.where(rng.random((F, H, W)) < 0.1, 0.0, rng.uniform(0.5, 3, (F, H, W)))
    M = rng.random((F, H, W)) < 0.4
    gC, gD, loss = orc.l1_upstream(C, D, Cgt, Dgt, M)
    tC = torch.tensor(C, requires_grad=True)
    tD = torch.tensor(D, requires_grad=True)
    m = torch.tensor(M)
    md = m & (tD.detach() != -1) & (torch.tensor(Dgt) > 0)
    lc = (tC - torch.tensor(Cgt)).abs()[m].sum() / (3 * m.sum())
    ld = (tD - torch.tensor(Dgt)).abs()[md].sum() / md.sum()
    (lc + ld).backward()
    np.testing.assert_allclose(gC, tC.grad.numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gD, tD.grad.numpy(), rtol=1e-12, atol=1e-15)
    assert abs(loss - float(lc + ld)) < 1e-12


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(6)
    n = 50
    x = rng.standard_normal((n, 3))
    un = rng.random(n) < 0.5
    t = torch.tensor(x[un], requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = x.copy(), np.zeros_like(x), np.zeros_like(x)
    for step in range(1, 6):
        g = rng.standard_normal((n, 3))
        t.grad = torch.tensor(g[un])
        opt.step()
        p, m, v = orc.adam_step(p, g, m, v, step, 1e-3, un)
    np.testing.assert_allclose(p[un], t.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert np.array_equal(p[~un], x[~un])
