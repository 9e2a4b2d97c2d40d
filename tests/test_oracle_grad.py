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


# ---------------------------------------------------------------- error bounds
# orc_backward_bound: per gradient entry, gamma times the absolute-value
# chain of the summed absolute camera-space terms, plus what an early exit
# below t_eps may change.

def _bound_case(seed, n=300):
    rng = np.random.default_rng(seed)
    pose_a, Rg, tg = random_pose(rng)
    sc = random_scene(rng, n, centre=tg + 2.0 * Rg[:, 2], spread=0.5, unstable_frac=0.7)
    poses = pose_a[None]
    P = orc.make_params(CAM)
    pix = all_pixels(1, H, W)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    return P, sc, poses, pix, gC, gD


def test_bound_dominates_the_gradient_at_unit_gamma():
    """With gamma = 1 every term may be off by 100 %, so the bound is at least
    |gradient| entry by entry (|sum t| <= sum |t|, |A x| <= |A| |x|): a term or
    coefficient missing from the absolute chain fails this."""
    P, sc, poses, pix, gC, gD = _bound_case(21)
    recs = orc.project(P, sc, poses)
    g, b = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(1.0, 0.0, np.inf))
    g0 = orc.backward(P, recs, sc, poses, pix, gC, gD)
    for k in g:
        assert np.array_equal(g[k], g0[k])
        assert np.all(b[k] >= np.abs(g[k]) * (1 - 1e-12)), k
        assert np.all(b[k][sc["unstable"] == 0] == 0)
    assert max(float(np.abs(b[k]).max()) for k in b) > 0


def test_bound_grows_with_gamma_and_early_exit():
    """More base error per term or a larger early-exit threshold can only
    widen the bound; with neither, what remains is the error model's own
    part (binary32 f, its amplification along the list), a small fraction of
    the unit-gamma bound."""
    P, sc, poses, pix, gC, gD = _bound_case(22)
    recs = orc.project(P, sc, poses)
    _, b1 = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(1.0, 0.0, np.inf))
    _, b3 = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(3e-6, 0.0, np.inf))
    _, bt = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(3e-6, 1e-3, np.inf))
    _, b0 = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(0.0, 0.0, np.inf))
    for k in b1:
        assert np.all(b0[k] <= b3[k]) and np.all(b3[k] <= bt[k]) and np.all(b3[k] <= b1[k])
        assert np.all(b0[k] <= 1e-3 * b1[k] + 1e-300)


@pytest.mark.parametrize("stop", [1, 3, 4, 6])
def test_bound_covers_an_early_exit(stop):
    """One pixel looking through a stack of near-opaque Gaussians: stopping
    the compositing once T < t_eps is the same as removing the Gaussians
    behind the stop from that pixel.  The gradient of the truncated stack
    (the oracle on the scene without them) differs from the full one by at
    most the bound's early-exit part (gamma = 0), entry by entry, and the
    dropped Gaussians' gradients are within it too."""
    n = 9
    z = 1.5 + 0.05 * np.arange(n)
    pos = np.stack([np.full(n, 0.002), np.full(n, -0.001), z], 1)
    rng = np.random.default_rng(23)
    sc = {"pos": pos.astype(np.float32), "scale": np.full((n, 3), 0.03, np.float32),
          "rot": np.tile(np.array([1.0, 0.0, 0.0, 0.0], np.float32), (n, 1)),
          "opacity": rng.uniform(0.9, 0.98, n).astype(np.float32),
          "color": rng.random((n, 3)).astype(np.float32), "unstable": np.ones(n, np.uint8)}
    poses = identity_pose()
    P = orc.make_params(CAM)
    pix = np.array([[0, W // 2, H // 2]], np.int32)
    gC = rng.standard_normal((1, 3))
    gD = np.zeros(1)
    recs = orc.project(P, sc, poses)
    ref = orc.render(P, recs, sc, pix)
    assert ref["nlist"][0] == n
    # transmission in front of each entry (list order = depth order here)
    f = []
    for i in range(n):
        sub = {k: v[i:i + 1] for k, v in sc.items()}
        f.append(1.0 - orc.render(P, orc.project(P, sub, poses), sub, pix)["trans"][0])
    Tk = np.concatenate([[1.0], np.cumprod(1.0 - np.array(f))])[:-1]
    # entries 0..stop blended
    t_eps = np.sqrt(Tk[stop] * Tk[stop + 1])    # T falls below it after entry `stop`
    assert Tk[stop + 1] < t_eps <= Tk[stop]
    g_full, b = orc.backward(P, recs, sc, poses, pix, gC, gD, bound=(0.0, t_eps, np.inf))
    keep = {k: v[:stop + 1] for k, v in sc.items()}
    rk = orc.project(P, keep, poses)
    g_tr = orc.backward(P, rk, keep, poses, pix, gC, gD)
    for k in g_full:
        full = g_full[k]
        trunc = np.zeros_like(full)
        trunc[:stop + 1] = g_tr[k]
        diff = np.abs(full - trunc)
        assert np.all(diff <= b[k] * (1 + 1e-9) + 1e-300), (k, diff, b[k])
        assert np.abs(b[k]).max() > 0
