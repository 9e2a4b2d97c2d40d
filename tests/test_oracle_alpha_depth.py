"""Pins of the alpha-blended depth oracle (oracle/alpha_depth.py): closed
forms for one and two Gaussians on a pixel, colour / transmission / index
map unchanged from the disc mode, and central finite differences of the
alpha-blended render against its backward (positions, which move both the
footprint and z, scales and rotations)."""
import numpy as np
import pytest

from oracle import alpha_depth as ad
from oracle import oracle as orc
from tests.scenes_small import all_pixels, identity_pose, random_pose, random_scene, scene_from, small_cam


def test_one_and_two_gaussians_closed_form():
    cam = small_cam(40, 30, 40.0)
    P = orc.make_params(cam)
    # centres on the optical axis project to (20, 15): pixel (19, 14) has
    # offset (0.5, 0.5) from the centre
    sc = scene_from([[0, 0, 2.0], [0, 0, 3.0]], [[0.05, 0.05, 0.05]] * 2, [[1, 0, 0, 0]] * 2, [0.6, 0.5],
                    [[1, 0, 0], [0, 1, 0]])
    poses = identity_pose()
    pix = np.array([[0, 19, 14]], np.int32)
    for n in (1, 2):
        s = {k: v[:n] for k, v in sc.items()}
        recs = orc.project(P, s, poses)
        out = ad.render(P, recs, s, pix)
        f = []
        for i in range(n):
            z = float(s["pos"][i, 2])
            sig = 40.0 * float(s["scale"][i, 0]) / z
            f.append(float(s["opacity"][i]) * np.exp(-0.5 * (0.25 + 0.25) / sig ** 2))
        D = 2.0 * f[0] + (3.0 * f[1] * (1.0 - f[0]) if n == 2 else 0.0)
        assert out["depth"][0] == pytest.approx(D, rel=1e-9)
        assert out["trans"][0] == pytest.approx(np.prod([1 - x for x in f]), rel=1e-12)


def test_colour_transmission_index_unchanged_and_no_blend_is_minus_one():
    cam = small_cam(40, 30, 40.0)
    rng = np.random.default_rng(1)
    sc = random_scene(rng, 30, spread=0.2)
    P = orc.make_params(cam)
    poses = identity_pose()
    recs = orc.project(P, sc, poses)
    pix = all_pixels(1, 30, 40)
    a = ad.render(P, recs, sc, pix)
    b = orc.render(P, recs, sc, pix)
    for k in ("color", "trans", "index"):
        assert np.array_equal(a[k], b[k])
    assert (a["depth"][b["trans"] == 1.0] == -1).all()
    assert (a["depth"][b["trans"] < 1.0] > 0).all()


def _loss(P, sc, poses, pix, gC, gD):
    recs = orc.project(P, sc, poses)
    out = ad.render(P, recs, sc, pix)
    d = np.where(out["depth"] == -1, 0.0, out["depth"])
    return float((out["color"] * gC).sum() + (d * gD).sum()), out["sig"]


def test_alpha_depth_backward_matches_finite_differences():
    cam = small_cam(40, 30, 40.0)
    rng = np.random.default_rng(3)
    pose_a, Rg, tg = random_pose(rng)
    target = tg + 2.0 * Rg[:, 2]
    from rtg_synth import look_at
    poses = np.stack([pose_a, look_at(tg + 0.2 * Rg[:, 0], target, up=-Rg[:, 1])])
    sc = random_scene(rng, 20, centre=target, spread=0.25, smin=0.02, smax=0.1, unstable_frac=0.8)
    P = orc.make_params(cam)
    pix = all_pixels(2, 30, 40)
    gC = rng.standard_normal((len(pix), 3))
    gD = rng.standard_normal(len(pix))
    recs = orc.project(P, sc, poses)
    grads = ad.backward(P, recs, sc, poses, pix, gC, gD)
    checked = {"pos": 0, "scale": 0, "rot": 0}
    scale = {k: np.abs(grads[k]).max() for k in checked}
    for name, width in (("pos", 3), ("scale", 3), ("rot", 4)):
        idx = [i for i in range(20) if sc["unstable"][i]]
        rng.shuffle(idx)
        for i in idx:
            if checked[name] >= 12:
                break
            c = int(rng.integers(width))
            p = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in sc.items()}
            x0 = p[name][i, c]
            h = 1e-5 * max(1.0, abs(x0)) if name != "scale" else 1e-5 * abs(x0)
            vals = []
            for sgn in (+1, -1):
                q = {k: v.copy() for k, v in p.items()}
                q[name][i, c] = x0 + sgn * h
                q32 = {k: (v.astype(np.float32) if v.dtype == np.float64 else v) for k, v in q.items()}
                vals.append((_loss(P, q32, poses, pix, gC, gD), float(q32[name][i, c])))
            if not np.array_equal(vals[0][0][1], vals[1][0][1]):
                continue
            fd = (vals[0][0][0] - vals[1][0][0]) / (vals[0][1] - vals[1][1])
            an = grads[name][i, c]
            assert abs(fd - an) <= 2e-6 * (abs(an) + 1e-2 * scale[name] + 1e-12), (name, i, c, fd, an)
            checked[name] += 1
    assert min(checked.values()) >= 8, checked
