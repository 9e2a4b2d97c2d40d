"""Pins of the mapping-iteration references (oracle/optim.py): the L2
regulariser against finite differences and its zero at the initial values,
the fusion of Eq. 9 against its closed form (a running mean weighted by the
confidence counts) and its special cases, and the top-error selection
against brute force on small frames."""
import numpy as np

from oracle import optim


def _state(rng, n):
    return {"pos": rng.standard_normal((n, 3)), "rot": rng.standard_normal((n, 4)),
            "scale": rng.uniform(0.01, 0.1, (n, 3))}


def test_reg_l2_gradient_and_zero_at_init():
    rng = np.random.default_rng(0)
    n = 30
    init = _state(rng, n)
    cur = {k: v + 0.01 * rng.standard_normal(v.shape) for k, v in init.items()}
    tr = (rng.random(n) < 0.5).astype(np.uint8)
    un = (rng.random(n) < 0.7).astype(np.uint8)
    loss, g = optim.reg_l2(1000.0, tr, un, cur, init)
    assert loss > 0
    l0, g0 = optim.reg_l2(1000.0, tr, un, init, init)
    assert l0 == 0 and all((v == 0).all() for v in g0.values())
    # central differences of the loss on unstable transparent rows
    h = 1e-6
    for k in ("pos", "rot", "scale"):
        for i in np.nonzero((tr != 0) & (un != 0))[0][:5]:
            for c in range(cur[k].shape[1]):
                p = {kk: v.copy() for kk, v in cur.items()}
                m = {kk: v.copy() for kk, v in cur.items()}
                p[k][i, c] += h
                m[k][i, c] -= h
                fd = (optim.reg_l2(1000.0, tr, un, p, init)[0] - optim.reg_l2(1000.0, tr, un, m, init)[0]) / (2 * h)
                assert abs(fd - g[k][i, c]) <= 1e-5 * max(1.0, abs(fd)), (k, i, c)
    # opaque and stable rows get no gradient; opaque rows add no loss
    assert all((v[(tr == 0) | (un == 0)] == 0).all() for v in g.values())
    cur2 = {k: v.copy() for k, v in cur.items()}
    cur2["pos"][tr == 0] += 1.0
    assert optim.reg_l2(1000.0, tr, un, cur2, init)[0] == loss


def test_fusion_is_a_confidence_weighted_running_mean():
    """G_o = (eta_{o-1} G_{o-1} + (eta_o - eta_{o-1}) G'_o) / eta_o: after
    several windows the fused value is the mean of the windows' results
    weighted by the optimisation steps each added."""
    rng = np.random.default_rng(1)
    n = 200
    eta = np.zeros(n, np.int64)
    G = None
    num = np.zeros((n, 3))
    for o in range(5):
        steps = rng.integers(0, 40, n)
        cur = rng.standard_normal((n, 3)).astype(np.float32)
        new_eta = eta + steps
        if G is None:
            G = cur.copy()
            G[steps == 0] = 0.0
            cur = np.where(steps[:, None] == 0, G, cur).astype(np.float32)
        fused = optim.fuse(eta, new_eta, {"x": G}, {"x": cur})["x"]
        num += steps[:, None] * cur.astype(np.float64)
        eta = new_eta
        G = fused
        ok = eta > 0
        np.testing.assert_allclose(G[ok], (num[ok] / eta[ok, None]), rtol=2e-5, atol=2e-6)


def test_fusion_special_cases():
    prev = {"x": np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]], np.float32)}
    cur = {"x": np.array([[9.0, 8.0], [7.0, 6.0], [1.0, 1.0]], np.float32)}
    out = optim.fuse(np.array([0, 4, 3]), np.array([0, 4, 6]), prev, cur)["x"]
    assert np.array_equal(out[0], cur["x"][0])          # eta' = 0: the window's values
    assert np.array_equal(out[1], prev["x"][1])         # no new steps: the previous values
    assert np.array_equal(out[2], np.array([3.0, 3.5], np.float32))   # w = 1/2: the midpoint


def test_top_error_selection_against_brute_force():
    rng = np.random.default_rng(2)
    F, H, W = 3, 7, 9
    Cin = rng.random((F, H, W, 3)).astype(np.float32)
    Cr = rng.random((F, H, W, 3)).astype(np.float32)
    # ties: copy some pixels' renders so their errors repeat exactly
    Cr[1, :2] = Cin[1, :2]                       # zero errors
    Cr[2, 3, :] = Cr[2, 4, :]
    Cin[2, 3, :] = Cin[2, 4, :]
    for frac in (0.0, 0.1, 0.4, 0.75, 1.0):
        m = optim.select_top_error(Cr, Cin, frac)
        e = optim.color_error(Cr, Cin)
        k = int(np.floor(frac * H * W))
        for f in range(F):
            ef = e[f].ravel()
            sel = m[f].ravel() != 0
            if k == 0:
                assert not sel.any()
                continue
            assert sel.sum() >= k
            # every selected error >= every unselected one, and the k-th
            # largest error is selected with all of its ties
            if (~sel).any():
                assert ef[sel].min() > ef[~sel].max()
            kth = sorted(ef, reverse=True)[k - 1]
            assert sel[ef == kth].all()
            if len(np.unique(ef)) == ef.size:
                assert sel.sum() == k
