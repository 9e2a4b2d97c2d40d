"""GPU parity of Gaussian adding (Eq. 6) and state management (Sec. 3.2)
against the reference in oracle/adding.py, through the C ABI, on seeded
synthetic frames (a smooth depth surface with holes and edges, colour and
depth errors, an index map over a Gaussian table with stable and unstable
rows) at a ragged size and at the 1200x680 keyframe size.

Bar: masks, which pixels add a Gaussian and in which order, the counts,
and every state change bit-exact; new discs' position, scale, opacity and
colour within binary32 rounding of the reference (1e-6 relative), their
orientation as the normal up to sign (the disc is symmetric)."""
import numpy as np
import pytest
import torch

from oracle import adding as A
from rtg_synth import camera
from tests.gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()
    from paper_2404_19706_amd import lib
    lib()
    yield


def _frame(seed, W, H, n_g=5000):
    rng = np.random.default_rng(seed)
    cam = camera(W, H, 0.8 * W, 0.8 * W)
    yy, xx = np.mgrid[0:H, 0:W]
    D = (2.0 + 0.5 * np.sin(xx / 37.0) + 0.3 * np.cos(yy / 23.0)).astype(np.float32)
    D[(xx // 40 + yy // 30) % 7 == 0] = 0.0                       # holes
    D[rng.random((H, W)) < 0.02] = 0.0
    C = rng.random((H, W, 3)).astype(np.float32)
    Dr = (D + rng.choice([0.0, 0.03, 0.2], (H, W), p=[0.6, 0.3, 0.1])).astype(np.float32)
    Dr[rng.random((H, W)) < 0.05] = -1.0
    Tr = rng.choice([0.1, 0.3, 0.8], (H, W), p=[0.6, 0.3, 0.1]).astype(np.float32)
    Cr = (C + rng.choice([0.0, 0.02, 0.2], (H, W, 1), p=[0.5, 0.3, 0.2])).astype(np.float32)
    I = rng.integers(-1, n_g, (H, W)).astype(np.int32)
    un = (rng.random(n_g) < 0.5).astype(np.uint8)
    rand = rng.random((H, W)).astype(np.float32)
    pose = np.concatenate([np.linalg.qr(rng.standard_normal((3, 3)))[0].ravel(), rng.uniform(-1, 1, 3)])
    if np.linalg.det(pose[:9].reshape(3, 3)) < 0:
        pose[:9] *= -1.0
    return cam, pose, C, D, Cr, Dr, Tr, I, un, rand


def _t(a, dt=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return (t if dt is None else t.to(dt)).cuda()


@pytest.mark.parametrize("W,H,rate,cap_extra", [(97, 61, 0.3, None), (1200, 680, 0.05, None), (97, 61, 0.5, 17)])
def test_add_gaussians_matches_reference(W, H, rate, cap_extra):
    from paper_2404_19706_amd import mapping as M
    cam, pose, C, D, Cr, Dr, Tr, I, un, rand = _frame(7 + W, W, H)
    n_cur = len(un)
    cap = n_cur + (cap_extra if cap_extra is not None else W * H)
    P = A.params(rate=rate)
    ref = A.add_gaussians(cam, P, pose, C, D, Cr, Dr, Tr, I, un, rand, 11, n_cur, cap)
    st = M.alloc_state(cap)
    st["unstable"][:n_cur] = _t(un)
    mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    counts = M.add_gaussians(cam, M.adding_params(rate=rate), _t(pose, torch.float64), _t(C), _t(D), _t(Cr), _t(Dr),
                             _t(Tr), _t(I), _t(rand), 11, n_cur, st, mask)
    torch.cuda.synchronize()
    n_add, n_cand = (int(v) for v in counts.cpu())
    print("adding %dx%d rate %.2f: %d pixels qualify, %d rows added" % (W, H, rate, n_cand, n_add), flush=True)
    assert np.array_equal(mask.cpu().numpy(), ref["mask"])
    assert n_cand == len(ref["candidates"]) and n_add == ref["n_added"] > 0
    rows = ref["rows"]
    sl = slice(n_cur, n_cur + n_add)
    got = {k: v[sl].cpu().numpy() for k, v in st.items()}
    np.testing.assert_allclose(got["pos"], rows["pos"], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(got["scale"], rows["scale"], rtol=1e-6, atol=0)
    np.testing.assert_array_equal(got["opacity"], rows["opacity"].astype(np.float32))
    np.testing.assert_array_equal(got["color"], rows["color"].astype(np.float32))
    assert np.all(got["unstable"] == 1) and np.all(got["eta"] == 0) and np.all(got["err"] == 0)
    assert np.all(got["tstamp"] == 11)
    # orientation: the rotated thin axis is the reference normal up to sign
    q = got["rot"].astype(np.float64)
    w, x, y, z = q.T
    ez = np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)], 1)
    assert np.all(np.abs(np.abs((ez * rows["normal"]).sum(1)) - 1.0) < 1e-5)
    # the existing rows are untouched
    assert np.array_equal(st["unstable"][:n_cur].cpu().numpy(), un)


def test_state_update_and_removal_match_reference():
    from paper_2404_19706_amd import mapping as M
    W, H, n = 160, 120, 3000
    cam, pose, C, D, Cr, Dr, Tr, I, un, rand = _frame(5, W, H, n_g=n)
    rng = np.random.default_rng(6)
    eta = rng.integers(0, 150, n).astype(np.int32)
    err = rng.integers(0, 7, n).astype(np.int32)
    ts = rng.integers(0, 400, n).astype(np.int32)
    P = A.params()
    k = 300
    ru, re, rr, rt, rkeep = A.state_update(P, Cr, Dr, I, C, D, un, eta, err, ts, k)
    st = M.alloc_state(n)
    st["unstable"][:] = _t(un)
    st["eta"][:] = _t(eta)
    st["err"][:] = _t(err)
    st["tstamp"][:] = _t(ts)
    keep = M.state_update(cam, M.adding_params(), _t(C), _t(D), _t(Cr), _t(Dr), _t(I), k, n, st)
    torch.cuda.synchronize()
    for name, r in (("unstable", ru), ("eta", re), ("err", rr), ("tstamp", rt)):
        assert np.array_equal(st[name].cpu().numpy(), r), name
    assert np.array_equal(keep.cpu().numpy().astype(bool), rkeep)
    assert 0 < int(rkeep.sum()) < n
    # removal: compact every per-Gaussian array by the keep mask
    st["pos"][:] = _t(rng.standard_normal((n, 3)).astype(np.float32))
    st["rot"][:] = _t(rng.standard_normal((n, 4)).astype(np.float32))
    dst = M.alloc_state(n)
    names = [s[0] for s in M.STATE_FIELDS]
    nout = M.compact_rows(n, keep, [st[k_] for k_ in names], [dst[k_] for k_ in names])
    torch.cuda.synchronize()
    m = int(nout.item())
    assert m == int(rkeep.sum())
    for k_ in names:
        ref = A.compact(rkeep, st[k_].cpu().numpy())[0]
        assert np.array_equal(dst[k_][:m].cpu().numpy(), ref), k_


def test_confidence_count_matches_reference():
    from paper_2404_19706_amd import mapping as M
    rng = np.random.default_rng(8)
    n = 10000
    un = (rng.random(n) < 0.4).astype(np.uint8)
    g = rng.standard_normal((n, 3)).astype(np.float32)
    g[rng.random(n) < 0.3] = 0.0
    eta = rng.integers(0, 50, n).astype(np.int32)
    te = _t(eta)
    M.confidence_count(n, _t(un), _t(g), te)
    torch.cuda.synchronize()
    assert np.array_equal(te.cpu().numpy(), A.confidence_count(un, g, eta))
