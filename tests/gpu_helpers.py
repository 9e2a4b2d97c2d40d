"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded inputs, and compare."""
import numpy as np
import torch

from oracle import oracle as orc


def need_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev_params(scene):
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous()  # noqa: E731
    return (t(scene["pos"]), t(scene["scale"]), t(scene["rot"]), t(scene["opacity"]), t(scene["color"]),
            t(scene["unstable"], torch.uint8))


def dev_poses(poses):
    return torch.as_tensor(np.ascontiguousarray(poses, np.float64).reshape(-1, 12)).to("cuda").contiguous()


def dev_mask(mask):
    return torch.as_tensor(np.ascontiguousarray(mask, np.uint8)).to("cuda").contiguous()


def rel_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


# Parity bars.  NORM_TOL is the normwise relative error ||x - ref|| / ||ref||
# per output tensor (the stated 1e-4).  The elementwise measure is
# |x - ref| / (|ref| + 1e-3 rms(ref) + floor) per element; its 99.99th
# percentile and maximum are gated (the rms term keeps near-zero entries,
# whose relative error is ill-conditioned, from dominating).
#   * colour, depth, transmission: 1e-4 for both.  The transmission's floor
#     is 2e4 t_eps: a pixel stops compositing once T < t_eps, so there its
#     T differs from the oracle's (which composites every listed Gaussian)
#     by less than t_eps in absolute terms.
#   * gradients: 1e-4 as well, with a per-entry floor of 1e4 times the
#     oracle's bound on the error of a binary32 evaluation of the same sums
#     (oracle.backward(..., bound=...); the model is in oracle.c at
#     orc_backward_bound): an entry is a sum over pixels of terms of both
#     signs; each term's relative error is GRAD_GAMMA (64 units in the last
#     place for its ~30 operations and its share of the accumulation) plus
#     the binary32 error of the opacities f that enter it, amplified in the
#     transmission by f / (1 - f) per Gaussian in front, all on magnitudes
#     that ignore cancellation, mapped to the parameters by the chain rule
#     in absolute values; plus what stopping each pixel below t_eps may drop
#     or change.  So |x - ref| <= 1e-4 (|ref| + 1e-3 rms) + bound is what
#     the gate asks.
NORM_TOL = 1e-4
EL_P9999_TOL = 1e-4
EL_MAX_TOL = 1e-4
GRAD_GAMMA = 64 * 2.0 ** -24
T_EPS = 1e-8          # the library's default early-exit transmission
PRECISE_KAPPA = 256.0  # footprints above this condition number use the factored form


def err_stats(a, ref, floor=0.0):
    """Normwise relative error, and the 99.99th percentile and maximum of the
    elementwise measure, of `a` against the reference `ref`."""
    a = np.asarray(a, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    if ref.size == 0:
        return {"norm": 0.0, "p9999": 0.0, "max": 0.0}
    d = np.abs(a - ref)
    nref = np.linalg.norm(ref)
    norm = float(np.linalg.norm(a - ref) / nref) if nref > 0 else float(np.linalg.norm(a - ref))
    rms = float(np.sqrt(np.mean(ref * ref)))
    den = np.abs(ref) + 1e-3 * rms + np.asarray(floor, np.float64).ravel()
    e = np.where(den > 0, d / np.where(den > 0, den, 1.0), d)
    return {"norm": norm, "p9999": float(np.percentile(e, 99.99)), "max": float(e.max())}


def fmt_stats(errs):
    return {k: ({kk: "%.2e" % vv for kk, vv in v.items()} if isinstance(v, dict) else v) for k, v in errs.items()}


def assert_parity(errs, norm_tol=NORM_TOL):
    """Gate every output's statistics (dict values of `errs` that are
    err_stats dicts)."""
    for k, v in errs.items():
        if not isinstance(v, dict) or "norm" not in v:
            continue
        assert v["norm"] <= norm_tol, (k, v)
        assert v["p9999"] <= EL_P9999_TOL, (k, v)
        assert v["max"] <= EL_MAX_TOL, (k, v)


def oracle_grads(P, recs, scene, poses, pix, gC, gD, t_eps=T_EPS):
    """The oracle's gradients and their binary32 error bounds."""
    return orc.backward(P, recs, scene, poses, pix, gC, gD, bound=(GRAD_GAMMA, t_eps, PRECISE_KAPPA))


def grad_stats(grads, gref, unstable=None, bound=None):
    """err_stats per gradient tensor (dict of device tensors against the
    oracle's arrays, with the oracle's error bounds as the floor: 1e4 times
    the bound, so that the 1e-4 gate admits the bound itself); rows of
    stable Gaussians must be exactly zero.  "bound_use" reports the largest
    |x - ref| / bound."""
    out = {}
    for k in ("pos", "scale", "rot", "opacity", "color"):
        got = grads[k].cpu().numpy()
        if unstable is not None:
            assert (got[np.asarray(unstable) == 0] == 0).all(), k
        fl = 0.0 if bound is None else bound[k] / EL_MAX_TOL
        out["d_" + k] = err_stats(got, gref[k], floor=fl)
        if bound is not None:
            d = np.abs(got.astype(np.float64) - gref[k]).ravel()
            b = np.asarray(bound[k]).ravel()
            out["d_" + k]["bound_use"] = float(np.max(np.where(b > 0, d / np.where(b > 0, b, 1), 0.0))) if d.size else 0.0
    return out


def gpu_forward(rast, scene, poses, mask):
    params = dev_params(scene)
    C, D, T, I, ws = rast.forward(params, dev_poses(poses), dev_mask(mask))
    torch.cuda.synchronize()
    st = rast.read_status(ws)
    return {"color": C.cpu().numpy(), "depth": D.cpu().numpy(), "trans": T.cpu().numpy(),
            "index": I.cpu().numpy(), "ws": ws, "params": params, "status": st,
            "tensors": (C, D, T, I)}


def oracle_forward(cam, scene, poses, mask, **kw):
    P = orc.make_params(cam, **kw)
    recs = orc.project(P, scene, poses)
    pix = orc.masked_pixels(mask)
    out = orc.render(P, recs, scene, pix)
    return P, recs, pix, out


def ws_view(rast, ws, name, dtype, count):
    off = rast.layout[name]
    nbytes = count * torch.tensor([], dtype=dtype).element_size()
    return ws[off:off + nbytes].view(dtype)


def check_depth_branch(gd, ref, recs, pix):
    """The Eq. 5 branch per hit pixel.  Where the oracle takes the centre
    depth, the GPU's depth is the stored binary32 centre depth, bit for bit;
    where it intersects the disc plane and the plane depth differs from the
    centre depth by more than 1e-5 relative, the GPU's depth is the plane
    depth (within 1e-5), never the centre depth.  Returns the counts of
    (plane, centre, indistinguishable plane) pixels."""
    idx = ref["index"]
    hit = idx >= 0
    f = pix[hit, 0]
    z32 = recs["z32"][f, idx[hit]].astype(np.float32)
    br = ref["branch"][hit]
    g = np.asarray(gd, np.float32)[hit]
    assert set(np.unique(br)) <= {1, 2}
    cen = br == 2
    assert np.array_equal(g[cen].view(np.uint32), z32[cen].view(np.uint32)), "centre-depth pixels"
    pl = br == 1
    plane = ref["depth"][hit][pl]
    sep = np.abs(plane - z32[pl]) > 1e-5 * np.abs(plane)
    gp = g[pl][sep].astype(np.float64)
    assert not np.any(g[pl][sep] == z32[pl][sep]), "plane pixels rendered with the centre depth"
    assert np.all(np.abs(gp - plane[sep]) <= 1e-5 * np.abs(plane[sep])), "plane depth"
    return {"plane": int(sep.sum()), "centre": int(cen.sum()), "plane_eq_centre": int((~sep).sum())}


def compare_forward(g, pix, out, recs=None, t_eps=T_EPS):
    """GPU outputs at the oracle's pixels; returns per-output statistics
    (err_stats; the transmission with the early-exit floor of t_eps), the
    index mismatch count and, with the oracle's records, the depth-branch
    counts (check_depth_branch)."""
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    gc = g["color"][f, y, x]
    gd = g["depth"][f, y, x]
    gt = g["trans"][f, y, x]
    gi = g["index"][f, y, x]
    errs = {"color": err_stats(gc, out["color"]), "trans": err_stats(gt, out["trans"], floor=2e4 * t_eps),
            "depth": err_stats(gd, out["depth"]),
            "index_mismatch": int((gi != out["index"]).sum())}
    if recs is not None and errs["index_mismatch"] == 0:
        errs["branch"] = check_depth_branch(gd, out, recs, pix)
    return errs
