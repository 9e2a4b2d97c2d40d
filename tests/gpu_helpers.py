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


def compare_forward(g, pix, out, tol=1e-4):
    """GPU outputs at the oracle's pixels; returns per-output errors."""
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    gc = g["color"][f, y, x]
    gd = g["depth"][f, y, x]
    gt = g["trans"][f, y, x]
    gi = g["index"][f, y, x]
    errs = {"color": rel_err(gc, out["color"]), "trans": rel_err(gt, out["trans"]),
            "depth": rel_err(gd, out["depth"]),
            "index_mismatch": int((gi != out["index"]).sum())}
    return errs
