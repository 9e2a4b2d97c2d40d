"""Python binding of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.
It shares no code with the HIP path.  Besides the C reference it holds two
small numpy references used by the harness:

* :func:`l1_upstream` -- gradient of the L1 colour and depth losses of
  Eq. (7)-(8) (w_c = w_d = 1; no depth loss where nothing is hit).
* :func:`adam_step` -- the textbook Adam update (Kingma & Ba, Alg. 1) applied
  to the rows of unstable Gaussians only (Sec. 3.2 optimises unstable
  Gaussians; the opacity learning rate is zero, supplementary Sec. C).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc (no FP contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("cutoff2", ctypes.c_float), ("dilation", ctypes.c_float),
                ("z_near", ctypes.c_float),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


REC_DTYPE = np.dtype([
    ("culled", np.int32), ("visible", np.int32), ("rect", np.int32, 4), ("axis", np.int32),
    ("mu32", np.float32, 2), ("conic32", np.float32, 3), ("z32", np.float32),
    ("tau32", np.float32), ("nc32", np.float32, 3), ("h32", np.float32),
    ("pc", np.float64, 3), ("mu", np.float64, 2), ("cov", np.float64, 3),
    ("conic", np.float64, 3), ("nc", np.float64, 3), ("h", np.float64),
], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.orc_sizeof_rec.restype = i32
        L.orc_sizeof_params.restype = i32
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        L.orc_project.argtypes = [P, i64, i32, P, P, P, P, P, P]
        L.orc_filter50.argtypes = [P, i32, P, P]
        L.orc_bin.argtypes = [P, i64, i32, P, P, i64, P, P, P, P]
        L.orc_bin.restype = i64
        L.orc_render.argtypes = [P, i64, i32, P, P, P, i64, P, P, P, P, P, P, P, P]
        L.orc_unstable_mask.argtypes = [P, i64, i32, P, P, i64, P, P]
        L.orc_pixel_lists.argtypes = [P, i64, i32, P, i64, P, i32, P, P]
        L.orc_backward.argtypes = [P, i64, i32, P, P, P, P, P, P, P, P, i64, P, P, P, P]
        L.orc_backward_bound.argtypes = [P, i64, i32, P, P, P, P, P, P, P, P, i64, P, P, P, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, P, P]
        assert L.orc_sizeof_rec() == REC_DTYPE.itemsize, (L.orc_sizeof_rec(), REC_DTYPE.itemsize)
        assert L.orc_sizeof_params() == ctypes.sizeof(Params)
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_params(cam, cutoff2=9.0, dilation=0.0, z_near=0.2, tile=(16, 16)):
    """cam: dict with fx, fy, cx, cy, width, height."""
    return Params(float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"]),
                  int(cam["width"]), int(cam["height"]), float(cutoff2), float(dilation),
                  float(z_near), int(tile[0]), int(tile[1]))


def _f32(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.shape == shape, (a.shape, shape)
    return a


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops (timing only)."""
    lib().orc_set_num_threads(int(n))


def project(params, scene, poses):
    """Projection records of every Gaussian in every frame, shape (F, N)."""
    N = scene["pos"].shape[0]
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 12)
    F = poses.shape[0]
    out = np.zeros(F * N, dtype=REC_DTYPE)
    pos = _f32(scene["pos"], (N, 3))
    sc = _f32(scene["scale"], (N, 3))
    rot = _f32(scene["rot"], (N, 4))
    op = _f32(scene["opacity"], (N,))
    lib().orc_project(ctypes.byref(params), N, F, _p(poses), _p(pos), _p(sc), _p(rot), _p(op), _p(out))
    return out.reshape(F, N)


def filter50(params, mask):
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.empty_like(mask)
    lib().orc_filter50(ctypes.byref(params), mask.shape[0], _p(mask), _p(out))
    return out


def bin_pairs(params, recs, mask):
    """Sorted (frame, tile, gid) pairs and per-(frame, tile) activity."""
    F, N = recs.shape
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    tw, th = params.tile_w, params.tile_h
    nt = ((params.width + tw - 1) // tw) * ((params.height + th - 1) // th)
    act = np.zeros(F * nt, dtype=np.uint8)
    recs_c = np.ascontiguousarray(recs.reshape(-1))
    e = np.zeros(1, dtype=np.int32)
    K = lib().orc_bin(ctypes.byref(params), N, F, _p(recs_c), _p(mask), 0, _p(e), _p(e), _p(e), _p(act))
    fr = np.zeros(max(K, 1), dtype=np.int32)
    ti = np.zeros(max(K, 1), dtype=np.int32)
    gi = np.zeros(max(K, 1), dtype=np.int32)
    K2 = lib().orc_bin(ctypes.byref(params), N, F, _p(recs_c), _p(mask), K, _p(fr), _p(ti), _p(gi), _p(act))
    assert K2 == K
    return {"K": int(K), "frame": fr[:K], "tile": ti[:K], "gid": gi[:K],
            "tile_active": act.reshape(F, nt)}


def masked_pixels(mask):
    """(P, 3) int32 array of (frame, x, y) for every set mask byte, in
    frame-major raster order."""
    f, y, x = np.nonzero(np.asarray(mask))
    return np.ascontiguousarray(np.stack([f, x, y], axis=1).astype(np.int32))


def _colors(scene, N):
    """Colours as the C oracle takes them, binary64: the binary32 parameter
    values, or scene["color64"] when a caller supplies colours computed in
    binary64 (the view-dependent colours of oracle.sh)."""
    if "color64" in scene:
        return np.ascontiguousarray(scene["color64"], dtype=np.float64).reshape(N, 3)
    return np.ascontiguousarray(_f32(scene["color"], (N, 3)), dtype=np.float64)


def render(params, recs, scene, pix):
    F, N = recs.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    NP = pix.shape[0]
    op = _f32(scene["opacity"], (N,))
    col = _colors(scene, N)
    out = {"color": np.zeros((NP, 3)), "depth": np.zeros(NP), "trans": np.zeros(NP),
           "index": np.zeros(NP, dtype=np.int32), "branch": np.zeros(NP, dtype=np.int32),
           "nlist": np.zeros(NP, dtype=np.int32), "sig": np.zeros(NP, dtype=np.uint64)}
    recs_c = np.ascontiguousarray(recs.reshape(-1))
    lib().orc_render(ctypes.byref(params), N, F, _p(recs_c), _p(op), _p(col), NP, _p(pix),
                     _p(out["color"]), _p(out["depth"]), _p(out["trans"]), _p(out["index"]),
                     _p(out["branch"]), _p(out["nlist"]), _p(out["sig"]))
    return out


def pixel_lists(params, recs, pix, max_len=4096):
    """L(u) of each pixel (Gaussian indices in list order): a list of
    arrays."""
    F, N = recs.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    NP = pix.shape[0]
    gid = np.zeros((NP, max_len), dtype=np.int32)
    ln = np.zeros(NP, dtype=np.int32)
    recs_c = np.ascontiguousarray(recs.reshape(-1))
    lib().orc_pixel_lists(ctypes.byref(params), N, F, _p(recs_c), NP, _p(pix), int(max_len), _p(gid), _p(ln))
    assert ln.max(initial=0) <= max_len
    return [gid[p, :ln[p]].copy() for p in range(NP)]


def unstable_mask(params, recs, unstable, pix):
    F, N = recs.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    un = np.ascontiguousarray(unstable, dtype=np.uint8).reshape(N)
    out = np.zeros(pix.shape[0], dtype=np.uint8)
    recs_c = np.ascontiguousarray(recs.reshape(-1))
    lib().orc_unstable_mask(ctypes.byref(params), N, F, _p(recs_c), _p(un), pix.shape[0], _p(pix), _p(out))
    return out


def unstable_mask_image(params, recs, unstable):
    F = recs.shape[0]
    W, H = params.width, params.height
    pix = masked_pixels(np.ones((F, H, W), dtype=np.uint8))
    return unstable_mask(params, recs, unstable, pix).reshape(F, H, W)


GRAD_FIELDS = (("pos", 3), ("scale", 3), ("rot", 4), ("opacity", 1), ("color", 3))


def backward(params, recs, scene, poses, pix, gC, gD, bound=None):
    """Parameter gradients of sum(gC . C) + sum(gD . D) over the listed
    pixels; rows of stable Gaussians are zero.  With bound=(gamma, t_eps,
    kappa_thr), returns (gradients, bounds): per entry, a bound on the error
    of a binary32 evaluation of the same sums (base relative error gamma per
    term, the error model of orc_backward_bound in oracle.c, pixels that
    stop compositing below t_eps, factored evaluation of footprints with
    condition number above kappa_thr)."""
    F, N = recs.shape
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    NP = pix.shape[0]
    poses = np.ascontiguousarray(poses, dtype=np.float64).reshape(-1, 12)
    gC = np.ascontiguousarray(gC, dtype=np.float64).reshape(NP, 3)
    gD = np.ascontiguousarray(gD, dtype=np.float64).reshape(NP)
    out = np.zeros((N, 14))
    recs_c = np.ascontiguousarray(recs.reshape(-1))
    pos = _f32(scene["pos"], (N, 3))
    sc = _f32(scene["scale"], (N, 3))
    rot = _f32(scene["rot"], (N, 4))
    op = _f32(scene["opacity"], (N,))
    col = _colors(scene, N)
    un = np.ascontiguousarray(scene["unstable"], dtype=np.uint8).reshape(N)
    args = (ctypes.byref(params), N, F, _p(poses), _p(recs_c), _p(pos), _p(sc), _p(rot),
            _p(op), _p(col), _p(un), NP, _p(pix), _p(gC), _p(gD))
    if bound is None:
        lib().orc_backward(*args, _p(out))
        return _split_grads(out)
    bnd = np.zeros((N, 14))
    lib().orc_backward_bound(*args, float(bound[0]), float(bound[1]), float(bound[2]), _p(out), _p(bnd))
    return _split_grads(out), _split_grads(bnd)


def _split_grads(out):
    res, o = {}, 0
    for name, w in GRAD_FIELDS:
        res[name] = out[:, o:o + w].reshape(-1, w) if w > 1 else out[:, o].copy()
        o += w
    return res


def l1_upstream(color, depth, color_gt, depth_gt, mask, w_c=1.0, w_d=1.0):
    """Upstream gradients of L = w_c/(3|M|) sum_{M,ch} |C - C*| +
    w_d/|M_D| sum_{M_D} |D - D*|, M_D = {u in M: D != -1, D* > 0}
    (Eq. 7-8; depth loss skipped where nothing is hit).  sign(0) = 0.
    Returns (gC, gD, loss) as dense float64 arrays on the image grid."""
    m = np.asarray(mask) != 0
    md = m & (np.asarray(depth) != -1.0) & (np.asarray(depth_gt) > 0)
    nm = max(int(m.sum()), 1)
    nd = max(int(md.sum()), 1)
    dc = np.asarray(color, np.float64) - np.asarray(color_gt, np.float64)
    dd = np.asarray(depth, np.float64) - np.asarray(depth_gt, np.float64)
    gC = np.where(m[..., None], np.sign(dc) * (w_c / (3.0 * nm)), 0.0)
    gD = np.where(md, np.sign(dd) * (w_d / nd), 0.0)
    loss = w_c * np.abs(dc)[m].sum() / (3.0 * nm) + w_d * np.abs(dd)[md].sum() / nd
    return gC, gD, loss


def adam_step(param, grad, m, v, step, lr, unstable, beta1=0.9, beta2=0.999, eps=1e-8):
    """Textbook Adam on the rows of unstable Gaussians, in float64; returns
    new (param, m, v).  step is the 1-based step count."""
    param = np.array(param, np.float64)
    m = np.array(m, np.float64)
    v = np.array(v, np.float64)
    rows = np.asarray(unstable) != 0
    g = np.asarray(grad, np.float64)[rows]
    m[rows] = beta1 * m[rows] + (1 - beta1) * g
    v[rows] = beta2 * v[rows] + (1 - beta2) * g * g
    mh = m[rows] / (1 - beta1 ** step)
    vh = v[rows] / (1 - beta2 ** step)
    param[rows] = param[rows] - lr * mh / (np.sqrt(vh) + eps)
    return param, m, v
