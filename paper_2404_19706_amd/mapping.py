"""Torch-facing binding of the adding and state-management calls
(include/rtg.h, Sec. 3.2): argument marshalling only; every step runs in
the library's kernels."""
from __future__ import annotations

import ctypes

import torch

from ._lib import AddingParams, Intrinsics, check, lib

STATE_FIELDS = (("pos", torch.float32, 3), ("scale", torch.float32, 3), ("rot", torch.float32, 4),
                ("opacity", torch.float32, 0), ("color", torch.float32, 3), ("unstable", torch.uint8, 0),
                ("eta", torch.int32, 0), ("err", torch.int32, 0), ("tstamp", torch.int32, 0))


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def adding_params(**kw):
    a = AddingParams()
    lib().rtg_adding_params_default(ctypes.byref(a))
    for k, v in kw.items():
        if not hasattr(a, k):
            raise TypeError("unknown adding parameter %r" % k)
        setattr(a, k, v)
    return a


def intrinsics(cam):
    return Intrinsics(float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"]),
                      int(cam["width"]), int(cam["height"]))


def alloc_state(capacity, device="cuda", sh_degree=0):
    """Per-Gaussian arrays with room for `capacity` rows (colour rows of
    SH coefficients (K, 3) with sh_degree > 0)."""
    out = {}
    for name, dt, w in STATE_FIELDS:
        shape = (capacity, w) if w else (capacity,)
        if name == "color" and sh_degree:
            shape = (capacity, (sh_degree + 1) ** 2, 3)
        out[name] = torch.zeros(shape, dtype=dt, device=device)
    return out


def add_gaussians(cam, prm, pose, color_in, depth_in, color_r, depth_r, trans_r, index_r, rand, frame_k, n_cur,
                  state, mask_out=None):
    """rtg_add_gaussians into `state` (rows n_cur..); returns a device int64
    tensor [rows added, pixels that qualified]."""
    intr = intrinsics(cam)
    ws = torch.empty(int(lib().rtg_adding_workspace_bytes(ctypes.byref(intr))), dtype=torch.uint8, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    cap = state["pos"].shape[0]
    check(lib().rtg_add_gaussians(ctypes.byref(intr), ctypes.byref(prm), _p(pose), _p(color_in), _p(depth_in),
                                  _p(color_r), _p(depth_r), _p(trans_r), _p(index_r), _p(rand), int(frame_k),
                                  int(n_cur), int(cap), _p(state["pos"]), _p(state["scale"]), _p(state["rot"]),
                                  _p(state["opacity"]), _p(state["color"]), _p(state["unstable"]),
                                  _p(state["eta"]), _p(state["err"]), _p(state["tstamp"]), _p(mask_out),
                                  _p(counts), _p(ws), ws.numel(), _s()), "rtg_add_gaussians")
    return counts


def confidence_count(n, unstable, d_color, eta):
    """eta + 1 for unstable rows with a non-zero colour gradient row
    (d_color of shape (n, 3) for RGB or (n, K, 3) for SH)."""
    width = int(d_color[0].numel()) if n > 0 else 3
    check(lib().rtg_confidence_count(int(n), width, _p(unstable), _p(d_color), _p(eta), _s()),
          "rtg_confidence_count")


def state_update(cam, prm, color_in, depth_in, color_r, depth_r, index_r, frame_k, n, state):
    """rtg_state_update on the first n rows of `state`; returns keep (uint8)."""
    intr = intrinsics(cam)
    keep = torch.empty(n, dtype=torch.uint8, device="cuda")
    flag = torch.empty(n, dtype=torch.uint8, device="cuda")
    check(lib().rtg_state_update(ctypes.byref(intr), ctypes.byref(prm), _p(color_in), _p(depth_in), _p(color_r),
                                 _p(depth_r), _p(index_r), int(frame_k), int(n), _p(state["unstable"]),
                                 _p(state["eta"]), _p(state["err"]), _p(state["tstamp"]), _p(keep), _p(flag), _s()),
          "rtg_state_update")
    return keep


def compact_rows(n, keep, src, dst):
    """rtg_compact_rows over matching lists of tensors (rows along dim 0);
    returns the kept count as a device int64 tensor."""
    k = len(src)
    S = (ctypes.c_void_p * k)(*[t.data_ptr() for t in src])
    D = (ctypes.c_void_p * k)(*[t.data_ptr() for t in dst])
    rb = (ctypes.c_int32 * k)(*[t[0].numel() * t.element_size() if t.dim() > 1 else t.element_size() for t in src])
    ws = torch.empty(int(lib().rtg_compact_workspace_bytes(int(n))), dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    check(lib().rtg_compact_rows(int(n), _p(keep), k, S, D, rb, _p(out), _p(ws), ws.numel(), _s()),
          "rtg_compact_rows")
    return out


# ---- the mapping iteration around the backward (Sec. 3.2, Eq. 8-9) -------

def reg_l2(w_reg, transparent, unstable, cur, init, grads, loss_out):
    """rtg_reg_l2: adds w_reg L_reg to loss_out (device float64 [1]) and its
    gradient to grads["pos"], ["scale"], ["rot"] of the unstable transparent
    rows; cur / init: dicts with "pos", "scale", "rot"."""
    n = int(transparent.shape[0])
    check(lib().rtg_reg_l2(n, float(w_reg), _p(transparent), _p(unstable), _p(cur["pos"]), _p(cur["scale"]),
                           _p(cur["rot"]), _p(init["pos"]), _p(init["scale"]), _p(init["rot"]),
                           _p(grads["pos"]), _p(grads["scale"]), _p(grads["rot"]), _p(loss_out), _s()),
          "rtg_reg_l2")


def fuse(eta_prev, eta_cur, prev, cur):
    """rtg_fuse (Eq. 9): fuses cur ("pos", "scale", "rot", "color"; updated in
    place) with prev, weighted by the confidence counts."""
    n = int(eta_cur.shape[0])
    width = int(cur["color"][0].numel()) if n > 0 else 3
    check(lib().rtg_fuse(n, width, _p(eta_prev), _p(eta_cur), _p(prev["pos"]), _p(prev["scale"]), _p(prev["rot"]),
                         _p(prev["color"]), _p(cur["pos"]), _p(cur["scale"]), _p(cur["rot"]), _p(cur["color"]),
                         _s()), "rtg_fuse")


def select_top_error(color_r, color_in, frac, mask_out=None):
    """rtg_select_top_error: uint8 mask [F][H][W] of the pixels whose colour
    error is at least the k-th largest of their frame, k = floor(frac H W)."""
    F, H, W = int(color_r.shape[0]), int(color_r.shape[1]), int(color_r.shape[2])
    nb = int(lib().rtg_select_workspace_bytes(F, H, W))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    if mask_out is None:
        mask_out = torch.empty((F, H, W), dtype=torch.uint8, device="cuda")
    check(lib().rtg_select_top_error(F, H, W, float(frac), _p(color_r), _p(color_in), _p(mask_out), _p(ws), nb,
                                     _s()), "rtg_select_top_error")
    return mask_out
