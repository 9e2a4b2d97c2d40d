"""Torch-facing binding of the frame-to-model tracking call (include/rtg.h,
Sec. 3.2 "Camera tracking", Eq. 10): argument marshalling only; every step
runs in the library's kernels."""
from __future__ import annotations

import ctypes

import torch

from ._lib import IcpParams, check, lib
from .mapping import intrinsics


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def icp_params(levels=None, iters=None, dist=None, sin_angle=None):
    prm = IcpParams()
    lib().rtg_icp_params_default(ctypes.byref(prm))
    if levels is not None:
        prm.levels = int(levels)
    if iters is not None:
        for k, v in enumerate(iters):
            prm.iters[k] = int(v)
    if dist is not None:
        prm.dist = float(dist)
    if sin_angle is not None:
        prm.sin_angle = float(sin_angle)
    return prm


def icp(cam, depth_in, depth_model, normal_model, pose_model, pose_init, prm=None, trace=False):
    """rtg_icp: the refined camera-to-world pose (device float64 (12,)) of the
    frame with depth depth_in against the model's rendered depth and normals
    at pose_model; with trace=True also the per-iteration trace (n, 48)."""
    prm = icp_params() if prm is None else prm
    intr = intrinsics(cam)
    nb = int(lib().rtg_icp_workspace_bytes(ctypes.byref(intr), prm.levels))
    if nb == 0:
        raise ValueError("invalid image size or levels for ICP")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    pose = torch.empty(12, dtype=torch.float64, device="cuda")
    n_it = sum(int(prm.iters[k]) for k in range(prm.levels))
    tr = torch.zeros((max(n_it, 1), 48), dtype=torch.float64, device="cuda") if trace else None
    check(lib().rtg_icp(ctypes.byref(intr), ctypes.byref(prm), _p(depth_in), _p(depth_model), _p(normal_model),
                        _p(pose_model), _p(pose_init), _p(pose), _p(tr), _p(ws), nb,
                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "rtg_icp")
    return (pose, tr) if trace else pose
