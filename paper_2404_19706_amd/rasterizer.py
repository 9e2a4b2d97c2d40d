"""Torch-facing binding of the HIP rasterizer: plans, workspaces, the
masked forward/backward as a ``torch.autograd.Function``, and the harness
calls (M_unstable, L1 loss, Adam).

PyTorch supplies device memory and the stream; every step of the path runs
in the library's kernels (see include/rtg.h for the ABI)."""
from __future__ import annotations

import ctypes

import torch

from ._lib import Intrinsics, check, default_config, lib

GRAD_NAMES = ("pos", "scale", "rot", "opacity", "color")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _req(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


class Rasterizer:
    """A plan for N Gaussians, F frames of one camera, and a pair capacity.

    cam: dict with fx, fy, cx, cy, width, height.  Config fields (tile_w,
    tile_h, cutoff2, dilation, z_near, t_eps, items_per_pop, tile_filter50,
    sort_cap, stage_cap, sh_degree, depth_mode, straggler_lanes,
    straggler_rest, static_share, fwd_items_per_pop, fwd_static_share) are
    keyword arguments.  With sh_degree D > 0 the colour parameters are SH
    coefficients of shape (n, K, 3), K = (D + 1)^2, instead of RGB colours
    (n, 3)."""

    def __init__(self, cam, n, frames=1, max_pairs=None, **cfg):
        self.cam = dict(cam)
        self.n = int(n)
        self.frames = int(frames)
        self.W, self.H = int(cam["width"]), int(cam["height"])
        if max_pairs is None:
            max_pairs = max(1 << 20, 64 * self.n * self.frames)
        self.max_pairs = int(min(max_pairs, (1 << 31) - 1))
        self.cfg = default_config(**cfg)
        intr = Intrinsics(float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"]),
                          self.W, self.H)
        plan = ctypes.c_void_p()
        check(lib().rtg_plan_create(ctypes.byref(self.cfg), ctypes.byref(intr), self.n, self.frames,
                                    self.max_pairs, ctypes.byref(plan)), "rtg_plan_create")
        self._plan = plan
        self.ws_bytes = int(lib().rtg_plan_workspace_bytes(plan))
        self.sh_degree = int(self.cfg.sh_degree)
        self.color_shape = (self.n, 3) if self.sh_degree == 0 else (self.n, (self.sh_degree + 1) ** 2, 3)
        lay = (ctypes.c_int64 * 10)()
        lib().rtg_plan_layout(plan, lay, 10)
        self.layout = dict(zip(["hot", "zkey", "rect", "vis", "tile_end", "tile_start", "pairs",
                                "tile_npx", "grad", "hdr"], list(lay)))

    def __del__(self):
        try:
            if getattr(self, "_plan", None):
                lib().rtg_plan_destroy(self._plan)
                self._plan = None
        except Exception:
            pass

    # ---------------------------------------------------------------- memory
    def new_workspace(self, device=None):
        ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device or "cuda")
        if ws.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        return ws

    def _check_params(self, pos, scale, rot, opacity, color, unstable):
        n = self.n
        _req(pos, torch.float32, (n, 3), "pos")
        _req(scale, torch.float32, (n, 3), "scale")
        _req(rot, torch.float32, (n, 4), "rot")
        _req(opacity, torch.float32, (n,), "opacity")
        _req(color, torch.float32, self.color_shape, "color")
        _req(unstable, torch.uint8, (n,), "unstable")

    def _check_poses(self, poses):
        _req(poses, torch.float64, (self.frames, 12), "poses")

    # ---------------------------------------------------------------- steps
    def project(self, ws, pos, scale, rot, opacity, color, unstable, poses):
        self._check_params(pos, scale, rot, opacity, color, unstable)
        self._check_poses(poses)
        check(lib().rtg_project(self._plan, _ptr(ws), _ptr(pos), _ptr(scale), _ptr(rot), _ptr(opacity),
                                _ptr(color), _ptr(unstable), _ptr(poses), _stream()), "rtg_project")

    def unstable_mask_into(self, ws, mask_out):
        _req(mask_out, torch.uint8, (self.frames, self.H, self.W), "mask_out")
        check(lib().rtg_unstable_mask(self._plan, _ptr(ws), _ptr(mask_out), _stream()), "rtg_unstable_mask")
        return mask_out

    def bin(self, ws, mask):
        _req(mask, torch.uint8, (self.frames, self.H, self.W), "mask")
        check(lib().rtg_bin(self._plan, _ptr(ws), _ptr(mask), _stream()), "rtg_bin")

    def alloc_outputs(self, device="cuda"):
        F, H, W = self.frames, self.H, self.W
        return (torch.zeros((F, H, W, 3), dtype=torch.float32, device=device),
                torch.full((F, H, W), -1.0, dtype=torch.float32, device=device),
                torch.ones((F, H, W), dtype=torch.float32, device=device),
                torch.full((F, H, W), -1, dtype=torch.int32, device=device))

    def render_into(self, ws, color, depth, trans, index):
        F, H, W = self.frames, self.H, self.W
        _req(color, torch.float32, (F, H, W, 3), "color")
        _req(depth, torch.float32, (F, H, W), "depth")
        _req(trans, torch.float32, (F, H, W), "trans")
        _req(index, torch.int32, (F, H, W), "index")
        check(lib().rtg_render(self._plan, _ptr(ws), _ptr(color), _ptr(depth), _ptr(trans), _ptr(index),
                               _stream()), "rtg_render")

    def render_normals_into(self, ws, normals):
        """Normal map of the last render on ws (camera frame, facing the
        camera; 0 on rendered pixels without a hit)."""
        _req(normals, torch.float32, (self.frames, self.H, self.W, 3), "normals")
        check(lib().rtg_render_normals(self._plan, _ptr(ws), _ptr(normals), _stream()), "rtg_render_normals")
        return normals

    def alloc_grads(self, device="cuda"):
        n = self.n
        return {"pos": torch.zeros((n, 3), device=device), "scale": torch.zeros((n, 3), device=device),
                "rot": torch.zeros((n, 4), device=device), "opacity": torch.zeros((n,), device=device),
                "color": torch.zeros(self.color_shape, device=device)}

    def alloc_adam_state(self, device="cuda"):
        """Zeroed Adam moments m, v of shape (n, 10 + 3K) and the step counter."""
        w = 10 + 3 * (1 if self.sh_degree == 0 else (self.sh_degree + 1) ** 2)
        return (torch.zeros((self.n, w), device=device), torch.zeros((self.n, w), device=device),
                torch.zeros(1, dtype=torch.int32, device=device))

    def backward_into(self, ws, params, poses, depth, trans, index, d_color, d_depth, grads):
        pos, scale, rot, opacity, color, unstable = params
        F, H, W = self.frames, self.H, self.W
        _req(d_color, torch.float32, (F, H, W, 3), "d_color")
        _req(d_depth, torch.float32, (F, H, W), "d_depth")
        check(lib().rtg_backward(self._plan, _ptr(ws), _ptr(pos), _ptr(scale), _ptr(rot), _ptr(opacity),
                                 _ptr(color), _ptr(unstable), _ptr(poses), _ptr(depth), _ptr(trans),
                                 _ptr(index), _ptr(d_color), _ptr(d_depth), _ptr(grads["pos"]),
                                 _ptr(grads["scale"]), _ptr(grads["rot"]), _ptr(grads["opacity"]),
                                 _ptr(grads["color"]), _stream()), "rtg_backward")
        return grads

    def backward_raster(self, ws, depth, trans, index, d_color, d_depth):
        check(lib().rtg_backward_raster(self._plan, _ptr(ws), _ptr(depth), _ptr(trans), _ptr(index),
                                        _ptr(d_color), _ptr(d_depth), _stream()), "rtg_backward_raster")

    def backward_project(self, ws, params, poses, grads):
        pos, scale, rot, opacity, color, unstable = params
        check(lib().rtg_backward_project(self._plan, _ptr(ws), _ptr(pos), _ptr(scale), _ptr(rot), _ptr(color),
                                         _ptr(unstable), _ptr(poses), _ptr(grads["pos"]), _ptr(grads["scale"]),
                                         _ptr(grads["rot"]), _ptr(grads["opacity"]), _ptr(grads["color"]),
                                         _stream()), "rtg_backward_project")

    def loss_l1_into(self, ws, color, depth, color_gt, depth_gt, d_color, d_depth, loss_out, w_c=1.0, w_d=1.0):
        check(lib().rtg_loss_l1(self._plan, _ptr(ws), _ptr(color), _ptr(depth), _ptr(color_gt), _ptr(depth_gt),
                                float(w_c), float(w_d), _ptr(d_color), _ptr(d_depth), _ptr(loss_out), _stream()),
              "rtg_loss_l1")

    def backward_raster_l1(self, ws, color, depth, trans, index, color_gt, depth_gt):
        check(lib().rtg_backward_raster_l1(self._plan, _ptr(ws), _ptr(color), _ptr(depth), _ptr(trans),
                                           _ptr(index), _ptr(color_gt), _ptr(depth_gt), _stream()),
              "rtg_backward_raster_l1")

    def backward_project_l1(self, ws, params, poses, grads, loss_out, w_c=1.0, w_d=1.0):
        pos, scale, rot, opacity, color, unstable = params
        check(lib().rtg_backward_project_l1(self._plan, _ptr(ws), _ptr(pos), _ptr(scale), _ptr(rot),
                                            _ptr(color), _ptr(unstable), _ptr(poses), float(w_c), float(w_d),
                                            _ptr(grads["pos"]), _ptr(grads["scale"]), _ptr(grads["rot"]),
                                            _ptr(grads["opacity"]), _ptr(grads["color"]), _ptr(loss_out),
                                            _stream()), "rtg_backward_project_l1")

    def adam(self, params, grads, m, v, step, lr=(1e-3, 2e-3, 1e-3, 1e-3), betas=(0.9, 0.999), eps=1e-15):
        """lr = (position, scale, rotation, colour or SH band 0[, SH bands
        1..D]); the last defaults to 0.05 times the band-0 rate."""
        pos, scale, rot, opacity, color, unstable = params
        w = 10 + 3 * (1 if self.sh_degree == 0 else (self.sh_degree + 1) ** 2)
        _req(m, torch.float32, (self.n, w), "m")
        _req(v, torch.float32, (self.n, w), "v")
        lr_rest = float(lr[4]) if len(lr) > 4 else 0.05 * float(lr[3])
        check(lib().rtg_adam(self._plan, _ptr(pos), _ptr(scale), _ptr(rot), _ptr(color), _ptr(unstable),
                             _ptr(grads["pos"]), _ptr(grads["scale"]), _ptr(grads["rot"]), _ptr(grads["color"]),
                             _ptr(m), _ptr(v), _ptr(step), float(lr[0]), float(lr[1]), float(lr[2]),
                             float(lr[3]), lr_rest, float(betas[0]), float(betas[1]), float(eps), _stream()),
              "rtg_adam")

    def read_status(self, ws):
        """Device counters (synchronises the stream): pairs, pixels, items,
        overflow, big tiles, error flags, and under "status" the call's
        return code (capacity overflow and device errors are reported there,
        not raised)."""
        c = (ctypes.c_int64 * 11)()
        st = lib().rtg_read_status(self._plan, _ptr(ws), c, _stream())
        out = dict(zip(["pairs", "pixels", "items", "overflow", "big_tiles", "err", "eval_fwd", "blend_fwd",
                        "walk_bwd", "part_bwd", "restaged_blocks"], list(c)))
        out["status"] = int(st)
        return out

    # ---------------------------------------------------------- convenience
    def forward(self, params, poses, mask, ws=None):
        """project -> bin -> render; returns (color, depth, trans, index, ws)."""
        ws = self.new_workspace() if ws is None else ws
        self.project(ws, *params, poses)
        self.bin(ws, mask)
        out = self.alloc_outputs()
        self.render_into(ws, *out)
        return (*out, ws)

    def unstable_mask(self, params, poses, ws=None):
        ws = self.new_workspace() if ws is None else ws
        self.project(ws, *params, poses)
        m = torch.empty((self.frames, self.H, self.W), dtype=torch.uint8, device="cuda")
        return self.unstable_mask_into(ws, m)


class _RasterizeMasked(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, scale, rot, opacity, color, unstable, poses, mask, rast):
        params = (pos.detach(), scale.detach(), rot.detach(), opacity.detach(), color.detach(), unstable)
        C, D, T, I, ws = rast.forward(params, poses, mask)
        ctx.rast = rast
        ctx.ws = ws
        ctx.save_for_backward(*params[:5], unstable, poses, D, T, I)
        ctx.mark_non_differentiable(T, I)
        return C, D, T, I

    @staticmethod
    def backward(ctx, gC, gD, gT, gI):
        pos, scale, rot, opacity, color, unstable, poses, D, T, I = ctx.saved_tensors
        rast = ctx.rast
        F, H, W = rast.frames, rast.H, rast.W
        gC = torch.zeros((F, H, W, 3), device=D.device) if gC is None else gC.float().contiguous()
        gD = torch.zeros((F, H, W), device=D.device) if gD is None else gD.float().contiguous()
        grads = rast.alloc_grads(device=D.device)
        rast.backward_into(ctx.ws, (pos, scale, rot, opacity, color, unstable), poses, D, T, I, gC, gD, grads)
        return grads["pos"], grads["scale"], grads["rot"], grads["opacity"], grads["color"], None, None, None, None


def rasterize_masked(pos, scale, rot, opacity, color, unstable, poses, mask, rasterizer):
    """Differentiable masked render: returns (color, depth, trans, index);
    gradients flow to pos, scale, rot, opacity and color of the unstable
    Gaussians (stable rows get zero)."""
    return _RasterizeMasked.apply(pos, scale, rot, opacity, color, unstable, poses, mask, rasterizer)
