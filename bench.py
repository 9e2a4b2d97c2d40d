"""Benchmark of the masked forward+backward rasterizer on one MI355X.

One step = the whole hot path on one batch of synthetic input: projection,
binning (tile lists, pairs, per-tile sort), forward compositing, the L1
colour + depth loss with its upstream gradients (folded into the two
backward kernels: the compositing backward forms the upstream per pixel and
sums the loss terms, the projection backward scales and writes the loss),
backward compositing and the projection backward (plus masked Adam for the
optimisation-loop workload c5).  Inputs are resident in HBM before the timed region; the step
is captured once in a HIP graph and replayed.

Prints ONE JSON line.  Default workload (c5, the largest): 5M surface
Gaussians over a 30x20x3 m floor, 16 keyframes of 1200x680 (fx = fy = 600)
on a random walk, per-frame masks M_unstable of uneven size (5-60 % of the
image), L1 colour + depth loss against a render of the scene with means
jittered by N(0, 1 cm), gradients for the unstable Gaussians and masked Adam;
one step = one optimisation iteration, 100 of them timed.  The tile shape and
work-queue granularity are autotuned unless given.  The line also carries
the roofline of the dominant kernel, the FP64 oracle timed on a bounded
sample on the host cores (first two keyframes), and, as extra figures, the
single-frame workload (c2) and the batched-vs-per-frame comparison on the
8-keyframe workload (c4).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3

# FP32 operations per unit of the method's own work: a (pixel, Gaussian)
# pair blended into a colour forward (offset and quadratic form, exp,
# opacity, weight, three colour FMAs, transmission and the depth test: 18
# operations + 1 exp), and a (pixel, Gaussian) pair contributing to the
# gradients backward (45 + 1 exp).  List entries that a pixel tests without
# blending are tiling overhead and count for nothing.
FLOPS_FWD_BLEND = 19.0
FLOPS_BWD_PART = 46.0

WORKLOADS = {
    "c1": "2k Gaussians uniform in a 1 m cube 2 m ahead, 1 frame 128x96 fx=fy=100, full mask, forward only",
    "c2": "100k surface Gaussians, 5x5x3 m room, 1 frame 640x480 fx=fy=525, full mask, fwd+bwd, "
          "L1 colour+depth vs render of means jittered N(0,1cm), all Gaussians unstable",
    "c3": "500k surface Gaussians, 10x8x3 m multi-room, 1 frame 1200x680 fx=fy=600, 20% unstable in "
          "spatial patches, mask = M_unstable, fwd+bwd",
    "c4": "1M surface Gaussians, 14x11x3 m multi-room, 8 keyframes 1200x680 on a random walk, per-frame "
          "M_unstable masks, one batched fwd+bwd",
    "c5": "5M surface Gaussians, 30x20x3 m floor (walls, boxes, cylinders), 16 keyframes 1200x680, per-frame "
          "M_unstable masks, masked fwd+bwd + masked Adam per iteration",
}
STAGES = ["project", "bin", "render", "loss", "backward_raster", "backward_project", "adam"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 50; 100 iterations for c5)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default="auto", help="WxH tile shape or 'auto' (autotuned with the queue mode)")
    ap.add_argument("--items-per-pop", type=int, default=0, help="queue granularity when --tile is given")
    ap.add_argument("--static-share", type=int, default=0,
                    help="percent of the items handed out round robin before the queue, when --tile is given")
    ap.add_argument("--fwd-items-per-pop", type=int, default=-1,
                    help="the forward compositing kernel's own queue granularity (-1: as --items-per-pop)")
    ap.add_argument("--fwd-static-share", type=int, default=-1,
                    help="the forward compositing kernel's own round-robin share (-1: as --static-share)")
    ap.add_argument("--t-eps", type=float, default=None,
                    help="transmission below which a pixel's colour stops (library default if omitted)")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra figures (single-frame c2 line, batched-vs-per-frame on c4)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    a = ap.parse_args()
    if a.steps is None:
        a.steps = 100 if a.workload == "c5" else 50
    return a


def copy_probe(mb):
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))


# --------------------------------------------------------------------------
# workload set-up: scene, poses, mask and targets resident on the device

def build_workload(name):
    import torch
    from paper_2404_19706_amd.autotune import fit_rasterizer
    from rtg_synth import jitter_means, make_config

    t0 = time.time()
    cfg = make_config(name)
    cam, sc, poses_np = cfg["cam"], cfg["scene"], cfg["poses"]
    N, F = len(sc["pos"]), poses_np.shape[0]
    H, W = cam["height"], cam["width"]

    def dev(a, dt=torch.float32):
        return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous()
    params = (dev(sc["pos"]), dev(sc["scale"]), dev(sc["rot"]), dev(sc["opacity"]), dev(sc["color"]),
              dev(sc["unstable"], torch.uint8))
    poses = dev(poses_np, torch.float64)
    full = torch.ones((F, H, W), dtype=torch.uint8, device="cuda")
    # targets: a full-mask render of the scene with jittered means
    jit = jitter_means(sc, 0.01, seed=1000 + int(name[1:]))
    jparams = (dev(jit["pos"]),) + params[1:]
    r, ws, _ = fit_rasterizer(cam, N, F, jparams, poses, full)
    Cgt, Dgt, Tt, It = r.alloc_outputs()
    r.render_into(ws, Cgt, Dgt, Tt, It)
    if cfg["mask"] == "full":
        mask = full
    else:
        mask = torch.empty((F, H, W), dtype=torch.uint8, device="cuda")
        r.project(ws, *params, poses)
        r.unstable_mask_into(ws, mask)
    torch.cuda.synchronize()
    del r, ws, Tt, It, jparams
    torch.cuda.empty_cache()
    log("workload %s: N=%d F=%d %dx%d mask %.3f (built in %.1fs)" % (name, N, F, W, H, float(mask.float().mean()),
                                                                    time.time() - t0))
    return {"name": name, "cam": cam, "sc": sc, "poses_np": poses_np, "N": N, "F": F, "H": H, "W": W,
            "params": params, "poses": poses, "mask": mask, "Cgt": Cgt, "Dgt": Dgt}


class Step:
    """One pass of the hot path on a fitted plan, with its persistent
    buffers (outputs, upstream gradients, parameter gradients, Adam state)."""

    def __init__(self, wl, tile, sched=(0, 0), adam=False, fwd_only=False, t_eps=None):
        import torch
        from paper_2404_19706_amd.autotune import fit_rasterizer, sched_kw
        self.wl = wl
        extra = {} if t_eps is None else {"t_eps": t_eps}
        self.rast, self.ws, _ = fit_rasterizer(wl["cam"], wl["N"], wl["F"], wl["params"], wl["poses"], wl["mask"],
                                               tile_w=tile[0], tile_h=tile[1], **sched_kw(sched), **extra)
        self.C, self.D, self.T, self.I = self.rast.alloc_outputs()
        self.gC = torch.zeros_like(self.C)
        self.gD = torch.zeros_like(self.D)
        self.loss = torch.zeros(1, device="cuda")
        self.grads = self.rast.alloc_grads()
        self.adam = adam
        self.fwd_only = fwd_only
        if adam:
            self.m = torch.zeros((wl["N"], 13), device="cuda")
            self.v = torch.zeros((wl["N"], 13), device="cuda")
            self.t = torch.zeros(1, dtype=torch.int32, device="cuda")

    def __call__(self, ev=None, adam=None):
        r, ws, wl = self.rast, self.ws, self.wl

        def mark(k):
            if ev is not None:
                ev[k].record()
        mark(0)
        r.project(ws, *wl["params"], wl["poses"])
        mark(1)
        r.bin(ws, wl["mask"])
        mark(2)
        r.render_into(ws, self.C, self.D, self.T, self.I)
        mark(3)
        if self.fwd_only:
            for k in range(4, 8):
                mark(k)
            return
        # the L1 loss is folded into the backward: the compositing backward
        # forms its upstream per pixel at unit scale and sums the loss terms,
        # the projection backward applies the scales and writes the loss
        mark(4)
        r.backward_raster_l1(ws, self.C, self.D, self.T, self.I, wl["Cgt"], wl["Dgt"])
        mark(5)
        r.backward_project_l1(ws, wl["params"], wl["poses"], self.grads, self.loss)
        mark(6)
        if self.adam if adam is None else adam:
            r.adam(wl["params"], self.grads, self.m, self.v, self.t)
        mark(7)


def capture(fn):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    return g


def time_region(fn, steps):
    """ms per call of fn over exactly `steps` calls, between two
    synchronisations."""
    import torch
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


# --------------------------------------------------------------------------
# batched keyframes vs per-frame passes

def compare_batched_plain(wl, steps, tile, sched):
    """The F-keyframe batch as one pass (one launch per kernel for all
    frames, graph-captured) against F single-frame passes of the same
    frames, eager and graph-captured.  Forward outputs must be
    bit-identical; gradients of the same upstream agree to rounding."""
    import torch
    from paper_2404_19706_amd.autotune import fit_rasterizer, sched_kw

    name = wl["name"]
    F = wl["F"]
    b = Step(wl, tile, sched)
    b()
    torch.cuda.synchronize()
    gb = capture(b)
    ms_b = time_region(gb.replay, steps)
    ms_b_eager = time_region(b, steps)

    P = wl["params"]

    def make_plains(sch):
        out = []
        for f in range(F):
            r, ws, _ = fit_rasterizer(wl["cam"], wl["N"], 1, wl["params"], wl["poses"][f:f + 1],
                                      wl["mask"][f:f + 1], tile_w=tile[0], tile_h=tile[1], **sched_kw(sch))
            out.append({"r": r, "ws": ws, "grads": r.alloc_grads(), "loss": torch.zeros(1, device="cuda")})
        return out

    def plain(upstream=None):
        for f, p in enumerate(plains):
            r, ws = p["r"], p["ws"]
            sl = slice(f, f + 1)
            r.project(ws, *P, wl["poses"][sl])
            r.bin(ws, wl["mask"][sl])
            r.render_into(ws, b.C[sl], b.D[sl], b.T[sl], b.I[sl])
            if upstream is None:
                r.backward_raster_l1(ws, b.C[sl], b.D[sl], b.T[sl], b.I[sl], wl["Cgt"][sl], wl["Dgt"][sl])
                r.backward_project_l1(ws, P, wl["poses"][sl], p["grads"], p["loss"])
            else:
                r.backward_raster(ws, b.D[sl], b.T[sl], b.I[sl], upstream[0][sl], upstream[1][sl])
                r.backward_project(ws, P, wl["poses"][sl], p["grads"])

    # the per-frame passes take the faster of the batch's schedule and plain
    # round robin (a single frame has few work items for the queue)
    best = None
    for sch in dict.fromkeys([tuple(sched), (0, 0)]):
        plains = make_plains(sch)
        plain()
        torch.cuda.synchronize()
        ms_e = time_region(plain, steps)
        g = capture(plain)
        ms_g = time_region(g.replay, steps)
        if best is None or ms_g < best[2]:
            best = (sch, ms_e, ms_g, plains, g)
        else:
            del g, plains
    plain_sched, ms_p_eager, ms_p, plains, gp = best

    # same outputs: forward bit-identical, gradients of one upstream summed
    b()
    b.rast.loss_l1_into(b.ws, b.C, b.D, wl["Cgt"], wl["Dgt"], b.gC, b.gD, b.loss)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (b.C, b.D, b.T, b.I)]
    up = (b.gC.clone(), b.gD.clone())
    gref = {k: v.clone() for k, v in b.grads.items()}
    for p in plains:
        for v in p["grads"].values():
            v.zero_()
    plain(upstream=up)
    torch.cuda.synchronize()
    same_fwd = all(bool(torch.equal(x, y)) for x, y in zip(ref, (b.C, b.D, b.T, b.I)))
    grel = 0.0
    for k in gref:
        s = sum(p["grads"][k].double() for p in plains)
        grel = max(grel, float((s - gref[k].double()).norm() / gref[k].double().norm().clamp_min(1e-300)))
    res = {"workload": "%s: %s" % (name, WORKLOADS[name]), "frames": F, "tile": "%dx%d" % tile,
           **sched_kw(sched), "batched_graph_ms": round(ms_b, 4),
           "batched_eager_ms": round(ms_b_eager, 4),
           "per_frame_eager_ms": round(ms_p_eager, 4), "per_frame_graph_ms": round(ms_p, 4),
           "per_frame_schedule": list(plain_sched),
           "speedup_vs_per_frame_eager": round(ms_p_eager / ms_b, 3),
           "speedup_vs_per_frame_graph": round(ms_p / ms_b, 3),
           "forward_bit_identical": same_fwd, "grad_rel_diff": float("%.3g" % grel),
           "frame_mask_fractions": [round(float(x), 4) for x in wl["mask"].float().mean((1, 2)).cpu()]}
    log("batched vs per-frame:", res)
    del gb, gp, plains, b
    torch.cuda.empty_cache()
    return res


# --------------------------------------------------------------------------

def traffic_from_profile(kernel, workload, tile):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload and tile shape, or None when there is none or the kernel
    source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%dx%d.txt" % (kernel, workload, tile[0], tile[1]))
    src = os.path.join(ROOT, "paper_2404_19706_amd", "csrc", "raster.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if kv.get("source_sha256_16") != digest:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measure(wl, args, tile_arg="auto", sched_arg=(0, 0), steps=None, warmup=None):
    """Time the step of one workload: autotune (unless a tile is given),
    warm up, capture, time exactly `steps` graph replays, then per-stage
    eager timings and the work counters of one pass.  Returns the numbers of
    the bench line for this workload."""
    import torch
    from paper_2404_19706_amd.autotune import Autotuner, sched_kw

    name = wl["name"]
    N, F, H, W = wl["N"], wl["F"], wl["H"], wl["W"]
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    adam = name == "c5"
    fwd_only = name == "c1"

    tune = None
    if tile_arg == "auto":
        tune = Autotuner(reps=5).tune(wl["cam"], wl["params"], wl["poses"], wl["mask"], wl["Cgt"], wl["Dgt"])
        tile = (tune["tile_w"], tune["tile_h"])
        sched = (tune["items_per_pop"], tune["static_share"], tune["fwd_items_per_pop"], tune["fwd_static_share"])
        log("autotune %s:" % name, json.dumps(tune))
    else:
        tile, sched = tuple(int(x) for x in tile_arg.split("x")), tuple(sched_arg)

    torch.cuda.reset_peak_memory_stats()
    step = Step(wl, tile, sched, adam=adam, fwd_only=fwd_only, t_eps=args.t_eps)
    for _ in range(max(warmup, 1)):
        step()
    torch.cuda.synchronize()
    st = step.rast.read_status(step.ws)
    check_status(st, "after warm-up")
    P_px = st["pixels"]
    log("%s: pairs %d pixels %d items %d" % (name, st["pairs"], P_px, st["items"]))

    graph = None if args.eager else capture(step)
    # ---- timed region: exactly `steps` steps ----
    ms_step = time_region(graph.replay if graph is not None else step, steps)
    peak_mem = torch.cuda.max_memory_allocated()
    # an overflow of the pair capacity during the replays (c5's Adam moves
    # the Gaussians) would skip the compositing: the line is void then
    check_status(step.rast.read_status(step.ws), "after the timed steps")

    # ---- per-stage durations: eager steps with events on the launch stream ----
    nst = 8
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nst)] for _ in range(steps)]
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    check_status(step.rast.read_status(step.ws), "after the per-stage steps")
    stage_ms = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, n in enumerate(STAGES)}
    if not adam:
        stage_ms.pop("adam")
    stage_ms.pop("loss")   # folded into the two backward stages
    if fwd_only:
        for k in ("backward_raster", "backward_project"):
            stage_ms.pop(k)
    eager_ms = float(np.mean([e[0].elapsed_time(e[nst - 1]) for e in evs]))

    # work counters of one pass (accumulated per wave since the last projection)
    step(adam=False)
    torch.cuda.synchronize()
    cnt = step.rast.read_status(step.ws)
    check_status(cnt, "after the counter pass")

    # VALU work of the method itself: 18 FP32 ops + 1 exp per blended
    # (pixel, Gaussian) pair forward, 45 + 1 per contributing pair backward;
    # list entries a pixel tests without blending are tiling overhead and
    # are not counted
    flops_f = FLOPS_FWD_BLEND * cnt["blend_fwd"]
    flops_b = FLOPS_BWD_PART * cnt["part_bwd"]
    dom = max(("render", flops_f), ("backward_raster", flops_b), key=lambda x: stage_ms.get(x[0], 0.0))
    kname = {"render": "k_raster_fwd", "backward_raster": "k_raster_bwd"}[dom[0]]
    achieved = dom[1] / (stage_ms[dom[0]] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": kname, "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic_from_profile(kname, name, tile),
                "kernel_ms": round(stage_ms[dom[0]], 4),
                "flops_per_unit": FLOPS_FWD_BLEND if dom[0] == "render" else FLOPS_BWD_PART,
                "work": {"eval_fwd": cnt["eval_fwd"], "blend_fwd": cnt["blend_fwd"], "walk_bwd": cnt["walk_bwd"],
                         "part_bwd": cnt["part_bwd"]},
                "tested_per_blended_fwd": round(cnt["eval_fwd"] / max(cnt["blend_fwd"], 1), 3),
                "walked_per_contribution_bwd": round(cnt["walk_bwd"] / max(cnt["part_bwd"], 1), 3)}
    mpix = P_px / (ms_step * 1e-3) / 1e6

    # algorithmic HBM bytes of one step (what the method must move; per-tile
    # re-reads of pair records are reuse and not counted): parameters 57 N,
    # projected records written and read 2 x 64 N_v, pairs written, sorted
    # and read 3 x 12 K, tile ranges 8 per (frame, tile), the mask F H W,
    # pixel outputs 28 P, loss reads of targets 16 P, backward pixel state
    # and upstream 44 P, camera-space gradient rows 60 N_u per frame, the
    # projection backward (57 + 64 + 60 + 56) N_u, Adam 7 x 56 N_u
    vis = step.ws[step.rast.layout["vis"]:step.rast.layout["vis"] + 4 * N].view(torch.int32)
    bits = torch.stack([(vis >> k) & 1 for k in range(F)]).sum(0)
    n_v = int(bits.sum())
    unst = wl["params"][5] != 0
    n_u = int(((bits > 0) & unst).sum())
    n_uf = int((bits * unst).sum())
    tiles = F * ((W + tile[0] - 1) // tile[0]) * ((H + tile[1] - 1) // tile[1])
    b_alg = 57 * N + 128 * n_v + 36 * st["pairs"] + 8 * tiles + F * H * W + 28 * P_px
    if not fwd_only:
        b_alg += (16 + 44) * P_px + 60 * n_uf + (57 + 64 + 60 + 56) * n_u + (7 * 56 * n_u if adam else 0)
    hbm_step = {"algorithmic_bytes": int(b_alg), "achieved_gbs": round(b_alg / (ms_step * 1e-3) / 1e9, 2),
                "peak_gbs": HBM_PEAK_GBS, "frac": round(b_alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                "visible_slots": n_v, "unstable_visible": n_u}

    fr = [round(float(x), 4) for x in wl["mask"].float().mean((1, 2)).cpu()]
    cfg = {"workload": "%s: %s" % (name, WORKLOADS[name]), "gaussians": N, "frames": F,
           "width": W, "height": H, "tile": "%dx%d" % tile, **sched_kw(sched),
           "t_eps": float(step.rast.cfg.t_eps), "masked_pixels": P_px,
           "mask_fraction": round(float(wl["mask"].float().mean()), 4), "frame_mask_fractions": fr,
           "pairs": st["pairs"], "mode": "eager" if graph is None else "hip_graph"}
    res = {"ms_per_step": ms_step, "value": mpix, "config": cfg, "stage_ms": stage_ms, "eager_ms": eager_ms,
           "peak_mem": peak_mem, "roofline": roofline, "hbm_step": hbm_step, "tile": tile, "sched": sched}
    if tune is not None:
        res["autotune"] = {k: tune[k] for k in ("tile_w", "tile_h", "items_per_pop", "static_share",
                                                "fwd_items_per_pop", "fwd_static_share", "table", "tune_seconds")}
    del graph, step
    torch.cuda.empty_cache()
    return res


def measure_mapping(wl, reps=20):
    """The steps either side of the optimisation (Sec. 3.2) on the first
    keyframe of a workload: render it with every pixel masked, then time
    Gaussian adding against the input frame (the workload's target images:
    a render of the scene with jittered means; depth <= 0 invalid), the
    state update and the confidence count over all Gaussians, and the
    removal compaction of the nine per-Gaussian arrays.  Returns a dict of
    mean milliseconds per call and counts."""
    import torch
    from paper_2404_19706_amd import mapping as M
    from paper_2404_19706_amd.autotune import fit_rasterizer

    cam, N, H, W = wl["cam"], wl["N"], wl["H"], wl["W"]
    full = torch.ones((1, H, W), dtype=torch.uint8, device="cuda")
    r, ws, st = fit_rasterizer(cam, N, 1, wl["params"], wl["poses"][:1].contiguous(), full)
    C, D, T, I = r.alloc_outputs()
    r.render_into(ws, C, D, T, I)
    check_status(r.read_status(ws), "mapping render")
    Cin, Din = wl["Cgt"][0].contiguous(), wl["Dgt"][0].contiguous()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    rand = torch.rand((H, W), device="cuda", generator=gen)
    cap = N + H * W
    state = M.alloc_state(cap)
    for k, t in zip(("pos", "scale", "rot", "opacity", "color", "unstable"), wl["params"]):
        state[k][:N] = t
    state["eta"][:N] = torch.randint(0, 150, (N,), device="cuda", generator=gen, dtype=torch.int32)
    state["err"][:N] = torch.randint(0, 6, (N,), device="cuda", generator=gen, dtype=torch.int32)
    state["tstamp"][:N] = torch.randint(0, 300, (N,), device="cuda", generator=gen, dtype=torch.int32)
    dcol = torch.randn((N, 3), device="cuda", generator=gen)
    prm = M.adding_params()
    pose0 = wl["poses"][0].contiguous()
    dst = M.alloc_state(cap)
    names = [f[0] for f in M.STATE_FIELDS]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            out = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, out

    add_ms, counts = timed(lambda: M.add_gaussians(cam, prm, pose0, Cin, Din, C[0], D[0], T[0], I[0], rand, 300, N,
                                                   state))
    n_add, n_cand = (int(v) for v in counts.cpu())
    n_all = N + n_add
    state_ms, keep = timed(lambda: M.state_update(cam, prm, Cin, Din, C[0], D[0], I[0], 300, n_all, state))
    conf_ms, _ = timed(lambda: M.confidence_count(N, state["unstable"], dcol, state["eta"]))
    comp_ms, nout = timed(lambda: M.compact_rows(n_all, keep, [state[k] for k in names], [dst[k] for k in names]))
    row_bytes = sum(state[k][0].numel() * state[k].element_size() for k in names)
    # algorithmic bytes: adding reads the two frames, the render and the
    # random numbers (48 B per pixel) and writes the new rows; the state
    # update reads a pixel's render and frame (36 B) and per Gaussian reads
    # and writes its 13 bytes of state plus its flag and keep bytes; the
    # compaction reads the keep byte and moves each kept row
    px = H * W
    add_b = 48 * px + row_bytes * n_add
    state_b = 36 * px + (2 * 13 + 3) * n_all
    comp_b = n_all + 2 * row_bytes * int(nout.item())
    # the rest of the mapping iteration (Eq. 8-9, global optimisation) and
    # tracking (Eq. 10) on the same frame
    from paper_2404_19706_amd import tracking
    un = wl["params"][5]
    transparent = (torch.rand(N, device="cuda", generator=gen) < 0.2).to(torch.uint8)
    cur = {k: wl["params"][i] for i, k in ((0, "pos"), (1, "scale"), (2, "rot"))}
    init = {k: (v + 1e-3 * torch.randn(v.shape, device="cuda", generator=gen)).contiguous() for k, v in cur.items()}
    rgrads = {k: torch.zeros_like(v) for k, v in cur.items()}
    rloss = torch.zeros(1, dtype=torch.float64, device="cuda")
    reg_ms, _ = timed(lambda: M.reg_l2(1000.0, transparent, un, cur, init, rgrads, rloss))
    fcur = {k: state[k][:N].clone() for k in ("pos", "scale", "rot", "color")}
    fprev = {k: v + 1e-3 for k, v in fcur.items()}
    eta_prev = state["eta"][:N].clone()
    eta_cur = eta_prev + torch.randint(0, 50, (N,), device="cuda", generator=gen, dtype=torch.int32)
    fuse_ms, _ = timed(lambda: M.fuse(eta_prev, eta_cur, fprev, fcur))
    sel_mask = torch.empty((1, H, W), dtype=torch.uint8, device="cuda")
    sel_ms, _ = timed(lambda: M.select_top_error(C, Cin[None].contiguous(), 0.4, sel_mask))
    nrm = torch.zeros((1, H, W, 3), device="cuda")
    nrm_ms, _ = timed(lambda: r.render_normals_into(ws, nrm))
    icp_ms, pose_t = timed(lambda: tracking.icp(cam, Din, D[0].contiguous(), nrm[0].contiguous(), pose0, pose0))
    out_iter = {"reg_l2_ms": round(reg_ms, 4), "fuse_ms": round(fuse_ms, 4), "select_top40_ms": round(sel_ms, 4),
                "render_normals_ms": round(nrm_ms, 4), "icp_ms": round(icp_ms, 4),
                "icp_iterations": 19, "selected_pixels": int(sel_mask.sum().item())}
    out = {"frame": "keyframe 0 of the workload, %dx%d, rendered with every pixel masked; input frame = the "
                    "render of the jittered-means scene" % (W, H),
           "gaussians": N, "pixels_qualified": n_cand, "rows_added": n_add, "rows_kept": int(nout.item()),
           "add_ms": round(add_ms, 4), "state_update_ms": round(state_ms, 4), "confidence_count_ms": round(conf_ms, 4),
           "compact_ms": round(comp_ms, 4),
           "hbm_gbs": {"add": round(add_b / add_ms / 1e6, 1), "state_update": round(state_b / state_ms / 1e6, 1),
                       "compact": round(comp_b / comp_ms / 1e6, 1)},
           "iteration_and_tracking": out_iter}
    log("mapping steps:", out)
    del r, ws, state, dst
    torch.cuda.empty_cache()
    return out


def check_status(st, where):
    if st["status"] != 0 or st["overflow"] or st["err"]:
        raise RuntimeError("device status %s %s: the measurement is void" % (st, where))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the rasterizer runs on one GPU only (--gpus 1); sharding over several GPUs is "
              "described in the design notes but not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2404_19706_amd.autotune import sched_kw
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)
        return

    wl = build_workload(args.workload)
    m = measure(wl, args, args.tile, (args.items_per_pop, args.static_share, args.fwd_items_per_pop,
                                      args.fwd_static_share))
    fwd_only = args.workload == "c1"
    metric = "masked fwd+bwd Mpix/s (1e-4 rel err vs FP64 oracle)"
    if fwd_only:
        metric = "masked fwd Mpix/s (1e-4 rel err vs FP64 oracle)"
    out = {"metric": metric, "value": round(m["value"], 3),
           "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(m["ms_per_step"], 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": m["config"],
           "stage_ms": {k: round(v, 4) for k, v in m["stage_ms"].items()},
           "eager_ms_per_step": round(m["eager_ms"], 4),
           "peak_device_memory_gib": round(m["peak_mem"] / 2 ** 30, 3), "roofline": m["roofline"],
           "hbm_step": m["hbm_step"]}
    if "autotune" in m:
        out["autotune"] = m["autotune"]

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds, frames=2 if wl["F"] > 2 else None)

    if not args.no_extra:
        extra = {}
        extra["mapping"] = measure_mapping(wl)
        del wl
        torch.cuda.empty_cache()
        # the single-frame workload as a second line of figures
        if args.workload != "c2":
            w2 = build_workload("c2")
            m2 = measure(w2, args, "auto", steps=50, warmup=10)
            extra["c2"] = {"workload": m2["config"]["workload"], "ms_per_step": round(m2["ms_per_step"], 4),
                           "value": round(m2["value"], 3), "unit": "Mpix/s", "tile": m2["config"]["tile"],
                           **sched_kw(m2["sched"]), "stage_ms": {k: round(v, 4) for k, v in m2["stage_ms"].items()},
                           "roofline": m2["roofline"], "hbm_step": m2["hbm_step"]}
            del w2
            torch.cuda.empty_cache()
        # batched keyframes vs per-frame passes on the 8-keyframe workload
        w4 = build_workload("c4")
        from paper_2404_19706_amd.autotune import Autotuner
        t4 = Autotuner(reps=3).tune(w4["cam"], w4["params"], w4["poses"], w4["mask"], w4["Cgt"], w4["Dgt"])
        out["batched_vs_plain"] = compare_batched_plain(w4, 20, (t4["tile_w"], t4["tile_h"]),
                                                        (t4["items_per_pop"], t4["static_share"],
                                                         t4["fwd_items_per_pop"], t4["fwd_static_share"]))
        out["extra"] = extra
    print(json.dumps(out), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds, frames=None):
    """The FP64 oracle (as it stands) on a seeded sample of the masked
    pixels: projection of every Gaussian plus forward and backward of the
    sample, on all host threads, then a smaller sample on one thread.  With
    `frames`, only the first `frames` keyframes are projected and sampled
    (a labelled subset of a batch too large for the oracle).  The sample size
    is chosen from a calibration run so that the timed run takes about
    `seconds`."""
    from oracle import oracle as orc

    sc, cam, poses_np = wl["sc"], wl["cam"], wl["poses_np"]
    F = wl["F"] if frames is None else min(frames, wl["F"])
    poses_np = poses_np[:F]
    mask = wl["mask"][:F].cpu().numpy()
    rng = np.random.default_rng(7)
    allpix = orc.masked_pixels(mask)
    P = orc.make_params(cam)
    threads = orc.num_threads()

    t = time.time()
    recs = orc.project(P, sc, poses_np)
    t_proj = time.time() - t

    def run(npx):
        pix = allpix[rng.choice(len(allpix), min(npx, len(allpix)), replace=False)]
        g = rng.standard_normal((len(pix), 3))
        gd = rng.standard_normal(len(pix))
        t = time.time()
        orc.render(P, recs, sc, pix)
        orc.backward(P, recs, sc, poses_np, pix, g, gd)
        return time.time() - t, len(pix)
    # grow the sample until it takes an eighth of the budget, then scale it
    n_try = 400
    dt, n = run(n_try)
    while dt < seconds / 8 and n < len(allpix):
        n_try *= 4
        dt, n = run(n_try)
    target = int(min(len(allpix), max(n, n * max(seconds - t_proj, 1.0) / max(dt, 1e-6))))
    t = time.time()
    orc.project(P, sc, poses_np)
    t_proj = time.time() - t
    dt, n = run(target)
    total = dt + t_proj
    # one thread: projection and a sample sized for about a quarter of the budget
    orc.set_num_threads(1)
    try:
        t = time.time()
        orc.project(P, sc, poses_np)
        t_proj1 = time.time() - t
        n1 = int(max(16, min(len(allpix), n * (seconds / 4) / max(dt * threads, 1e-6))))
        dt1, n1 = run(n1)
    finally:
        orc.set_num_threads(threads)
    # per-pixel time plus the projection, per pixel of the multi-thread sample
    one = n / (dt1 / n1 * n + t_proj1)
    res = {"value": round(n / total / 1e6, 6), "unit": "Mpix/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "one_thread_value": round(one / 1e6, 7),
           "sample": "%d of %d masked pixels (seeded) of keyframes 0-%d of %d, projection of all %d Gaussians into "
                     "those keyframes (%.1f s) + forward + backward of the sample (%.1f s); one thread: %d pixels "
                     "(%.1f s) + projection (%.1f s), scaled to the same sample"
                     % (n, len(allpix), F - 1, wl["F"], len(sc["pos"]), t_proj, dt, n1, dt1, t_proj1)}
    log("cpu baseline:", res)
    return res


if __name__ == "__main__":
    main()
