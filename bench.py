"""Benchmark of the masked forward+backward rasterizer on one MI355X.

One step = the whole hot path on one batch of synthetic input: projection,
binning (tile lists, pairs, per-tile sort), forward compositing, the L1
colour + depth loss with its upstream gradients, backward compositing and
the projection backward (plus Adam for the optimisation-loop workload).
Inputs are resident in HBM before the timed region; the step is captured
once in a HIP graph and replayed.

Prints ONE JSON line.  Default workload: 100k surface Gaussians in a 5x5x3 m
room, one 640x480 frame (fx = fy = 525), full mask, L1 loss against a
render of the scene with means jittered by N(0, 1 cm), gradients for all
Gaussians.  Other workloads (--workload c3/c4) are for the design notes.
"""
from __future__ import annotations

import argparse
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

# FP32 operations per unit of algorithmic work (counted from the kernels'
# arithmetic, see the design notes): a list entry tested against a pixel
# (offset, quadratic form: 10), a Gaussian blended into a colour (exp, opacity,
# weight, three colour FMAs, transmission: 12); backward: an entry walked back
# (decision 10 + exp/opacity 3) and a (pixel, Gaussian) contribution (~47).
FLOPS_FWD_EVAL, FLOPS_FWD_BLEND = 10.0, 12.0
FLOPS_BWD_WALK, FLOPS_BWD_PART = 13.0, 47.0

WORKLOADS = {
    "c2": "100k surface Gaussians, 5x5x3 m room, 1 frame 640x480 fx=fy=525, full mask, fwd+bwd, "
          "L1 colour+depth vs render of means jittered N(0,1cm), all Gaussians unstable",
    "c3": "500k surface Gaussians, 10x8x3 m multi-room, 1 frame 1200x680 fx=fy=600, 20% unstable in "
          "spatial patches, mask = M_unstable, fwd+bwd",
    "c4": "1M surface Gaussians, 14x11x3 m multi-room, 8 keyframes 1200x680 on a random walk, per-frame "
          "M_unstable masks, one batched fwd+bwd",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--items-per-pop", type=int, default=0)
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of graph replays")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle parity check")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="only run a device copy of this many MiB (counter calibration) and exit")
    return ap.parse_args()


def copy_probe(mb):
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); multi-GPU sharding is described in the "
              "design notes but not built", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe_mb:
        copy_probe(args.copy_probe_mb)
        return
    from paper_2404_19706_amd import Rasterizer
    from rtg_synth import jitter_means, make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    tw, th = (int(x) for x in args.tile.split("x"))
    t0 = time.time()
    cfg = make_config(args.workload)
    cam, sc, poses_np = cfg["cam"], cfg["scene"], cfg["poses"]
    N, F = len(sc["pos"]), poses_np.shape[0]
    log("workload %s: N=%d F=%d %dx%d (scene built in %.1fs)" % (args.workload, N, F, cam["width"],
                                                                   cam["height"], time.time() - t0))
    dev = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous()  # noqa
    params = (dev(sc["pos"]), dev(sc["scale"]), dev(sc["rot"]), dev(sc["opacity"]), dev(sc["color"]),
              dev(sc["unstable"], torch.uint8))
    poses = dev(poses_np, torch.float64)
    rast = Rasterizer(cam, N, F, max_pairs=max(1 << 22, 48 * N * F), tile_w=tw, tile_h=th,
                      items_per_pop=args.items_per_pop)
    ws = rast.new_workspace()
    H, W = cam["height"], cam["width"]

    # ---- inputs resident in HBM: mask, targets ----
    if cfg["mask"] == "full":
        mask = torch.ones((F, H, W), dtype=torch.uint8, device="cuda")
    else:
        mask = torch.empty((F, H, W), dtype=torch.uint8, device="cuda")
        rast.project(ws, *params, poses)
        rast.unstable_mask_into(ws, mask)
    jit = jitter_means(sc, 0.01, seed=1000 + int(args.workload[1:]))
    jparams = (dev(jit["pos"]),) + params[1:]
    Cgt, Dgt, _, _ = rast.alloc_outputs()
    Ttmp = torch.ones_like(Dgt)
    Itmp = torch.full_like(Dgt, -1, dtype=torch.int32)
    rast.project(ws, *jparams, poses)
    rast.bin(ws, torch.ones_like(mask))
    rast.render_into(ws, Cgt, Dgt, Ttmp, Itmp)
    torch.cuda.synchronize()
    mask_frac = float(mask.float().mean())
    log("mask fraction %.3f" % mask_frac)

    # ---- persistent buffers of the step ----
    C, D, T, I = rast.alloc_outputs()
    gC = torch.zeros_like(C)
    gD = torch.zeros_like(D)
    loss = torch.zeros(1, device="cuda")
    grads = rast.alloc_grads()

    def step(ev=None):
        def mark(k):
            if ev is not None:
                ev[k].record()
        mark(0)
        rast.project(ws, *params, poses)
        mark(1)
        rast.bin(ws, mask)
        mark(2)
        rast.render_into(ws, C, D, T, I)
        mark(3)
        rast.loss_l1_into(ws, C, D, Cgt, Dgt, gC, gD, loss)
        mark(4)
        rast.backward_raster(ws, D, T, I, gC, gD)
        mark(5)
        rast.backward_project(ws, params, poses, grads)
        mark(6)

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    st = rast.read_status(ws)
    if st["status"] != 0:
        raise RuntimeError("device status %s" % st)
    P_px = st["pixels"]
    log("pairs %d pixels %d items %d" % (st["pairs"], P_px, st["items"]))

    graph = None
    if not args.eager:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(3):
            graph.replay()
        torch.cuda.synchronize()

    # ---- timed region: K steps (graph replays), then K eager steps with
    # per-stage events on the launch stream for the per-kernel durations ----
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    stop.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / args.steps

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    names = ["project", "bin", "render", "loss", "backward_raster", "backward_project"]
    stage_ms = {n: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, n in enumerate(names)}
    eager_ms = float(np.mean([e[0].elapsed_time(e[6]) for e in evs]))

    # counters accumulated over every render/backward since the last project
    rast.project(ws, *params, poses)
    rast.bin(ws, mask)
    rast.render_into(ws, C, D, T, I)
    rast.loss_l1_into(ws, C, D, Cgt, Dgt, gC, gD, loss)
    rast.backward_raster(ws, D, T, I, gC, gD)
    rast.backward_project(ws, params, poses, grads)
    torch.cuda.synchronize()
    cnt = rast.read_status(ws)

    flops_f = FLOPS_FWD_EVAL * cnt["eval_fwd"] + FLOPS_FWD_BLEND * cnt["blend_fwd"]
    flops_b = FLOPS_BWD_WALK * cnt["walk_bwd"] + FLOPS_BWD_PART * cnt["part_bwd"]
    dom = max(("render", flops_f), ("backward_raster", flops_b), key=lambda x: stage_ms[x[0]])
    achieved = dom[1] / (stage_ms[dom[0]] * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": {"render": "k_raster_fwd", "backward_raster": "k_raster_bwd"}[dom[0]],
                "achieved": round(achieved, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                "work": {"eval_fwd": cnt["eval_fwd"], "blend_fwd": cnt["blend_fwd"], "walk_bwd": cnt["walk_bwd"],
                         "part_bwd": cnt["part_bwd"]}}
    mpix = P_px / (ms_step * 1e-3) / 1e6

    out = {"metric": "masked fwd+bwd Mpix/s (1e-4 rel err vs FP64 oracle)", "value": round(mpix, 3),
           "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "%s: %s" % (args.workload, WORKLOADS[args.workload]), "gaussians": N,
                      "frames": F, "width": W, "height": H, "tile": args.tile, "masked_pixels": P_px,
                      "mask_fraction": round(mask_frac, 4), "pairs": st["pairs"],
                      "mode": "eager" if graph is None else "hip_graph"},
           "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()}, "eager_ms_per_step": round(eager_ms, 4),
           "roofline": roofline}

    # ---- parity of the timed iteration against the oracle (sampled) ----
    if not args.no_check:
        out["check"] = parity_check(rast, cam, sc, poses_np, params, poses, mask, C, D, T, I, ws)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cam, sc, poses_np, mask.cpu().numpy(), args.cpu_seconds)
    print(json.dumps(out), flush=True)


def parity_check(rast, cam, sc, poses_np, params, poses, mask, C, D, T, I, ws, n_px=1500):
    """Forward values at sampled masked pixels of the timed iteration, and
    gradients of a sampled-pixel upstream, against the FP64 oracle."""
    import torch
    from oracle import oracle as orc

    rng = np.random.default_rng(123)
    m = mask.cpu().numpy()
    allpix = orc.masked_pixels(m)
    pix = allpix[rng.choice(len(allpix), min(n_px, len(allpix)), replace=False)]
    P = orc.make_params(cam, tile=(rast.cfg.tile_w, rast.cfg.tile_h))
    recs = orc.project(P, sc, poses_np)
    ref = orc.render(P, recs, sc, pix)
    f, x, y = pix[:, 0], pix[:, 1], pix[:, 2]
    Cn, Dn, Tn, In = (a.cpu().numpy() for a in (C, D, T, I))

    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a, float) - b) / max(np.linalg.norm(b), 1e-300))
    res = {"pixels": int(len(pix)), "color": rel(Cn[f, y, x], ref["color"]), "depth": rel(Dn[f, y, x], ref["depth"]),
           "trans": rel(Tn[f, y, x], ref["trans"]), "index_mismatch": int((In[f, y, x] != ref["index"]).sum())}
    gC = np.zeros(Cn.shape, np.float32)
    gD = np.zeros(Dn.shape, np.float32)
    gC[f, y, x] = rng.standard_normal((len(pix), 3)).astype(np.float32)
    gD[f, y, x] = rng.standard_normal(len(pix)).astype(np.float32)
    grads = rast.alloc_grads()
    rast.backward_into(ws, params, poses, D, T, I, torch.as_tensor(gC).cuda(), torch.as_tensor(gD).cuda(), grads)
    torch.cuda.synchronize()
    gref = orc.backward(P, recs, sc, poses_np, pix, gC[f, y, x], gD[f, y, x])
    for k in ("pos", "scale", "rot", "opacity", "color"):
        res["d_" + k] = rel(grads[k].cpu().numpy(), gref[k])
    res["pass"] = bool(res["index_mismatch"] == 0 and max(v for k, v in res.items()
                                                           if k not in ("pixels", "index_mismatch")) <= 1e-4)
    res = {k: (float("%.3g" % v) if isinstance(v, float) else v) for k, v in res.items()}
    log("parity:", res)
    return res


def cpu_baseline(cam, sc, poses_np, mask, seconds):
    """The FP64 oracle (as it stands) on a seeded sample of the masked
    pixels: projection of every Gaussian plus forward and backward of the
    sample, on all host threads."""
    from oracle import oracle as orc

    rng = np.random.default_rng(7)
    allpix = orc.masked_pixels(mask)
    P = orc.make_params(cam)

    def run(npx):
        pix = allpix[rng.choice(len(allpix), min(npx, len(allpix)), replace=False)]
        g = rng.standard_normal((len(pix), 3))
        gd = rng.standard_normal(len(pix))
        t = time.time()
        recs = orc.project(P, sc, poses_np)
        orc.render(P, recs, sc, pix)
        orc.backward(P, recs, sc, poses_np, pix, g, gd)
        return time.time() - t, len(pix)
    dt, n = run(200)
    target = int(min(len(allpix), max(200, 200 * seconds / max(dt, 1e-3))))
    dt, n = run(target)
    res = {"value": round(n / dt / 1e6, 6), "unit": "Mpix/s", "cores": orc.num_threads(), "kind": "oracle",
           "sample": "%d of %d masked pixels (seeded), projection of all %d Gaussians + forward + backward, "
                     "%.1f s" % (n, len(allpix), len(sc["pos"]), dt)}
    log("cpu baseline:", res)
    return res


if __name__ == "__main__":
    main()
