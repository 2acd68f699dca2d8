"""Benchmark: block-wise LoD render of a 20M-Gaussian synthetic city at 1600x900.

One step = LoD-render every evaluation view once (48 views: heights 50/150/400 m,
8 positions each, pitch -90 and -45 degrees), one frame at a time:
    lod_select -> preprocess -> bin_sort -> rasterize_fwd
replayed from a HIP graph.  `value` = frames per second over the step.

Also reported: per-view FPS distribution (mean / median / min, as in the paper's
Fig. 5), the plain comparator (same library, LoD off: every block at the finest
level, eager launches), fwd+bwd ms/view for LoD and plain, the roofline of the
dominant kernel measured with HIP events, and the CPU oracle's frame time.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 20000000]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 VALU peak without packed-FP32 instructions (which this build does not
# emit): 256 CUs x 64 FMA lanes per clock x 2 flops x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 78.6
# algorithmic FP32 work of one (pixel, Gaussian) evaluation inside the footprint:
# offset (4), conic quadratic form (7), exp (1), alpha (1), transmittance (2),
# alpha*T (1), colour update (3 FMA = 6)
FLOPS_PER_EVAL = 22


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=20_000_000, help="finest-level Gaussians")
    ap.add_argument("--n-xy", type=int, default=8, help="camera positions per height")
    ap.add_argument("--bwd-views", type=int, default=12, help="views used for the fwd+bwd timing")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--frames-only", action="store_true", help="only the timed LoD frames (for profilers)")
    ap.add_argument("--bwd-only", action="store_true", help="only the LoD fwd+bwd loop (for profilers)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 512 MiB device-to-device copies (reference for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2404_01133_amd import gs, render, synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    W, H = 1600, 900
    thresholds = (200.0, 500.0)
    t0 = time.time()
    fine, block_id, u, cells = synth.city_finest(args.n, seed=2)
    log("generated %d Gaussians in %.1fs" % (args.n, time.time() - t0))
    scene = render.DeviceScene.from_finest(fine, block_id, u, cells, device=dev)
    scene.compute_bounds(4.0)
    torch.cuda.synchronize()
    n_stored = sum(lv.n for lv in scene.levels)
    log("scene on device: %d stored Gaussians, %d blocks (%.1fs)" % (n_stored, scene.n_blocks, time.time() - t0))
    cams = synth.city_views(seed=2, n_xy=args.n_xy, width=W, height=H)
    V = len(cams)
    cams_all = gs.cameras_to_device(cams, dev)
    cam_slot = [cams_all[v * 152:(v + 1) * 152] for v in range(V)]

    # ---- capacities from one eager pass over every view -------------------------
    frame = render.Frame(scene.n_blocks, 1, W, H, scene.max_records_per_view(), 1 << 22, device=dev)
    stats = []
    evals = []
    for v in range(V):
        render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds)
        c = frame.host_counts()
        stats.append(c)
        # (pixel, Gaussian) evaluations the compositing must do: sum of the visible footprints' areas
        nr = c["records"]
        rec = frame.records[: nr * gs.record_bytes()].view(torch.int32).view(nr, 12)
        w = ((rec[:, 2] >> 16) & 0xFFFF).to(torch.int64) + 1
        h = ((rec[:, 3] >> 16) & 0xFFFF).to(torch.int64) + 1
        evals.append(int(((w * h) * (frame.tiles_touched[:nr] > 0)).sum().item()))
    n_sel = np.array([s["records"] for s in stats])
    n_vis = np.array([s["visible"] for s in stats])
    n_pairs = np.array([s["pairs"] for s in stats])
    n_eval = np.array(evals, dtype=np.float64)
    log("per view: N_sel mean %.0f (max %d), N_vis mean %.0f, pairs mean %.0f (max %d)" %
        (n_sel.mean(), n_sel.max(), n_vis.mean(), n_pairs.mean(), n_pairs.max()))

    if args.bwd_only:
        grads = [lv.zeros_like() for lv in scene.levels]
        target = torch.rand((1, 3, H, W), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
        for _ in range(2):
            for v in range(0, V, max(1, V // args.bwd_views)):
                render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, check=False)
                d = torch.sign(frame.rgb - target) / frame.rgb.numel()
                render.backward_frame(scene, frame, cam_slot[v], d, grads)
        torch.cuda.synchronize()
        print(json.dumps({"bwd_only": True}))
        return

    # ---- HIP graph of one step (all views, one frame each) -------------------------
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        render.render_frame(scene, frame, cam_slot[0], thresholds=thresholds, check=False)  # warm the stream
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            for v in range(V):
                render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, check=False)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_total / args.steps
    fps = V * args.steps / t_total
    if frame.host_counts()["flags"]:
        raise RuntimeError("capacity flag raised during the timed frames: %s" % frame.host_counts())
    log("LoD graph: %.3f ms/step, %.1f FPS" % (ms_per_step, fps))
    if args.copy_calibration:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.frames_only:
        print(json.dumps({"metric": "FPS", "value": fps, "ms_per_step": ms_per_step,
                          "n_sel_mean": float(n_sel.mean()), "n_vis_mean": float(n_vis.mean()),
                          "pairs_mean": float(n_pairs.mean())}))
        return

    # ---- per-view FPS distribution (one graph per view) ----------------------------
    per_view_ms = []
    with torch.cuda.stream(stream):
        for v in range(V):
            gv = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gv, stream=stream):
                render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, check=False)
            for _ in range(2):
                gv.replay()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 10
            e0.record(stream)
            for _ in range(reps):
                gv.replay()
            e1.record(stream)
            e1.synchronize()
            per_view_ms.append(e0.elapsed_time(e1) / reps)
            del gv
    per_view_ms = np.array(per_view_ms)
    fps_views = 1e3 / per_view_ms

    # ---- dominant kernels timed with HIP events (eager, on their own stream) -------
    kern_ms = {"preprocess": [], "rasterize_fwd": [], "bin_sort": []}
    blocks = scene.blocks_struct()
    with torch.cuda.stream(stream):
        for v in range(V):
            c = cam_slot[v]
            gs.lod_select(blocks, thresholds, gs.GS_LOD_BLOCKWISE, c, 1, frame.level, frame.offsets, frame.counts,
                          stream)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record(stream)
            gs.preprocess([lv.struct() for lv in scene.levels], blocks, frame.level, frame.offsets, c, 1, W, H, 3,
                          frame.tuning, frame.record_capacity, frame.records, frame.depth_keys, frame.tiles_touched,
                          frame.counts, stream)
            ev[1].record(stream)
            gs.bin_sort(frame.records, frame.depth_keys, frame.tiles_touched, 1, W, H, frame.tuning,
                        frame.record_capacity, frame.pair_capacity, frame.pair_tiles, frame.pair_records,
                        frame.tile_ranges, frame.counts, frame.sort_ws, stream)
            ev[2].record(stream)
            gs.rasterize_fwd(frame.records, frame.pair_records, frame.tile_ranges, 1, W, H, (0.0, 0.0, 0.0),
                             frame.tuning, frame.rgb, frame.T, frame.n_last, stream)
            ev[3].record(stream)
            ev[3].synchronize()
            kern_ms["preprocess"].append(ev[0].elapsed_time(ev[1]))
            kern_ms["bin_sort"].append(ev[1].elapsed_time(ev[2]))
            kern_ms["rasterize_fwd"].append(ev[2].elapsed_time(ev[3]))
    pre_ms = float(np.mean(kern_ms["preprocess"]))
    # preprocess algorithmic bytes per launch: 12 B centre + 8 B (depth key, tiles touched) per selected record,
    # 224 B (rotation, scale, opacity, SH) read + 48 B record written per visible record
    pre_bytes = float(np.mean(20.0 * n_sel + 272.0 * n_vis))
    pre_gbs = pre_bytes / (pre_ms * 1e-3) / 1e9
    ras_ms = float(np.mean(kern_ms["rasterize_fwd"]))
    ras_flops = float(np.mean(n_eval)) * FLOPS_PER_EVAL
    ras_tflops = ras_flops / (ras_ms * 1e-3) / 1e12
    log("kernel ms (mean over views): preprocess %.4f, bin_sort %.4f, rasterize_fwd %.4f" %
        (pre_ms, np.mean(kern_ms["bin_sort"]), np.mean(kern_ms["rasterize_fwd"])))

    out_extra = {}
    # ---- plain comparator: LoD off, every block at the finest level, eager ----------
    if not args.no_plain:
        pframe = render.Frame(scene.n_blocks, 1, W, H, scene.n_finest, 1 << 23, device=dev)
        render.render_frame(scene, pframe, cam_slot[0], mode=gs.GS_LOD_ALL_FINEST, thresholds=())
        for v in range(V):
            render.render_frame(scene, pframe, cam_slot[v], mode=gs.GS_LOD_ALL_FINEST, thresholds=())
        torch.cuda.synchronize()
        tp = time.perf_counter()
        reps = 2
        for _ in range(reps):
            for v in range(V):
                render.render_frame(scene, pframe, cam_slot[v], mode=gs.GS_LOD_ALL_FINEST, thresholds=(),
                                    check=False)
        torch.cuda.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - tp) / (reps * V)
        out_extra["plain_fps"] = 1e3 / plain_ms
        out_extra["lod_speedup_vs_plain"] = (1e3 / plain_ms) and fps / (1e3 / plain_ms)
        log("plain (LoD off, eager): %.3f ms/frame, %.1f FPS" % (plain_ms, 1e3 / plain_ms))
        # LoD eager, same protocol, for an apples-to-apples launch mode
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(reps):
            for v in range(V):
                render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, check=False)
        torch.cuda.synchronize()
        out_extra["lod_eager_fps"] = reps * V / (time.perf_counter() - tp)

    # ---- fwd + bwd ms/view (L1 loss against a seeded target) ------------------------
    if not args.no_bwd:
        grads = [lv.zeros_like() for lv in scene.levels]
        target = torch.rand((1, 3, H, W), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
        views = list(range(0, V, max(1, V // args.bwd_views)))[: args.bwd_views]

        def fwd_bwd(fr, mode, thr):
            for v in views:
                render.render_frame(scene, fr, cam_slot[v], mode=mode, thresholds=thr, check=False)
                d = torch.sign(fr.rgb - target) / fr.rgb.numel()
                render.backward_frame(scene, fr, cam_slot[v], d, grads)

        fwd_bwd(frame, gs.GS_LOD_BLOCKWISE, thresholds)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        fwd_bwd(frame, gs.GS_LOD_BLOCKWISE, thresholds)
        torch.cuda.synchronize()
        out_extra["fwd_bwd_ms_per_view_lod"] = 1e3 * (time.perf_counter() - tb) / len(views)
        if not args.no_plain:
            fwd_bwd(pframe, gs.GS_LOD_ALL_FINEST, ())
            torch.cuda.synchronize()
            tb = time.perf_counter()
            fwd_bwd(pframe, gs.GS_LOD_ALL_FINEST, ())
            torch.cuda.synchronize()
            out_extra["fwd_bwd_ms_per_view_plain"] = 1e3 * (time.perf_counter() - tb) / len(views)
        log("fwd+bwd ms/view: %s" % {k: v for k, v in out_extra.items() if k.startswith("fwd_bwd")})
        del grads

    # ---- CPU oracle on a bounded sample: one full LoD frame -------------------------
    cpu = None
    if not args.no_cpu:
        import oracle
        from oracle import lod as olod
        oracle.build(force=False)
        vi = int(np.argsort(n_sel[V // 3:2 * V // 3])[len(n_sel[V // 3:2 * V // 3]) // 2]) + V // 3  # a 150 m view
        cam = cams[vi]
        fractions = (0.30, 0.50, 1.00)
        memb = synth.level_membership(block_id, u, scene.n_blocks, fractions)
        lvl_cnt = np.stack([m[1] for m in memb], axis=1)
        bounds = np.concatenate([[0], np.cumsum(lvl_cnt[:, -1])])
        lo = np.zeros((scene.n_blocks, 3))
        hi = np.zeros((scene.n_blocks, 3))
        t_c0 = time.perf_counter()
        for b in range(scene.n_blocks):
            lo[b], hi[b] = olod.mad_bounds(fine.means[:, bounds[b]:bounds[b + 1]])
        level_ref, _ = olod.lod_select(lo, hi, cells, thresholds, [cam], lvl_cnt)
        t_lod = time.perf_counter() - t_c0
        sel = []
        for b in range(scene.n_blocks):
            l = level_ref[0, b]
            if l < 0:
                continue
            idx = memb[l][0]
            idx = idx[(idx >= bounds[b]) & (idx < bounds[b + 1])]
            sel.append((idx, l))
        idx_all = np.concatenate([s[0] for s in sel])
        scale_k = np.concatenate([np.full(len(s[0]), 1.0 if s[1] == 2 else 1.3, np.float32) for s in sel])
        agg = synth.GaussianSet(fine.means[:, idx_all], (fine.scales[:, idx_all] * scale_k).astype(np.float32),
                                fine.quats[:, idx_all], fine.opac[idx_all], fine.sh[:, :, idx_all])
        tc = time.perf_counter()
        oracle.render(agg, cam)
        t_render = time.perf_counter() - tc
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": 1.0 / t_render, "unit": "frames/s", "cores": cores, "kind": "oracle",
               "sample": "one full 1600x900 LoD frame (view %d, 150 m, %d selected Gaussians): FP64 projection + "
                         "untiled per-pixel compositing; the per-scene MAD boxes and selection (%.1fs) are not "
                         "counted" % (vi, agg.opac.shape[0], t_lod)}
        log("cpu oracle: %.2f s/frame on %d threads" % (t_render, cores))

    result = {
        "metric": "FPS @1600x900 on 20M-Gaussian LoD scene",
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "block-wise LoD render, synthetic city, %d finest Gaussians (%d stored over 3 levels), "
                               "8x8 blocks, 1600x900, %d views per step (heights 50/150/400 m, pitch -90/-45)" %
                               (args.n, n_stored, V),
                   "n_gaussians": args.n, "width": W, "height": H, "views_per_step": V,
                   "distance_thresholds_m": list(thresholds), "launch": "hipGraph, one frame at a time"},
        "fps_mean_view": float(fps_views.mean()),
        "fps_median_view": float(np.median(fps_views)),
        "fps_min_view": float(fps_views.min()),
        "gaussians_per_s": float(n_sel.mean() * fps),
        "n_sel_mean": float(n_sel.mean()), "n_vis_mean": float(n_vis.mean()), "pairs_mean": float(n_pairs.mean()),
        "roofline": {"bound": "alu", "kernel": "rasterize_fwd (raster_fwd_kernel<16,16,256>)",
                     "achieved": ras_tflops, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ras_tflops / VALU_FP32_PEAK_TFLOPS, "traffic": None, "avg_launch_ms": ras_ms,
                     "algorithmic_flops_per_launch": ras_flops, "evals_per_launch": float(np.mean(n_eval)),
                     "flops_per_eval": FLOPS_PER_EVAL},
        "roofline_preprocess": {"bound": "hbm", "kernel": "preprocess", "achieved": pre_gbs, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": pre_gbs / HBM_PEAK_GBS, "traffic": None,
                                "avg_launch_ms": pre_ms, "algorithmic_bytes_per_launch": pre_bytes},
        "kernel_ms": {k: float(np.mean(v)) for k, v in kern_ms.items()},
        "cpu_baseline": cpu,
    }
    result.update(out_extra)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
