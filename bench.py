"""Benchmark of the MI355X rendering path.

Headline (one JSON line): block-wise LoD render of a 20M-Gaussian synthetic city
at 1600x900.  One step = every evaluation view rendered once (48 views: heights
50/150/400 m, 8 positions each, pitch -90 and -45 degrees), each frame
lod_select -> lod_refine -> preprocess -> bin_sort -> rasterize_fwd (the chunk
refinement drops the chunks the projection would cull whole, images unchanged;
--no-refine leaves it out), replayed from a HIP graph, with the tile launch
shape chosen by the autotuner (bit-identical images required).  Each call renders several views in one batched pass (--views-per-call,
default 8: one record space, one binning, one compositing launch over all their
tiles) and calls are kept in flight on separate streams with their own buffers
(--in-flight, default 4), so the latency-bound binning of one call overlaps the
compositing of another; `value` = frames per second over the step,
`fps_one_frame_in_flight` the same step one view per call, one call at a time
(--flight-sweep times every pairing of --sweep-calls and --sweep-views).

In the same line: per-view FPS (mean / median / min, and per height and pitch:
the paper's Fig. 5 split), the plain comparator (LoD off: every block at the
finest level, eager, default 16x16 tiles), the point-wise LoD comparator, the
reduced-precision levels, fwd+bwd ms/view for LoD and plain, rooflines of the
stages timed with HIP events (the longest one is `roofline`), the
whole-frame HBM fraction, the CPU oracle on a bounded sample (six city frames;
the other configurations' oracle times under cpu_baseline.other_configs), and
the other configurations as their own keys: small_render (4096 Gaussians,
256x256), single_view (1M Gaussians, 1920x1080, fwd and fwd+bwd), batched (16
views of one 2M-Gaussian block, fwd+L1+bwd in one call), uneven (32 blocks of
0.2M-3M Gaussians, 4 views each at 1280x720, LoD + fwd + bwd), assignment
(Eqs. 3-5 for 32 poses).

--workload small|single|batched|uneven|assign prints one of those alone (uneven
then autotunes its launch shape).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 20000000] [--workload lod]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BIN_SORT_KERNELS = ("clear_front, depth_hist, radix_pass<compact>, 2 radix_pass, radix_pass<pairs>, emit, emit_big, "
                    "2 tile radix_pass, ranges")
REFINE_KERNELS = "refine_clear, refine_test, refine_scan, refine_expand"
# published FP32 vector peak of MI355X (packed FP32); the library is compiled
# without packed-FP32 instructions, whose ceiling is half of it: 256 CUs x 64 FMA
# lanes per clock x 2 flops x 2.4 GHz = 78.6 TFLOP/s
VALU_FP32_PEAK_TFLOPS = 157.3
VALU_FP32_UNPACKED_TFLOPS = 78.6
# algorithmic work of one evaluated (pixel, Gaussian) entry of the forward
# compositing: 14 FP32 operations and one exponential, counted as 15
FLOPS_PER_EVAL = 15

# HBM bytes per launch (the binning: its 11 launches; the refinement: its 4) from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs of `bench.py --stages-only` scaled by a 512 MiB copy, for launches of the given views
# per call, valid for the kernel sources with the given fingerprint only
MEASURED_TRAFFIC = {
    "preprocess_kernel": (("preprocess.hip", "project.h", "gs_common.h"), "2f2db44ee46c9077", 8, 1411.33e6),
    "raster_fwd_kernel<16,16,256>": (("raster.hip", "tile.h", "project.h", "gs_common.h"), "6ead4438b5cf0fa1", 8,
                                     667.98e6),
    "bin_sort": (("sort.hip", "radix.h", "scan.h", "gs_common.h"), "7c172e1976d40684", 8, 1281.02e6),
    "lod_refine": (("refine.hip", "radix.h", "scan.h", "project.h", "gs_common.h"), "d204861f3281dbaa", 8, 35.5e6),
}


def source_fingerprint(files):
    import hashlib
    m = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2404_01133_amd", "csrc")
    for f in files:
        with open(os.path.join(base, f), "rb") as fh:
            m.update(fh.read())
    return m.hexdigest()[:16]


def measured_traffic(kernel, views_per_launch):
    """HBM bytes per launch, or None if not measured for this kernel and call shape or its source changed since."""
    if kernel not in MEASURED_TRAFFIC:
        return None
    files, fp, views, nbytes = MEASURED_TRAFFIC[kernel]
    return nbytes if views == views_per_launch and source_fingerprint(files) == fp else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("lod", "small", "single", "batched", "uneven", "assign"), default="lod")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline LoD line only (skip the small, single-view, batched, uneven and assignment legs)")
    ap.add_argument("--n", type=int, default=20_000_000, help="finest-level Gaussians (lod workload)")
    ap.add_argument("--n-xy", type=int, default=8, help="camera positions per height")
    ap.add_argument("--bwd-views", type=int, default=12, help="views used for the fwd+bwd timing")
    ap.add_argument("--in-flight", type=int, default=4,
                    help="calls rendered concurrently in the timed graph (own buffers and stream each)")
    ap.add_argument("--views-per-call", type=int, default=8,
                    help="views rendered by one batched call in the timed graph (divides the view count)")
    ap.add_argument("--sweep-calls", default="1,2,4,8", help="calls in flight tried by --flight-sweep")
    ap.add_argument("--sweep-views", default="1,2,4,8", help="views per call tried by --flight-sweep")
    ap.add_argument("--flight-sweep", action="store_true",
                    help="time calls in flight 1/2/4/8 x views per call 1/2/4/8 and print them (no headline)")
    ap.add_argument("--no-refine", action="store_true",
                    help="time the LoD frames without the chunk refinement (gs_lod_refine)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-pointwise", action="store_true", help="skip the point-wise LoD comparator")
    ap.add_argument("--no-reduced", action="store_true", help="skip the reduced-precision levels variant")
    ap.add_argument("--pointwise-only", action="store_true",
                    help="only the timed point-wise LoD frames (for profilers)")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--frames-only", action="store_true", help="only the timed LoD frames (for profilers)")
    ap.add_argument("--bwd-only", action="store_true", help="only the LoD fwd+bwd loop (for profilers)")
    ap.add_argument("--stages-only", action="store_true",
                    help="only the HIP-event stage timing of the LoD calls (for profilers)")
    ap.add_argument("--tuning", default=None, help="tile_w,tile_h,batch,flags instead of autotuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 512 MiB device-to-device copies (reference for HBM byte counters)")
    return ap.parse_args()


def evals_to_termination(torch, frame, chunk=1 << 16):
    """E of one rendered single-view frame: the (pixel, Gaussian) entries the
    compositing evaluates, i.e. for every pixel the entries of its tile list
    before its termination (n_last) whose footprint rectangle holds the pixel.
    (The same set for every tile shape: a record whose rectangle holds a pixel is
    in that pixel's tile list.)"""
    tw, th = frame.tuning.tile_w, frame.tuning.tile_h
    W, H = frame.W, frame.H
    tx_n, ty_n = frame.tiles_x, frame.tiles_y
    m = frame.host_counts()["pairs"]
    if m == 0:
        return 0
    nl = torch.zeros((ty_n * th, tx_n * tw), dtype=torch.int32, device=frame.device)
    nl[:H, :W] = frame.n_last[0]
    nl = nl.view(ty_n, th, tx_n, tw).permute(0, 2, 1, 3).reshape(ty_n * tx_n, th, tw)
    tiles = frame.pair_tiles[:m].to(torch.int64)
    recs = frame.pair_records[:m].to(torch.int64)
    start = frame.tile_ranges[:, 0].to(torch.int64)
    raw = frame.records.view(torch.int32).view(-1, 12)
    ax = torch.arange(tw, device=frame.device)
    ay = torch.arange(th, device=frame.device)
    total = 0
    for c0 in range(0, m, chunk):
        t = tiles[c0:c0 + chunk]
        k = torch.arange(c0, min(m, c0 + chunk), device=frame.device, dtype=torch.int64) - start[t]
        r = raw[recs[c0:c0 + chunk]]
        px, py = r[:, 2].to(torch.int64) & 0xFFFFFFFF, r[:, 3].to(torch.int64) & 0xFFFFFFFF
        i0, j0 = px & 0xFFFF, py & 0xFFFF
        i1, j1 = i0 + (px >> 16), j0 + (py >> 16)
        ox, oy = (t % tx_n) * tw, (t // tx_n) * th
        mx = ((ax[None] + ox[:, None]) >= i0[:, None]) & ((ax[None] + ox[:, None]) <= i1[:, None])
        my = ((ay[None] + oy[:, None]) >= j0[:, None]) & ((ay[None] + oy[:, None]) <= j1[:, None])
        walked = nl[t] > k[:, None, None]
        total += int((walked & my[:, :, None] & mx[:, None, :]).sum().item())
    return total


def graph_of(torch, fn, stream):
    g = torch.cuda.CUDAGraph()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        fn()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            fn()
    torch.cuda.synchronize()
    return g


def timed_replays(torch, g, steps, warmup):
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


# -------------------------------------------------------------------------------------------
def workload_lod(args, torch, gs, render, synth):
    dev = "cuda:0"
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
    rc = scene.max_records_per_view()
    # chunk refinement between the selection and the projection (same images, fewer records)
    refine = not args.no_refine

    def new_frame(tw=16, th=16, batch=256, flags=0):
        f = render.Frame(scene.n_blocks, 1, W, H, rc, 1 << 22, gs.tuning_struct(tw, th, batch, flags), device=dev)
        for v in range(V):  # grow the pair capacity to fit every view
            render.render_frame(scene, f, cam_slot[v], thresholds=thresholds, refine=refine)
        return f

    # ---- capacities and per-view statistics from one eager pass ----------------------
    frame = render.Frame(scene.n_blocks, 1, W, H, rc, 1 << 22, device=dev)
    stats, evals = [], []
    for v in range(V):
        render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds)
        c = frame.host_counts()
        stats.append(c)
        # (pixel, Gaussian) entries the compositing evaluates, up to each pixel's termination
        # (torch kernels, outside every timed region; skipped in the profiler-only modes)
        if not (args.frames_only or args.bwd_only or args.pointwise_only or args.stages_only):
            evals.append(evals_to_termination(torch, frame))
    n_sel = np.array([s["records"] for s in stats])
    n_vis = np.array([s["visible"] for s in stats])
    n_pairs = np.array([s["pairs"] for s in stats])
    n_eval = np.array(evals if evals else [0.0], dtype=np.float64)
    log("per view: N_sel mean %.0f (max %d), N_vis mean %.0f, pairs mean %.0f (max %d), evals mean %.0f" %
        (n_sel.mean(), n_sel.max(), n_vis.mean(), n_pairs.mean(), n_pairs.max(), n_eval.mean()))
    # records left per view after the chunk refinement (the same visible records and pairs)
    n_rec = n_sel
    if refine:
        refd = []
        for v in range(V):
            render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, refine=True)
            c = frame.host_counts()
            if (c["visible"], c["pairs"]) != (int(n_vis[v]), int(n_pairs[v])):
                raise RuntimeError("view %d: refined counts %s differ from the selection's" % (v, c))
            refd.append(c["records"])
        n_rec = np.array(refd)
        log("chunk refinement: records mean %.0f of %.0f selected (%.1f %%), %d chunks" %
            (n_rec.mean(), n_sel.mean(), 100.0 * n_rec.mean() / max(1.0, n_sel.mean()),
             int(scene.chunk_off[-1].item())))
    # every stream of the step is made here, before anything else makes streams, so
    # the K streams of the in-flight graph land on distinct hardware queues
    K = max(1, args.in_flight)
    stream = torch.cuda.Stream()
    side = [torch.cuda.Stream() for _ in range(max(K, 8 if args.flight_sweep else 1) - 1)]

    def lod_step(f):
        return lambda: [render.render_frame(scene, f, cam_slot[v], thresholds=thresholds, check=False, refine=refine)
                        for v in range(V)]

    if args.pointwise_only:
        print(json.dumps(pointwise_frames(args, torch, gs, render, scene, cam_slot, thresholds, W, H,
                                          frame.tuning, stream, None)))
        return
    if args.bwd_only:
        grads = [lv.zeros_like() for lv in scene.levels]
        target = torch.rand((1, 3, H, W), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
        for _ in range(2):
            for v in range(0, V, max(1, V // args.bwd_views)):
                render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds, check=False, refine=refine)
                d = torch.sign(frame.rgb - target) / frame.rgb.numel()
                render.backward_frame(scene, frame, cam_slot[v], d, grads)
        torch.cuda.synchronize()
        print(json.dumps({"bwd_only": True}))
        return

    # ---- launch shape: autotuned (bit-identical images required) or given ------------
    default_step_ms = None
    tune_report = None
    if args.tuning:
        tw, th, b, fl = (int(x) for x in args.tuning.split(","))
        frame = new_frame(tw, th, b, fl)
    elif not (args.no_autotune or args.frames_only or args.stages_only):
        from paper_2404_01133_amd import autotune
        frames = {(16, 16): frame}
        gate_views = [0, V // 3, 2 * V // 3, V - 1]

        def make_runner(cand):
            key = (cand.tile_w, cand.tile_h)
            if key not in frames:
                frames[key] = new_frame(*key)
            f = frames[key]
            f.tuning = cand.tuning()

            def images():
                out = []
                for v in gate_views:
                    render.render_frame(scene, f, cam_slot[v], thresholds=thresholds, check=False, refine=refine)
                    out.append(f.rgb.clone())
                return torch.cat(out)
            return lod_step(f), images

        t_at = time.time()
        best, tune_report = autotune.tune("lod_city_%d_%dx%d_%dviews" % (args.n, W, H, V), make_runner, stream=stream,
                                          use_cache=False)
        log("autotune: best %s at %.3f ms/step (default %.3f ms), %d candidates rejected, %.1fs" %
            (best.as_dict(), tune_report["best_ms"], tune_report["default_ms"], tune_report["rejected"],
             time.time() - t_at))
        default_step_ms = tune_report["default_ms"]
        frame = frames[(best.tile_w, best.tile_h)]
        frame.tuning = best.tuning()
        for key in list(frames):
            if key != (best.tile_w, best.tile_h):
                del frames[key]
    tun = frame.tuning
    tuning_desc = dict(tile_w=tun.tile_w, tile_h=tun.tile_h, batch=tun.batch, flags=tun.flags)

    # ---- stages timed with HIP events on the stream they run on, in the call shape of
    #      the timed step (P_ views per call), one call at a time; work per launch is
    #      the sum over the call's views -------------------------------------------------
    def time_stages(P_):
        if V % P_:
            raise ValueError("views per call must divide the %d views" % V)
        sf = frame if P_ == 1 else render.Frame(scene.n_blocks, P_, W, H, P_ * rc, P_ * frame.pair_capacity,
                                                gs.tuning_struct(tun.tile_w, tun.tile_h, tun.batch, tun.flags),
                                                device=dev)
        n_calls = V // P_
        calls = [cams_all[c * P_ * 152:(c + 1) * P_ * 152] for c in range(n_calls)]
        for c in range(n_calls):  # capacities, and the counts of a call equal the sums over its views
            render.render_frame(scene, sf, calls[c], thresholds=thresholds, refine=refine)
            hc = sf.host_counts()
            want = (int(n_rec[c * P_:(c + 1) * P_].sum()), int(n_vis[c * P_:(c + 1) * P_].sum()),
                    int(n_pairs[c * P_:(c + 1) * P_].sum()))
            if (hc["records"], hc["visible"], hc["pairs"]) != want:
                raise RuntimeError("call %d counts %s differ from the sums over its views %s" % (c, hc, want))
        kms = {"preprocess": [], "rasterize_fwd": [], "bin_sort": []}
        if refine:
            kms["lod_refine"] = []
        blocks = scene.blocks_struct()
        levels = [lv.struct() for lv in scene.levels]
        with torch.cuda.stream(stream):
            for rep in range(2):  # the first round warms up
                for c in range(n_calls):
                    cc = calls[c]
                    gs.lod_select(blocks, thresholds, gs.GS_LOD_BLOCKWISE, cc, P_, sf.level, sf.offsets, sf.counts,
                                  stream)
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
                    ev[0].record(stream)
                    if refine:
                        r = sf.refined
                        gs.lod_refine(blocks, sf.level, cc, P_, W, H, scene.chunk_off, scene.chunk_bounds,
                                      scene.max_chunks, sf.record_capacity, r["gather"], r["view_off"], sf.counts,
                                      r["ws"], stream)
                    ev[1].record(stream)
                    level, offsets, gather = sf.selection()
                    gs.preprocess(levels, blocks, level, offsets, cc, P_, W, H, 3, sf.pre_tuning(),
                                  sf.record_capacity, sf.records, sf.depth_keys, sf.tiles_touched, sf.counts, stream,
                                  gather=gather)
                    ev[2].record(stream)
                    gs.bin_sort(sf.records, sf.depth_keys, sf.tiles_touched, P_, W, H, sf.tuning, sf.record_capacity,
                                sf.pair_capacity, sf.pair_tiles, sf.pair_records, sf.tile_ranges, sf.counts,
                                sf.sort_ws, stream, sf.tile_queue)
                    ev[3].record(stream)
                    gs.rasterize_fwd(sf.records, sf.pair_records, sf.tile_ranges, P_, W, H, (0.0, 0.0, 0.0),
                                     sf.tuning, sf.rgb, sf.T, sf.n_last, stream, sf.tile_queue)
                    ev[4].record(stream)
                    ev[4].synchronize()
                    if rep:
                        if refine:
                            kms["lod_refine"].append(ev[0].elapsed_time(ev[1]))
                        kms["preprocess"].append(ev[1].elapsed_time(ev[2]))
                        kms["bin_sort"].append(ev[2].elapsed_time(ev[3]))
                        kms["rasterize_fwd"].append(ev[3].elapsed_time(ev[4]))
        if sf.host_counts()["flags"]:
            raise RuntimeError("capacity flag raised during the stage timing: %s" % sf.host_counts())
        del sf
        pre_ms = float(np.mean(kms["preprocess"]))
        bin_ms = float(np.mean(kms["bin_sort"]))
        ras_ms = float(np.mean(kms["rasterize_fwd"]))
        ref_ms = float(np.mean(kms["lod_refine"])) if refine else 0.0
        log("stage ms per call of %d views (mean over %d calls): %spreprocess %.4f, bin_sort %.4f, "
            "rasterize_fwd %.4f" % (P_, n_calls, "lod_refine %.4f, " % ref_ms if refine else "", pre_ms, bin_ms,
                                    ras_ms))
        per_call = lambda a: a.reshape(n_calls, P_).sum(axis=1).astype(np.float64)
        c_rec, c_vis, c_pairs = per_call(n_rec), per_call(n_vis), per_call(n_pairs)
        c_eval = per_call(n_eval) if n_eval.size == V else np.zeros(n_calls)
        # preprocess: 12 B centre + 8 B (depth key, tiles touched) per record (+ 4 B gather entry after
        # the refinement); 224 B (rotation, scale, opacity, SH) read + 48 B record written per visible record
        pre_bytes = float(np.mean((24.0 if refine else 20.0) * c_rec + 272.0 * c_vis))
        # binning, one-pass lower bound: pairs written once and read once (24 B per pair) + the range scan (8 B)
        bin_bytes = float(np.mean(32.0 * c_pairs))
        # what the sort's own passes move at 24 B per element per pass: four depth passes (the first over
        # every selected record, the others over the visible ones) and ceil(tile bits / 8) tile passes
        n_tile_ids = frame.tiles_x * frame.tiles_y * P_
        tbits = max(0, int(n_tile_ids - 1).bit_length())
        tpasses = (tbits + 7) // 8
        sort_bytes = float(np.mean(24.0 * (c_rec + 3.0 * c_vis + tpasses * c_pairs)))
        # forward compositing: 15 operations per evaluated entry (14 FP32 + one exponential)
        ras_flops = float(np.mean(c_eval)) * FLOPS_PER_EVAL
        ras_name = "raster_fwd_kernel<%d,%d,%d>" % (tun.tile_w, tun.tile_h, tun.batch)
        st = {
            "preprocess": {"bound": "hbm", "kernel": "preprocess_kernel", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                           "achieved": pre_bytes / (pre_ms * 1e-3) / 1e9, "avg_launch_ms": pre_ms,
                           "algorithmic_bytes_per_launch": pre_bytes,
                           "traffic": measured_traffic("preprocess_kernel", P_)},
            "bin_sort": {"bound": "hbm", "kernel": "bin_sort stage (%s)" % BIN_SORT_KERNELS, "unit": "GB/s",
                         "peak": HBM_PEAK_GBS, "achieved": bin_bytes / (bin_ms * 1e-3) / 1e9,
                         "avg_launch_ms": bin_ms, "algorithmic_bytes_per_launch": bin_bytes, "bytes_per_pair": 32,
                         "sort_design_bytes": sort_bytes,
                         "sort_design_frac": sort_bytes / (bin_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "tile_passes": tpasses, "traffic": measured_traffic("bin_sort", P_)},
            "rasterize_fwd": {"bound": "alu", "kernel": ras_name, "unit": "TFLOP/s", "peak": VALU_FP32_PEAK_TFLOPS,
                              "achieved": ras_flops / (ras_ms * 1e-3) / 1e12, "avg_launch_ms": ras_ms,
                              "algorithmic_flops_per_launch": ras_flops, "evals_per_launch": float(np.mean(c_eval)),
                              "flops_per_eval": FLOPS_PER_EVAL, "frac_of_unpacked_fp32_ceiling": None,
                              "traffic": measured_traffic(ras_name, P_)},
        }
        if refine:
            # per (view, chunk): the 32 B box read, a size written and read twice, an offset written
            # and read (20 B); 4 B gather entry written per record kept
            n_chunks = int(scene.chunk_off[-1].item())
            ref_bytes = float(np.mean(P_ * n_chunks * 52.0 + 4.0 * c_rec))
            st["lod_refine"] = {"bound": "hbm", "kernel": "lod_refine stage (%s)" % REFINE_KERNELS, "unit": "GB/s",
                                "peak": HBM_PEAK_GBS, "achieved": ref_bytes / (ref_ms * 1e-3) / 1e9,
                                "avg_launch_ms": ref_ms, "algorithmic_bytes_per_launch": ref_bytes,
                                "chunks": n_chunks, "traffic": measured_traffic("lod_refine", P_)}
        for r in st.values():
            r["frac"] = r["achieved"] / r["peak"]
            r["views_per_launch"] = P_
        st["rasterize_fwd"]["frac_of_unpacked_fp32_ceiling"] = \
            st["rasterize_fwd"]["achieved"] / VALU_FP32_UNPACKED_TFLOPS
        return st, max(st, key=lambda k: st[k]["avg_launch_ms"]), kms

    def copy_calibration():
        # a plain 512 MiB device copy, for scaling the HBM counters of a profiler run
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def copy_rate_gbs():
        # measured ceiling beside the published one: a plain 512 MiB device-to-device copy
        # (read + write bytes over its HIP-event time, best of five)
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        best = float("inf")
        with torch.cuda.stream(stream):
            for _ in range(6):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                dst.copy_(src)
                e1.record(stream)
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1))
        del src, dst
        return 2.0 * (512 << 20) / (best * 1e-3) / 1e9

    if args.stages_only:
        st, dom, _ = time_stages(max(1, args.views_per_call))
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps({"stages_only": True, "roofline": dict(st[dom], stage=dom), "rooflines": st}))
        return

    # ---- HIP graph of one step (all views, one frame each) ---------------------------
    # one frame at a time on one stream ...
    graph = graph_of(torch, lod_step(frame), stream)
    seq_s = timed_replays(torch, graph, args.steps, args.warmup)
    del graph
    fps_seq = V / seq_s
    if frame.host_counts()["flags"]:
        raise RuntimeError("capacity flag raised during the timed frames: %s" % frame.host_counts())
    log("LoD graph, one frame in flight (%s): %.3f ms/step, %.1f FPS" % (tuning_desc, 1e3 * seq_s, fps_seq))
    # ... and K calls in flight, each rendering P views (one batched call: one record space,
    # one binning, one compositing launch over all P views' tiles): call c takes views
    # [cP, (c+1)P) on stream c mod K with its own buffers, so the latency-bound binning of
    # one call overlaps the compositing of another and is shared by P views
    def in_flight_fps(K_, P_):
        if V % P_:
            raise ValueError("views per call must divide the %d views" % V)
        K_ = min(K_, V // P_)  # no more buffers than calls
        if K_ == 1 and P_ == 1:
            return seq_s
        flight = [frame if P_ == 1 and k == 0 else
                  render.Frame(scene.n_blocks, P_, W, H, P_ * rc, P_ * frame.pair_capacity,
                               gs.tuning_struct(tun.tile_w, tun.tile_h, tun.batch, tun.flags), device=dev)
                  for k in range(K_)]
        calls = [cams_all[c * P_ * 152:(c + 1) * P_ * 152] for c in range(V // P_)]
        for c in range(V // P_):
            render.render_frame(scene, flight[c % K_], calls[c], thresholds=thresholds, refine=refine)

        def pipelined_step():
            cur = torch.cuda.current_stream()
            for s2 in side[:K_ - 1]:
                s2.wait_stream(cur)
            streams = [cur] + side[:K_ - 1]
            for c in range(V // P_):
                with torch.cuda.stream(streams[c % K_]):
                    render.render_frame(scene, flight[c % K_], calls[c], thresholds=thresholds, check=False,
                                        refine=refine)
            for s2 in side[:K_ - 1]:
                cur.wait_stream(s2)

        graph = graph_of(torch, pipelined_step, stream)
        t = timed_replays(torch, graph, args.steps, args.warmup)
        del graph
        for f in flight:
            if f.host_counts()["flags"]:
                raise RuntimeError("capacity flag raised during the timed frames: %s" % f.host_counts())
        # every buffer holds the same images as the one-at-a-time path (its last call's views),
        # which renders here without the chunk refinement
        for k in range(K_):
            c = (V // P_ - 1) - ((V // P_ - 1 - k) % K_)
            for p_ in range(P_):
                render.render_frame(scene, frame, cam_slot[c * P_ + p_], thresholds=thresholds)
                if not torch.equal(frame.rgb[0], flight[k].rgb[p_]):
                    raise RuntimeError("in-flight buffer %d differs from the sequential render of view %d" %
                                       (k, c * P_ + p_))
        del flight
        return t

    P = max(1, args.views_per_call)
    if args.flight_sweep:
        sweep = {}
        for K_ in (int(x) for x in args.sweep_calls.split(",")):
            for P_ in (int(x) for x in args.sweep_views.split(",")):
                if K_ - 1 <= len(side) and V % P_ == 0:
                    t = in_flight_fps(K_, P_)
                    sweep["%dx%d" % (K_, P_)] = V / t
                    log("calls in flight %d x views per call %d: %.1f FPS" % (K_, P_, V / t))
        print(json.dumps({"flight_sweep": sweep}))
        return None
    step_s = in_flight_fps(K, P)
    ms_per_step = 1e3 * step_s
    fps = V / step_s
    log("LoD graph, %d calls in flight x %d views per call: %.3f ms/step, %.1f FPS" % (K, P, ms_per_step, fps))
    if args.copy_calibration:
        copy_calibration()
    if args.frames_only:
        print(json.dumps({"metric": "FPS", "value": fps, "fps_one_frame_in_flight": fps_seq,
                          "ms_per_step": ms_per_step, "tuning": tuning_desc,
                          "n_sel_mean": float(n_sel.mean()), "n_vis_mean": float(n_vis.mean()),
                          "pairs_mean": float(n_pairs.mean())}))
        return

    # ---- per-view FPS distribution (one graph per view) ------------------------------
    per_view_ms = []
    for v in range(V):
        gv = graph_of(torch, lambda: render.render_frame(scene, frame, cam_slot[v], thresholds=thresholds,
                                                         check=False, refine=refine), stream)
        with torch.cuda.stream(stream):
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
    fps_views = 1e3 / np.array(per_view_ms)

    # ---- per-height / per-pitch FPS (the paper's Fig. 5 reports mean and minimum
    #      FPS per camera height for looking-down cameras) ---------------------------
    heights, pitches = (50.0, 150.0, 400.0), (-90.0, -45.0)
    per_group = {}
    for hi, h in enumerate(heights):
        for pi, p in enumerate(pitches):
            sel = fps_views[(hi * len(pitches) + pi) * args.n_xy:(hi * len(pitches) + pi + 1) * args.n_xy]
            per_group["%dm_pitch%d" % (h, p)] = {"fps_mean": float(sel.mean()), "fps_min": float(sel.min()),
                                                 "views": int(sel.size)}

    stage, dominant, kern_ms = time_stages(P)
    # whole frame against HBM: the algorithmic bytes of one forward frame (N_sel centres and
    # tiles touched, N_vis parameters and records, pairs written/read/scanned/gathered, image, T, n_last)
    b_fwd = float(np.mean((28.0 if refine else 24.0) * n_rec + 276.0 * n_vis + 72.0 * n_pairs)) + 20.0 * W * H
    copy_gbs = copy_rate_gbs()
    log("device copy: %.0f GB/s (read + write)" % copy_gbs)
    for r in stage.values():
        if r["bound"] == "hbm":
            r["frac_of_measured_copy"] = r["achieved"] / copy_gbs
    frame_hbm = {"bytes_per_frame": b_fwd,
                 "frac_one_frame_in_flight": b_fwd * fps_seq / (HBM_PEAK_GBS * 1e9),
                 "frac_frames_in_flight": b_fwd * fps / (HBM_PEAK_GBS * 1e9),
                 "measured_copy_gbs": copy_gbs,
                 "frac_frames_in_flight_of_measured_copy": b_fwd * fps / (copy_gbs * 1e9)}

    out_extra = {}
    # ---- plain comparator: LoD off, every block at the finest level, eager, 16x16 ----
    pframe = None
    if not args.no_plain:
        pframe = render.Frame(scene.n_blocks, 1, W, H, scene.n_finest, 1 << 23, device=dev)
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
        log("plain (LoD off, eager, 16x16): %.3f ms/frame, %.1f FPS" % (plain_ms, 1e3 / plain_ms))
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(reps):
            lod_step(frame)()
        torch.cuda.synchronize()
        out_extra["lod_eager_fps"] = reps * V / (time.perf_counter() - tp)
        # like for like: both eager, one frame at a time
        out_extra["lod_speedup_vs_plain"] = out_extra["lod_eager_fps"] / out_extra["plain_fps"]

    # ---- point-wise LoD comparator (the baseline of the block-wise strategy) -----------
    if not args.no_pointwise:
        out_extra["pointwise"] = pointwise_frames(args, torch, gs, render, scene, cam_slot, thresholds, W, H,
                                                  frame.tuning, stream, fps_seq)

    # ---- reduced-precision coarse levels (binary16 attributes, fewer SH bands) ---------
    if not args.no_reduced:
        out_extra["reduced_precision"] = reduced_frames(args, torch, gs, render, scene, cam_slot, thresholds, W, H,
                                                        frame.tuning, stream, fps_seq)

    # ---- fwd + bwd ms/view (L1 loss against a seeded target) --------------------------
    if not args.no_bwd:
        grads = [lv.zeros_like() for lv in scene.levels]
        target = torch.rand((1, 3, H, W), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
        views = list(range(0, V, max(1, V // args.bwd_views)))[: args.bwd_views]

        def fwd_bwd(fr, mode, thr, ref):
            for v in views:
                render.render_frame(scene, fr, cam_slot[v], mode=mode, thresholds=thr, check=False, refine=ref)
                d = torch.sign(fr.rgb - target) / fr.rgb.numel()
                render.backward_frame(scene, fr, cam_slot[v], d, grads)

        # the plain comparator renders the whole finest level, unrefined
        for fr, mode, thr, ref, key in ((frame, gs.GS_LOD_BLOCKWISE, thresholds, refine, "lod"),
                                        (pframe, gs.GS_LOD_ALL_FINEST, (), False, "plain")):
            if fr is None:
                continue
            fwd_bwd(fr, mode, thr, ref)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            fwd_bwd(fr, mode, thr, ref)
            torch.cuda.synchronize()
            out_extra["fwd_bwd_ms_per_view_" + key] = 1e3 * (time.perf_counter() - tb) / len(views)
        log("fwd+bwd ms/view: %s" % {k: v for k, v in out_extra.items() if k.startswith("fwd_bwd")})
        del grads
    del pframe

    # ---- CPU oracle on a bounded sample: one full LoD frame ---------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_frames(scene, fine, block_id, u, cells, cams, args.n_xy, thresholds, synth)
    del scene, fine

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
                   "distance_thresholds_m": list(thresholds),
                   "launch": "hipGraph of the %d views: %d calls in flight on %d streams, %d views per call%s" %
                             (V, K, K, P, ", chunk refinement" if refine else ""),
                   "tuning": tuning_desc},
        "fps_one_frame_in_flight": fps_seq,
        "fps_mean_view": float(fps_views.mean()),
        "fps_median_view": float(np.median(fps_views)),
        "fps_min_view": float(fps_views.min()),
        "default_tuning_fps": (V / (default_step_ms * 1e-3)) if default_step_ms else None,
        "gaussians_per_s": float(n_sel.mean() * fps),
        "n_sel_mean": float(n_sel.mean()), "n_vis_mean": float(n_vis.mean()), "pairs_mean": float(n_pairs.mean()),
        "n_records_mean": float(n_rec.mean()), "chunk_refinement": refine,
        "roofline": dict(stage[dominant], stage=dominant),
        "rooflines": stage,
        "frame_hbm": frame_hbm,
        "per_height_pitch": per_group,
        "stage_ms_per_call": {k: float(np.mean(v)) for k, v in kern_ms.items()},
        "stage_ms_per_view": {k: float(np.mean(v)) / P for k, v in kern_ms.items()},
        "cpu_baseline": cpu,
    }
    if tune_report:
        result["autotune"] = {k: tune_report[k] for k in ("best", "best_ms", "default_ms", "rejected")}
        # fastest step per flags value (0: one work-group per tile, 2: work queue)
        by_flags = {}
        for r in tune_report["results"]:
            key = str(r["flags"])
            by_flags[key] = min(by_flags.get(key, float("inf")), r["ms"])
        result["autotune"]["best_ms_by_flags"] = by_flags
    result.update(out_extra)
    return result


def pointwise_frames(args, torch, gs, render, scene, cam_slot, thresholds, W, H, tuning, stream, blockwise_fps):
    """The same views with the point-wise selection (every Gaussian of every level
    tested against the distance intervals and the frustum), HIP graph, same launch
    shape, one frame at a time (compared with the block-wise step run the same
    way); plus the selection kernel's time and HBM roofline (12 B of centre read
    per stored Gaussian, 4 B of gather index written per selected one)."""
    dev = "cuda:0"
    V = len(cam_slot)
    f = render.Frame(scene.n_blocks, 1, W, H, scene.max_records_per_view(), 1 << 22, tuning, device=dev)
    sel = []
    for v in range(V):
        render.render_frame(scene, f, cam_slot[v], mode=render.LOD_POINTWISE, thresholds=thresholds)
        sel.append(f.host_counts()["records"])
    step = lambda: [render.render_frame(scene, f, cam_slot[v], mode=render.LOD_POINTWISE, thresholds=thresholds,
                                        check=False) for v in range(V)]
    g = graph_of(torch, step, stream)
    step_s = timed_replays(torch, g, max(3, args.steps // 2), 1)
    del g
    if f.host_counts()["flags"]:
        raise RuntimeError("capacity flag raised during the point-wise frames: %s" % f.host_counts())
    pw_fps = V / step_s
    levels = [lv.struct() for lv in scene.levels]
    n_stored = sum(lv.n for lv in scene.levels)
    sel_ms = []
    with torch.cuda.stream(stream):
        for v in range(V):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gs.lod_select_points(levels, thresholds, cam_slot[v], 1, f.record_capacity, f.gather, f.pts_offsets,
                                 f.counts, f.pts_ws, stream)
            e1.record(stream)
            e1.synchronize()
            sel_ms.append(e0.elapsed_time(e1))
    ms = float(np.mean(sel_ms))
    nbytes = 12.0 * n_stored + 4.0 * float(np.mean(sel))
    gbs = nbytes / (ms * 1e-3) / 1e9
    log("point-wise LoD: %.1f FPS (%.3f ms/frame), selection %.4f ms, %.0f GB/s, %.0f records/view" %
        (pw_fps, 1e3 / pw_fps, ms, gbs, float(np.mean(sel))))
    out = {"fps": pw_fps, "ms_per_frame": 1e3 / pw_fps, "n_sel_mean": float(np.mean(sel)),
           "select_kernels": "point_flags_kernel + point_scan_kernel + point_write_kernel", "select_ms": ms,
           "select_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": nbytes}}
    if blockwise_fps:
        out["blockwise_speedup"] = blockwise_fps / pw_fps
    return out


def reduced_frames(args, torch, gs, render, scene, cam_slot, thresholds, W, H, tuning, stream, fp32_fps,
                   sh_degrees=(1, 2, 3), half_levels=(0, 1)):
    """The same block-wise LoD frames with the coarse levels stored at reduced
    precision: binary16 attributes for levels 0 and 1, SH degrees 1 / 2 / 3 for
    levels 0 / 1 / 2 (Sec. 3.3.1), one frame at a time (compared with the FP32
    step run the same way).  A different scene, so a variant beside the headline,
    not the headline."""
    dev = "cuda:0"
    V = len(cam_slot)
    rs = scene.reduced_precision(sh_degrees, half_levels)
    f = render.Frame(scene.n_blocks, 1, W, H, scene.max_records_per_view(), 1 << 22, tuning, device=dev)
    for v in range(V):
        render.render_frame(rs, f, cam_slot[v], thresholds=thresholds)
    step = lambda: [render.render_frame(rs, f, cam_slot[v], thresholds=thresholds, check=False) for v in range(V)]
    g = graph_of(torch, step, stream)
    step_s = timed_replays(torch, g, max(3, args.steps // 2), 1)
    del g
    if f.host_counts()["flags"]:
        raise RuntimeError("capacity flag raised during the reduced-precision frames: %s" % f.host_counts())
    blocks = rs.blocks_struct()
    levels = [lv.struct() for lv in rs.levels]
    pre_ms = []
    with torch.cuda.stream(stream):
        for v in range(V):
            gs.lod_select(blocks, thresholds, gs.GS_LOD_BLOCKWISE, cam_slot[v], 1, f.level, f.offsets, f.counts,
                          stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gs.preprocess(levels, blocks, f.level, f.offsets, cam_slot[v], 1, W, H, 3, f.tuning, f.record_capacity,
                          f.records, f.depth_keys, f.tiles_touched, f.counts, stream)
            e1.record(stream)
            e1.synchronize()
            pre_ms.append(e0.elapsed_time(e1))
    fps = V / step_s
    stored = sum(t.numel() * t.element_size() for lv in rs.levels[:-1]
                 for t in (lv.means, lv.scales, lv.quats, lv.opac, lv.sh))
    log("reduced-precision levels: %.1f FPS (%.3f ms/frame), preprocess %.4f ms" %
        (fps, 1e3 / fps, float(np.mean(pre_ms))))
    del rs
    return {"fps": fps, "ms_per_frame": 1e3 / fps, "speedup_vs_fp32_levels": fps / fp32_fps,
            "preprocess_ms": float(np.mean(pre_ms)), "sh_degrees": list(sh_degrees),
            "binary16_levels": list(half_levels), "coarse_level_bytes": int(stored)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_oracle_frames(scene, fine, block_id, u, cells, cams, n_xy, thresholds, synth):
    """The oracle (FP64, untiled, OpenMP over pixels) on six seeded LoD views of
    the city, two per height (first position at each pitch), each a full
    1600x900 frame on its oracle-selected aggregated set; the per-scene MAD
    boxes are computed once and not counted."""
    import oracle
    from oracle import lod as olod
    oracle.build(force=False)
    fractions = (0.30, 0.50, 1.00)
    memb = synth.level_membership(block_id, u, scene.n_blocks, fractions)
    lvl_cnt = np.stack([m[1] for m in memb], axis=1)
    bounds = np.concatenate([[0], np.cumsum(lvl_cnt[:, -1])])
    lo = np.zeros((scene.n_blocks, 3))
    hi = np.zeros((scene.n_blocks, 3))
    for b in range(scene.n_blocks):
        lo[b], hi[b] = olod.mad_bounds(fine.means[:, bounds[b]:bounds[b + 1]])
    views = [(hi_ * 2 + pi) * n_xy for hi_ in range(3) for pi in range(2)]
    times, n_agg = [], []
    for vi in views:
        cam = cams[vi]
        level_ref, _ = olod.lod_select(lo, hi, cells, thresholds, [cam], lvl_cnt)
        sel = []
        for b in range(scene.n_blocks):
            l = level_ref[0, b]
            if l < 0:
                continue
            idx = memb[l][0]
            idx = idx[(idx >= bounds[b]) & (idx < bounds[b + 1])]
            sel.append((idx, l))
        idx_all = np.concatenate([s_[0] for s_ in sel])
        scale_k = np.concatenate([np.full(len(s_[0]), 1.0 if s_[1] == 2 else 1.3, np.float32) for s_ in sel])
        agg = synth.GaussianSet(fine.means[:, idx_all], (fine.scales[:, idx_all] * scale_k).astype(np.float32),
                                fine.quats[:, idx_all], fine.opac[idx_all], fine.sh[:, :, idx_all])
        tc = time.perf_counter()
        oracle.render(agg, cam)
        times.append(time.perf_counter() - tc)
        n_agg.append(agg.opac.shape[0])
    t = float(np.mean(times))
    log("cpu oracle (city LoD frames): %.2f s/frame on %d threads" % (t, cpu_threads()))
    return {"value": 1.0 / t, "unit": "frames/s", "cores": cpu_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "six full 1600x900 LoD frames of the 20M city (views %s: two per height 50/150/400 m, pitch "
                      "-90 and -45), each on its oracle-selected set (%d Gaussians on average): FP64 projection + "
                      "untiled per-pixel compositing; per-scene MAD boxes not counted" %
                      (views, int(np.mean(n_agg))),
            "ms_per_view": [1e3 * x for x in times]}


def cpu_oracle_views(g_list, cams, dimgs, fwd_only=False):
    """Wall-clock of the oracle per view: forward render and (unless fwd_only) its exact backward."""
    import oracle
    oracle.build(force=False)
    fwd, bwd = [], []
    for g, cam, d in zip(g_list, cams, dimgs):
        t0 = time.perf_counter()
        oracle.render(g, cam)
        fwd.append(time.perf_counter() - t0)
        if not fwd_only:
            t0 = time.perf_counter()
            oracle.render_bwd(g, cam, d)
            bwd.append(time.perf_counter() - t0)
    out = {"fwd_ms_per_view": 1e3 * float(np.mean(fwd)), "views": len(fwd)}
    if bwd:
        out["fwd_bwd_ms_per_view"] = 1e3 * float(np.mean(np.array(fwd) + np.array(bwd)))
    return out


def timed_ms(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / reps


def single_set_case(args, torch, gs, render, g, cam, target, reps, tag, cpu):
    """One Gaussian set, one view, LoD off (every Gaussian): forward and forward +
    L1 backward latency, eager and from a HIP graph; optionally the oracle."""
    dev = "cuda:0"
    scene = render.DeviceScene.single(g, device=dev)
    cams_dev = gs.cameras_to_device([cam], dev)
    n = scene.n_finest
    f = render.Frame(1, 1, cam.width, cam.height, n, max(1 << 16, 4 * n), device=dev)
    render.render_frame(scene, f, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=())
    grads = [scene.levels[0].zeros_like()]
    tgt = torch.from_numpy(target[None]).to(dev)

    def fwd():
        render.render_frame(scene, f, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=(), check=False)

    def fwd_bwd():
        fwd()
        render.backward_frame(scene, f, cams_dev, torch.sign(f.rgb - tgt) / f.rgb.numel(), grads)

    stream = torch.cuda.Stream()
    out = {"n_gaussians": n, "width": cam.width, "height": cam.height, "counts": f.host_counts(),
           "fwd_ms_eager": timed_ms(torch, fwd, reps), "fwd_bwd_ms_eager": timed_ms(torch, fwd_bwd, reps)}
    for key, fn in (("fwd_ms_graph", fwd), ("fwd_bwd_ms_graph", fwd_bwd)):
        gph = graph_of(torch, fn, stream)
        out[key] = 1e3 * timed_replays(torch, gph, reps, 2)
        del gph
    if f.host_counts()["flags"]:
        raise RuntimeError("capacity flag raised in the %s case: %s" % (tag, f.host_counts()))
    log("%s: fwd %.3f ms (graph %.3f), fwd+bwd %.3f ms (graph %.3f)" %
        (tag, out["fwd_ms_eager"], out["fwd_ms_graph"], out["fwd_bwd_ms_eager"], out["fwd_bwd_ms_graph"]))
    if cpu:
        img = f.rgb[0].cpu().numpy()
        d = (np.sign(img - target) / img.size).astype(np.float64)
        out["cpu_oracle"] = cpu_oracle_views([g], [cam], [d])
        log("%s cpu oracle: %s" % (tag, out["cpu_oracle"]))
    return out


def workload_small(args, torch, gs, render, synth, cpu=True):
    """4096 Gaussians in [-1,1]^3 at 256x256 (seed 0): absolute latency."""
    g, cam = synth.small_render_case(4096, seed=0)
    target = np.random.default_rng(0).uniform(size=(3, cam.height, cam.width)).astype(np.float32)
    return single_set_case(args, torch, gs, render, g, cam, target, 50, "small render 4096 @ 256x256", cpu)


def workload_single(args, torch, gs, render, synth, cpu=True):
    """1M Gaussians over a 200 x 200 x 40 m box, one 1920x1080 view (seed 1), L1 against U[0,1]."""
    g, cam, target = synth.single_view_training_case()
    return single_set_case(args, torch, gs, render, g, cam, target, 10, "single view 1M @ 1920x1080", cpu)


# -------------------------------------------------------------------------------------------
def workload_batched(args, torch, gs, render, synth):
    """16 training views of one 2M-Gaussian block in one call vs 16 plain calls."""
    dev = "cuda:0"
    W, H, V = 1600, 900, 16
    cell = 153.1
    fine, block_id, u, cells = synth.city_finest(2_000_000, seed=3, area_m2=cell * cell, grid=(1, 1))
    scene = render.DeviceScene.from_finest(fine, block_id, u, cells, fractions=(1.0,), device=dev)
    cams = synth.orbit_views((0.0, 0.0), n_views=V, radius=60.0, height=60.0, width=W, h_px=H)
    cams_dev = gs.cameras_to_device(cams, dev)
    target = torch.rand((V, 3, H, W), generator=torch.Generator(device=dev).manual_seed(3), device=dev)
    grads = [lv.zeros_like() for lv in scene.levels]
    flags = gs.GS_TUNE_SHARED_SELECTION | gs.GS_TUNE_WORK_QUEUE
    fb = render.Frame(1, V, W, H, V * scene.n_finest, 1 << 24, gs.tuning_struct(16, 16, 256, flags), device=dev)
    render.render_frame(scene, fb, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=())
    counts = fb.host_counts()

    def step():
        render.render_frame(scene, fb, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=(), check=False)
        d = torch.sign(fb.rgb - target) / fb.rgb.numel()
        render.backward_frame(scene, fb, cams_dev, d, grads)

    stream = torch.cuda.Stream()
    g = graph_of(torch, step, stream)
    t_batched = timed_replays(torch, g, args.steps, args.warmup)
    del g
    # comparator: 16 plain single-view calls, default shape, eager
    f1 = render.Frame(1, 1, W, H, scene.n_finest, 1 << 22, device=dev)
    slots = [cams_dev[v * 152:(v + 1) * 152] for v in range(V)]
    for v in range(V):
        render.render_frame(scene, f1, slots[v], mode=gs.GS_LOD_ALL_FINEST, thresholds=())

    def plain():
        for v in range(V):
            render.render_frame(scene, f1, slots[v], mode=gs.GS_LOD_ALL_FINEST, thresholds=(), check=False)
            d = torch.sign(f1.rgb - target[v:v + 1]) / f1.rgb.numel()
            render.backward_frame(scene, f1, slots[v], d, grads)

    plain()
    torch.cuda.synchronize()
    reps = max(1, args.steps // 4)
    t0 = time.perf_counter()
    for _ in range(reps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    out = {"metric": "fwd+bwd ms/view, 16 views of one 2M-Gaussian block, batched vs plain",
           "value": 1e3 * t_batched / V, "unit": "ms/view", "higher_is_better": False,
           "plain_ms_per_view": 1e3 * t_plain / V, "speedup_vs_plain": t_plain / t_batched,
           "views": V, "n_gaussians": scene.n_finest, "width": W, "height": H,
           "launch": "one batched call per step, hipGraph; shared selection + work queue",
           "records": counts["records"], "visible": counts["visible"], "pairs": counts["pairs"],
           "dtype": "f32", "data": "synthetic"}
    log("batched 16 x 2M: %.3f ms/view (plain %.3f)" % (out["value"], out["plain_ms_per_view"]))
    if not args.no_cpu:
        vv = [0, 4, 8, 12]
        render.render_frame(scene, fb, cams_dev, mode=gs.GS_LOD_ALL_FINEST, thresholds=())
        img = fb.rgb.cpu().numpy()
        tg = target.cpu().numpy()
        ds = [(np.sign(img[v] - tg[v]) / fb.rgb.numel()).astype(np.float64) for v in vv]
        out["cpu_oracle"] = cpu_oracle_views([fine] * len(vv), [cams[v] for v in vv], ds)
        log("batched cpu oracle: %s" % out["cpu_oracle"])
    return out


def workload_uneven(args, torch, gs, render, synth, tune=True):
    """32 uneven blocks x 4 views at 1280x720: LoD select + fwd + bwd batched
    (autotuned launch shape, or the library default with the work queue)."""
    from paper_2404_01133_amd import autotune
    dev = "cuda:0"
    W, H = 1280, 720
    thresholds = (200.0, 500.0)
    t_gen = time.time()
    fine, block_id, u, cells, cams = synth.uneven_finest(seed=4)
    scene = render.DeviceScene.from_finest(fine, block_id, u, cells, device=dev)
    scene.compute_bounds(4.0)
    log("uneven scene: %d finest Gaussians, %d blocks (%.1fs)" % (fine.n, scene.n_blocks, time.time() - t_gen))
    V = len(cams)
    chunk = 16  # views per batched call (bounds the record and pair buffers)
    cams_dev = gs.cameras_to_device(cams, dev)
    target = torch.rand((chunk, 3, H, W), generator=torch.Generator(device=dev).manual_seed(4), device=dev)
    grads = [lv.zeros_like() for lv in scene.levels]
    rc = chunk * scene.max_records_per_view() // 4
    refine = not args.no_refine  # chunk refinement in the batched and the per-view steps

    def chunk_slot(k):
        return cams_dev[k * chunk * 152:(k + 1) * chunk * 152]

    frames = {}

    def get_frame(tw, th):
        if (tw, th) not in frames:
            f = render.Frame(scene.n_blocks, chunk, W, H, rc, 1 << 24, gs.tuning_struct(tw, th, 256), device=dev)
            for k in range(V // chunk):
                render.render_frame(scene, f, chunk_slot(k), thresholds=thresholds, refine=refine)
            frames[(tw, th)] = f
        return frames[(tw, th)]

    def step_with(f):
        def run():
            for k in range(V // chunk):
                render.render_frame(scene, f, chunk_slot(k), thresholds=thresholds, check=False, refine=refine)
                d = torch.sign(f.rgb - target) / f.rgb.numel()
                render.backward_frame(scene, f, chunk_slot(k), d, grads)
        return run

    def make_runner(cand):
        f = get_frame(cand.tile_w, cand.tile_h)
        f.tuning = cand.tuning()

        def images():
            render.render_frame(scene, f, chunk_slot(0), thresholds=thresholds, check=False, refine=refine)
            return f.rgb.clone()
        return step_with(f), images

    if tune:
        best, report = autotune.tune("uneven_32blocks_%dviews_%dx%d" % (V, W, H), make_runner, use_cache=False,
                                     log=log)
        f = get_frame(best.tile_w, best.tile_h)
        f.tuning = best.tuning()
        tuned = {k: report[k] for k in ("best", "best_ms", "default_ms", "rejected")}
    else:
        f = get_frame(16, 16)
        f.tuning = gs.tuning_struct(16, 16, 256, gs.GS_TUNE_WORK_QUEUE)
        tuned = {"best": {"tile_w": 16, "tile_h": 16, "batch": 256, "flags": gs.GS_TUNE_WORK_QUEUE},
                 "autotuned": False}
    stream = torch.cuda.Stream()
    g = graph_of(torch, step_with(f), stream)
    t_batched = timed_replays(torch, g, max(2, args.steps // 4), 1)
    del g
    # comparator: per-view calls, default shape, eager
    f1 = render.Frame(scene.n_blocks, 1, W, H, scene.max_records_per_view(), 1 << 22, device=dev)
    slots = [cams_dev[v * 152:(v + 1) * 152] for v in range(V)]
    for v in range(V):
        render.render_frame(scene, f1, slots[v], thresholds=thresholds, refine=refine)

    def plain():
        for v in range(V):
            render.render_frame(scene, f1, slots[v], thresholds=thresholds, check=False, refine=refine)
            d = torch.sign(f1.rgb - target[v % chunk:v % chunk + 1]) / f1.rgb.numel()
            render.backward_frame(scene, f1, slots[v], d, grads)

    plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out = {"metric": "LoD fwd+bwd ms/view, 32 uneven blocks x 4 views, batched vs per-view",
           "value": 1e3 * t_batched / V, "unit": "ms/view", "higher_is_better": False,
           "per_view_default_ms_per_view": 1e3 * t_plain / V, "speedup": t_plain / t_batched,
           "views": V, "views_per_call": chunk, "width": W, "height": H, "tuning": tuned,
           "n_finest": scene.n_finest, "chunk_refinement": refine, "dtype": "f32", "data": "synthetic"}
    log("uneven 32 blocks x 4 views: %.3f ms/view (per-view calls %.3f)" % (out["value"],
                                                                          out["per_view_default_ms_per_view"]))
    if not args.no_cpu:
        from oracle import lod as olod
        vv = [0, 37, 74, 111]
        fractions = (0.30, 0.50, 1.00)
        memb = synth.level_membership(block_id, u, scene.n_blocks, fractions)
        lvl_cnt = np.stack([m[1] for m in memb], axis=1)
        bounds = np.concatenate([[0], np.cumsum(lvl_cnt[:, -1])])
        lo = np.zeros((scene.n_blocks, 3))
        hi = np.zeros((scene.n_blocks, 3))
        for b in range(scene.n_blocks):
            lo[b], hi[b] = olod.mad_bounds(fine.means[:, bounds[b]:bounds[b + 1]])
        level_ref, _ = olod.lod_select(lo, hi, cells, thresholds, [cams[v] for v in vv], lvl_cnt)
        aggs, ds = [], []
        tg = target.cpu().numpy()
        for k, v in enumerate(vv):
            parts = []
            for b in range(scene.n_blocks):
                l = level_ref[k, b]
                if l < 0:
                    continue
                idx = memb[l][0]
                parts.append((idx[(idx >= bounds[b]) & (idx < bounds[b + 1])], l))
            idx_all = np.concatenate([p_[0] for p_ in parts])
            sk = np.concatenate([np.full(len(p_[0]), 1.0 if p_[1] == 2 else 1.3, np.float32) for p_ in parts])
            aggs.append(synth.GaussianSet(fine.means[:, idx_all], (fine.scales[:, idx_all] * sk).astype(np.float32),
                                          fine.quats[:, idx_all], fine.opac[idx_all], fine.sh[:, :, idx_all]))
            render.render_frame(scene, f1, slots[v], thresholds=thresholds)
            img = f1.rgb[0].cpu().numpy()
            ds.append((np.sign(img - tg[v % chunk]) / img.size).astype(np.float64))
        out["cpu_oracle"] = cpu_oracle_views(aggs, [cams[v] for v in vv], ds)
        out["cpu_oracle"]["selected_gaussians_mean"] = float(np.mean([a_.n for a_ in aggs]))
        log("uneven cpu oracle: %s" % out["cpu_oracle"])
    return out


def workload_assign(args, torch, gs, render, synth):
    """Training-data assignment (Eqs. 3-5) of 32 poses to the 36 blocks of a
    contracted 6 x 6 partition (Table S3's MatrixCity grid, eps = 0.05) of a
    3M-Gaussian coarse prior, 960x540 renders: batched full renders, skipped
    leave-one-out renders for blocks without visible records, SSIM, Eqs. 3-5.
    Comparator: the same without skipping (every pose rendered B + 1 times)."""
    from paper_2404_01133_amd import assignment
    dev = "cuda:0"
    W, H = 960, 540
    fine, _, u, _ = synth.city_finest(3_000_000, seed=5, area_m2=1.5e6, grid=(8, 8))
    box = (-204.0, -204.0, 204.0, 204.0)   # central third of the 1225 m square (foreground)
    scene, _ = render.DeviceScene.from_partition(fine, u, box, 6, 6, fractions=(1.0,), device=dev)
    cams = synth.city_views(seed=5, heights=(100.0, 200.0), n_xy=8, width=W, height=H)
    P = len(cams)

    def run(skip):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = assignment.assign_poses(scene, cams, W, H, eps=0.05, poses_per_call=4, views_per_call=16,
                                    skip_invisible=skip)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    run(True)  # warm-up (buffers, code objects)
    reps = max(1, args.steps // 10)
    best = None
    for _ in range(reps):
        r, t = run(True)
        best = t if best is None else min(best, t)
    rn, tn = run(False)
    assert (rn["b"] == r["b"]).all()
    log("assignment: %.2f ms/pose (%d leave-one-out renders), all renders %.2f ms/pose (%d)" %
        (1e3 * best / P, r["renders"], 1e3 * tn / P, rn["renders"]))
    return {"metric": "data assignment ms/pose, 6x6 contracted blocks of a 3M-Gaussian prior, 960x540",
            "value": 1e3 * best / P, "unit": "ms/pose", "higher_is_better": False,
            "all_renders_ms_per_pose": 1e3 * tn / P, "speedup_vs_all_renders": tn / best,
            "poses": P, "blocks": scene.n_blocks, "leave_one_out_renders": r["renders"],
            "leave_one_out_renders_all": rn["renders"], "assigned_pairs": int(r["b"].sum()),
            "b1_pairs": int(r["b1"].sum()), "b2_pairs": int(r["b2"].sum()), "eps": 0.05,
            "dtype": "f32", "data": "synthetic"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2404_01133_amd import gs, render, synth

    torch.cuda.set_device(0)
    if args.workload == "lod":
        result = workload_lod(args, torch, gs, render, synth)
        if result is None:  # a profiler-only mode printed its own line
            return
        if not args.no_extra:
            # the other configurations of the scope table, timed in the same run (their own keys)
            cpu = result.get("cpu_baseline")
            plan = {}
            for key, fn in (("small_render", workload_small), ("single_view", workload_single)):
                r = fn(args, torch, gs, render, synth, cpu=not args.no_cpu)
                if "cpu_oracle" in r:
                    plan[key] = r.pop("cpu_oracle")
                result[key] = r
            for key, fn in (("batched", workload_batched),
                            ("uneven", lambda *a: workload_uneven(*a, tune=False)),
                            ("assignment", workload_assign)):
                r = fn(args, torch, gs, render, synth)
                if "cpu_oracle" in r:
                    plan[key] = r.pop("cpu_oracle")
                result[key] = r
                torch.cuda.empty_cache()
            if cpu is not None:
                cpu["other_configs"] = plan
        print(json.dumps(result))
    elif args.workload == "small":
        print(json.dumps(workload_small(args, torch, gs, render, synth, cpu=not args.no_cpu)))
    elif args.workload == "single":
        print(json.dumps(workload_single(args, torch, gs, render, synth, cpu=not args.no_cpu)))
    elif args.workload == "batched":
        print(json.dumps(workload_batched(args, torch, gs, render, synth)))
    elif args.workload == "uneven":
        print(json.dumps(workload_uneven(args, torch, gs, render, synth)))
    else:
        print(json.dumps(workload_assign(args, torch, gs, render, synth)))


if __name__ == "__main__":
    main()
