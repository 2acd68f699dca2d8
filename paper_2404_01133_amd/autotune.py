"""Autotuner for the tile kernels' launch shape.

Searches tile shape x LDS batch depth x work-queue mode for a given workload,
times every candidate on the device (HIP-graph replays timed with HIP events),
and accepts a candidate only if its images are bit-identical to those of the
default shape (the compositing gate makes the image independent of the tile
shape, so any difference is a bug, not a trade-off).  Results are cached as
JSON keyed by (device name, workload key); the cache path comes from
GS_AUTOTUNE_CACHE or defaults to ~/.cache/gs_autotune.json.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import torch

from . import gs

TILE_SHAPES = ((16, 16), (8, 8), (16, 8), (32, 8), (32, 16))
BATCHES = (256, 128, 64)  # the first candidate is the library default 16x16 / 256
QUEUE_FLAGS = (0, gs.GS_TUNE_WORK_QUEUE)


@dataclass
class Candidate:
    tile_w: int
    tile_h: int
    batch: int
    flags: int

    def tuning(self, extra_flags=0) -> gs.gs_tuning:
        return gs.tuning_struct(self.tile_w, self.tile_h, self.batch, self.flags | extra_flags)

    def as_dict(self):
        return dict(tile_w=self.tile_w, tile_h=self.tile_h, batch=self.batch, flags=self.flags)


def candidates(tile_shapes=TILE_SHAPES, batches=BATCHES, queue_flags=QUEUE_FLAGS):
    return [Candidate(tw, th, b, f) for (tw, th) in tile_shapes for b in batches for f in queue_flags]


def cache_path() -> str:
    return os.environ.get("GS_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gs_autotune.json"))


def _load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_graph(run, reps=3, warmup=1, stream=None) -> float:
    """Capture `run()` in a HIP graph and return the mean replay time in ms.

    `stream` first waits for the caller's current stream, so work still queued
    there (a copy of the last output, say) finishes before `run()` overwrites
    the buffers it reads."""
    stream = stream or torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        run()  # eager warm-up on the capture stream
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            run()
        for _ in range(warmup):
            g.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        e1.synchronize()
    del g
    return e0.elapsed_time(e1) / reps


def tune(key: str, make_runner, search=None, reps=3, use_cache=True, log=None, stream=None):
    """Pick the fastest launch shape for a workload.

    make_runner(candidate) -> (run, images): `run()` issues the workload on the
    current stream without host synchronisation; `images()` returns the output
    images (a tensor) after a run.  The first candidate of `search` is the
    reference for the bit-identity gate.  All candidates are timed on `stream`
    (one new stream if None).  Returns (best Candidate, report)."""
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    ckey = "%s|%s" % (dev, key)
    cache = _load_cache() if use_cache else {}
    if ckey in cache:
        c = cache[ckey]["best"]
        return Candidate(c["tile_w"], c["tile_h"], c["batch"], c["flags"]), cache[ckey]
    search = search or candidates()
    stream = stream or torch.cuda.Stream()
    ref = None
    results = []
    for cand in search:
        run, images = make_runner(cand)
        ms = time_graph(run, reps=reps, stream=stream)
        run()
        torch.cuda.synchronize()
        img = images()
        if ref is None:
            ref = img.clone()
            ok = True
        else:
            ok = bool(torch.equal(img, ref))
        # the copies above are queued on the current stream; the next candidate's
        # runs reuse the frame buffers they read
        torch.cuda.synchronize()
        results.append(dict(cand.as_dict(), ms=ms, identical=ok))
        if log:
            log("autotune %s: %s %.4f ms %s" % (key, cand.as_dict(), ms, "" if ok else "REJECTED (image differs)"))
        del run, images
    good = [r for r in results if r["identical"]]
    best = min(good, key=lambda r: r["ms"])
    report = {"best": {k: best[k] for k in ("tile_w", "tile_h", "batch", "flags")}, "best_ms": best["ms"],
              "default_ms": results[0]["ms"], "rejected": sum(1 for r in results if not r["identical"]),
              "results": results}
    if use_cache:
        cache[ckey] = report
        _store_cache(cache)
    return Candidate(best["tile_w"], best["tile_h"], best["batch"], best["flags"]), report
