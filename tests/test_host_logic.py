"""Host logic that needs no GPU: the autotuner's search space and result cache,
and bench.py's refusal of a multi-GPU run."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_search_space_starts_at_the_library_default():
    from paper_2404_01133_amd import autotune, gs
    cands = autotune.candidates()
    keys = [(c.tile_w, c.tile_h, c.batch, c.flags) for c in cands]
    assert len(keys) == len(set(keys)) == 5 * 3 * 2
    # the first candidate is the reference of the bit-identity gate
    assert keys[0] == (16, 16, 256, 0)
    assert {k[3] for k in keys} == {0, gs.GS_TUNE_WORK_QUEUE}
    t = cands[1].tuning(extra_flags=gs.GS_TUNE_SHARED_SELECTION)
    assert (t.tile_w, t.tile_h, t.batch) == (cands[1].tile_w, cands[1].tile_h, cands[1].batch)
    assert t.flags == cands[1].flags | gs.GS_TUNE_SHARED_SELECTION


def test_autotune_cache_round_trip_and_corrupt_file(tmp_path, monkeypatch):
    from paper_2404_01133_amd import autotune
    path = tmp_path / "sub" / "cache.json"
    monkeypatch.setenv("GS_AUTOTUNE_CACHE", str(path))
    assert autotune.cache_path() == str(path)
    assert autotune._load_cache() == {}  # missing file
    entry = {"dev|key": {"best": {"tile_w": 32, "tile_h": 8, "batch": 128, "flags": 2}, "best_ms": 1.5}}
    autotune._store_cache(entry)  # creates the directory, replaces atomically
    assert json.loads(path.read_text()) == entry
    assert autotune._load_cache() == entry
    assert not [p for p in os.listdir(path.parent) if ".tmp" in p]
    path.write_text("{not json")
    assert autotune._load_cache() == {}


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")  # no JSON result line
