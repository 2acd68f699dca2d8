"""gs_bin_sort_static (workspace in the library's static device array, no
allocation) against gs_bin_sort (caller's workspace) on the same projected
frames: two calls in a row, the second on a smaller input, so the second runs
over what the first left in the array."""
import numpy as np
import pytest
import torch

from paper_2404_01133_amd import gs, render, synth

from gpu_util import scaled_city

pytestmark = pytest.mark.gpu


def _projected_frame(n, seed, n_xy, W, H, pair_capacity):
    """A block-wise LoD frame of a small city, rendered once (selection and
    projection are what both binning calls read)."""
    bs = scaled_city(n, seed=seed)
    scene = render.DeviceScene.from_block_scene(bs)
    scene.compute_bounds(4.0)
    cams = synth.city_views(seed=seed, n_xy=n_xy, width=W, height=H)
    V = len(cams)
    f = render.Frame(bs.n_blocks, V, W, H, V * scene.max_records_per_view(), pair_capacity,
                     gs.tuning_struct(16, 16, 256, gs.GS_TUNE_WORK_QUEUE))
    render.render_frame(scene, f, gs.cameras_to_device(cams))
    torch.cuda.synchronize()
    return f


def _bin(f, static):
    """Bin f's records into fresh output buffers with one of the two entry points."""
    d = f.device
    out = dict(tiles=torch.full((f.pair_capacity,), -1, dtype=torch.int32, device=d),
               recs=torch.full((f.pair_capacity,), -1, dtype=torch.int32, device=d),
               ranges=torch.full((f.n_tiles, 2), -1, dtype=torch.int32, device=d),
               queue=torch.full((2 + f.n_tiles,), 7, dtype=torch.int32, device=d),
               counts=f.counts.clone())
    args = (f.records, f.depth_keys, f.tiles_touched, f.V, f.W, f.H, f.tuning, f.record_capacity, f.pair_capacity,
            out["tiles"], out["recs"], out["ranges"], out["counts"])
    if static:
        gs.bin_sort_static(*args, tile_queue=out["queue"])
    else:
        gs.bin_sort(*args, f.sort_ws, tile_queue=out["queue"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    ca, cb = a["counts"], b["counts"]
    np.testing.assert_array_equal(ca, cb)
    assert ca[gs.GS_COUNT_FLAGS] == 0
    m = int(ca[gs.GS_COUNT_PAIRS])
    assert m > 0
    np.testing.assert_array_equal(a["tiles"][:m], b["tiles"][:m])
    np.testing.assert_array_equal(a["recs"][:m], b["recs"][:m])
    np.testing.assert_array_equal(a["ranges"], b["ranges"])
    # the queue's order inside a length bin depends on atomics: compare it as a
    # permutation of the tiles in non-increasing bins, heads reset
    for q in (a["queue"], b["queue"]):
        assert q[0] == 0 and q[1] == 0
        tiles = q[2:]
        assert sorted(tiles.tolist()) == list(range(tiles.shape[0]))
        lens = a["ranges"][tiles, 1] - a["ranges"][tiles, 0]
        bins = np.where(lens == 0, 32, 31 - np.floor(np.log2(np.maximum(lens, 1))).astype(np.int64))
        assert (np.diff(bins) >= 0).all()
    return m


def test_static_scratch_bin_sort_equals_workspace_bin_sort_twice():
    big = _projected_frame(100_000, seed=60, n_xy=2, W=480, H=270, pair_capacity=1 << 21)
    small = _projected_frame(40_000, seed=61, n_xy=1, W=160, H=96, pair_capacity=1 << 17)
    assert small.record_capacity < big.record_capacity and small.pair_capacity < big.pair_capacity
    for tag, f in (("first call, larger input", big), ("second call, smaller input", small)):
        print("case:", tag, "records", f.record_capacity, "pairs", f.pair_capacity, flush=True)
        ref = _bin(f, static=False)
        got = _bin(f, static=True)
        m = _same(got, ref)
        print("  pairs", m, flush=True)


def test_static_scratch_rejects_capacities_beyond_the_array():
    f = _projected_frame(20_000, seed=62, n_xy=1, W=160, H=96, pair_capacity=1 << 16)
    before = f.counts.clone()
    need = gs.workspace_bytes(gs.GS_WS_BIN_SORT, 1 << 22, 1 << 24, 1, 160, 96, f.tuning)
    assert need > gs.GS_STATIC_SCRATCH_BYTES
    with pytest.raises(gs.GsError) as e:
        gs.bin_sort_static(f.records, f.depth_keys, f.tiles_touched, f.V, f.W, f.H, f.tuning, 1 << 22, 1 << 24,
                           f.pair_tiles, f.pair_records, f.tile_ranges, f.counts)
    assert e.value.status == gs.GS_ERR_SCRATCH
    torch.cuda.synchronize()
    assert torch.equal(f.counts, before)  # nothing was launched
