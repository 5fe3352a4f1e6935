"""Batched runs (many maps of different grid sizes in one pass per phase).

* Round 0 of every map with the oracle's accepted steps replayed (per map)
  matches the oracle: positions within the stated 1e-4 grid units, areas
  within the bound those positions imply (dx times the region's L1
  perimeter; the 1e-6 relative area tolerance itself applies to the area
  kernel on identical vertices, see test_gpu_geometry).
* A full batched run ends like each map's own loop through the single-map
  entry points: the same maps stop below 1 % (round counts within one), the
  others reach the round cap with the same final error (maps whose smallest
  regions are a few grid cells stall above 1 % at their grid size, in both).
* Launch shapes (transform and integration workgroup sizes) and graph replay
  change where work happens, not what is computed: results are bitwise equal.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1802_07625_amd as ffb
import synth
from gpu_util import area_bound, dev_f64, to_np

pytestmark = pytest.mark.gpu

SMALL = ["c4_2", "c4_3", "c4_8", "c4_1", "c4_11", "c4_6"]      # L = 128, 128, 256, 512, 256, 128


def _maps(names):
    return [synth.workload(n) for n in names]


def test_round0_replayed_matches_oracle():
    maps = _maps(SMALL)
    refs = [oracle.iterate(m, m.value, m.xy.astype(np.float64), m.n_vertices, 4.0) for m in maps]
    offs = np.cumsum([0] + [len(r.h) for r in refs]).astype(np.int32)
    steps = np.concatenate([r.h for r in refs])
    b = ffb.Batch(maps)
    print(f"[batch] maps={len(maps)} points={b.points.shape[0]} shapes={b.shapes()}", flush=True)
    replay = (torch.as_tensor(offs, device="cuda"), dev_f64(steps))
    b.step(ffb.BatchOpts(use_graph=False), replay=replay)
    rounds, mx, stats, area = b.results()
    area = to_np(area)
    for k, (m, r) in enumerate(zip(maps, refs)):
        assert stats[k, 0] == len(r.h) and stats[k, 3] == 0, (k, stats[k])
        p = to_np(b.map_points(k)).astype(np.float64)
        dx = np.abs(p - r.points).max()
        a = area[b.region_offsets[k]:b.region_offsets[k + 1]]
        da = np.abs(a / r.area_after - 1).max()
        print(f"[batch] {SMALL[k]} L={m.lx} V={m.n_vertices} steps={len(r.h)} max|dx|={dx:.3e} "
              f"max rel d area={da:.3e} max err gpu={mx[k]:.6f} oracle={r.max_err_after:.6f}",
              flush=True)
        assert dx < 1e-4
        bound = area_bound(m, r.points[:m.n_vertices], dx) + 1e-12 * np.abs(r.area_after)
        assert np.all(np.abs(a - r.area_after) <= bound)


def _single_loop(m, max_rounds=30):
    pts = torch.as_tensor(m.xy.astype(np.float32), device="cuda")
    geom = ffb.Geometry.from_map(m, xy=pts)
    ctx = ffb.Context(m.lx, m.ly, max_points=pts.shape[0])
    value = dev_f64(m.value)
    area = None
    for k in range(max_rounds):
        res = ffb.iterate(ctx, geom, value, pts, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        if mx < 0.01:
            return k + 1, mx, to_np(pts)
    return max_rounds, mx, to_np(pts)


def test_run_matches_single_map_loops():
    names = [f"c4_{i}" for i in range(12)]
    maps = _maps(names)
    b = ffb.Batch(maps)
    it = b.run(ffb.BatchOpts())
    rounds, mx, stats, _ = b.results()
    print(f"[batch] run iterations={it} rounds={rounds.tolist()}", flush=True)
    assert it == rounds.max()
    for k, m in enumerate(maps):
        r1, mx1, p1 = _single_loop(m)
        print(f"[batch] {names[k]} L={m.lx} R={m.n_regions} rounds batch={rounds[k]} "
              f"single={r1} max err batch={mx[k]:.4f} single={mx1:.4f}", flush=True)
        assert (mx[k] < 0.01) == (mx1 < 0.01)
        assert abs(int(rounds[k]) - r1) <= 1
        if mx1 >= 0.01:
            assert mx[k] == pytest.approx(mx1, rel=1e-3)


def _run(names, use_graph=True, shapes=None, extra=False):
    maps = _maps(names)
    ex = [synth.grid_nodes(m.lx, m.ly) for m in maps] if extra else None
    b = ffb.Batch(maps, extra_points=ex)
    if shapes:
        b.set_shapes(*shapes)
    it = b.run(ffb.BatchOpts(use_graph=use_graph))
    rounds, mx, stats, area = b.results()
    return it, rounds, mx, to_np(b.points), to_np(area)


def test_graph_replay_equals_direct_launches():
    names = ["c4_2", "c4_8", "c4_1", "c4_3"]
    a = _run(names, use_graph=True)
    b = _run(names, use_graph=False)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[3], b[3])
    np.testing.assert_array_equal(a[4], b[4])


def test_launch_shapes_do_not_change_results():
    names = ["c4_2", "c4_8", "c4_1"]
    a = _run(names, shapes=(64, 256), extra=True)
    b = _run(names, shapes=(512, 1024), extra=True)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[3], b[3])
    np.testing.assert_array_equal(a[4], b[4])


def test_autotune_picks_valid_shapes_and_keeps_results():
    names = ["c4_2", "c4_8", "c4_1"]
    ref = _run(names)
    maps = _maps(names)
    b = ffb.Batch(maps)
    sh = b.autotune(ffb.BatchOpts())
    print(f"[batch] autotuned {sh}", flush=True)
    assert sorted(sh["widths"]) == sorted({m.lx for m in maps})
    assert all(t in (64, 128, 256, 512) for t in sh["fft_threads"])
    assert sh["advect_threads"] in (256, 512, 1024)
    it = b.run(ffb.BatchOpts())
    rounds, _, _, area = b.results()
    assert it == ref[0]
    np.testing.assert_array_equal(to_np(b.points), ref[3])


def test_batch_rejects_bad_descriptions():
    import ctypes
    m = synth.workload("c4_2")
    b = ffb.Batch([m])
    b.close()
    d = ffb.api.FFBBatchDesc()
    h = ctypes.c_void_p()
    assert ffb.lib().ffb_batch_create(ctypes.byref(h), ctypes.byref(d), None) == ffb.FFB_E_INVALID
    with pytest.raises(ffb.FFBError):
        b2 = ffb.Batch([m])
        b2.set_shapes(96, 0)


# Maps whose transform lengths reach every group shape of the batched
# transforms: rows and columns of length 8, 16, 32 and 64 (groups of 1 to 8
# lanes, several groups per wavefront) and 1024 (a group of two wavefronts,
# with the cross-wavefront scan and barriers).
EXTREME = [
    dict(L=8, ly=16, n_seeds=3, seed=41, density="lognormal", inner=(1.0, 7.0),
         inner_y=(2.0, 14.0), target_vertices=80),
    dict(L=32, ly=64, n_seeds=6, seed=42, density="lognormal", inner=(4.0, 28.0),
         inner_y=(8.0, 56.0), target_vertices=600),
    dict(L=1024, ly=16, n_seeds=8, seed=43, density="lognormal", inner=(100.0, 924.0),
         inner_y=(2.0, 14.0), target_vertices=3000),
    dict(L=64, ly=1024, n_seeds=8, seed=44, density="lognormal", inner=(8.0, 56.0),
         inner_y=(100.0, 924.0), target_vertices=3000),
]


@pytest.mark.parametrize("fft_threads", [64, 512])
def test_round0_replayed_matches_oracle_at_every_transform_length(fft_threads):
    from synth.voronoi import make_map
    maps = [make_map(name=f"x{k}", **kw) for k, kw in enumerate(EXTREME)]
    refs = [oracle.iterate(m, m.value, m.xy.astype(np.float64), m.n_vertices, 4.0) for m in maps]
    offs = np.cumsum([0] + [len(r.h) for r in refs]).astype(np.int32)
    steps = np.concatenate([r.h for r in refs])
    b = ffb.Batch(maps)
    b.set_shapes(fft_threads, 0)
    print(f"[batch] extreme sizes shapes={b.shapes()}", flush=True)
    assert sorted(b.shapes()["widths"]) == [8, 16, 32, 64, 1024]
    replay = (torch.as_tensor(offs, device="cuda"), dev_f64(steps))
    b.step(ffb.BatchOpts(use_graph=False), replay=replay)
    rounds, mx, stats, area = b.results()
    area = to_np(area)
    for k, (m, r) in enumerate(zip(maps, refs)):
        assert stats[k, 0] == len(r.h) and stats[k, 3] == 0, (k, stats[k])
        p = to_np(b.map_points(k)).astype(np.float64)
        dx = np.abs(p - r.points).max()
        a = area[b.region_offsets[k]:b.region_offsets[k + 1]]
        print(f"[batch] {m.lx}x{m.ly} V={m.n_vertices} steps={len(r.h)} max|dx|={dx:.3e}",
              flush=True)
        assert dx < 1e-4
        bound = area_bound(m, r.points[:m.n_vertices], dx) + 1e-12 * np.abs(r.area_after)
        assert np.all(np.abs(a - r.area_after) <= bound)
