"""Rectangular boxes (Lx != Ly) and regions with several rings: holes
(enclaves whose host region has a clockwise ring on the same vertices) and
multipolygons (two cells in one region).  The paper's equations hold for any
Lx x Ly box (Eq. 5-7) and a region may be any set of polygons (main text,
areas as sums of signed polygon areas); every step is checked against the
oracle at the bars of the square maps: areas at rtol 1e-12 on identical
vertices, densities within 1e-5 of the density scale, positions within
1e-4 grid units with the oracle's schedule replayed, areas after a round
within dx times each region's L1 perimeter, whole loops by outcome, and the
gradient against the oracle's central differences.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1802_07625_amd as ffb
import synth
from gpu_util import area_bound, dev_f64, gpu_gradient, map_points, new_ctx, stats_of, to_np

pytestmark = pytest.mark.gpu


def _setup(name):
    m = synth.workload(name)
    pts = map_points(m)
    d = torch.as_tensor(pts, device="cuda")
    geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    print(f"[rect] {name} lx={m.lx} ly={m.ly} R={m.n_regions} rings={m.n_rings} "
          f"V={m.n_vertices} P={pts.shape[0]}", flush=True)
    return m, pts, d, geom, ctx, dev_f64(m.value)


def test_maps_have_holes_and_multipolygons():
    for name in ("rect_128x64", "rect_256x512", "rect_1024x512"):
        m = synth.workload(name)
        counts = np.bincount(m.ring_region, minlength=m.n_regions)
        signed = []
        for g in range(m.n_rings):
            p = m.xy[m.ring_vidx[m.ring_offsets[g]:m.ring_offsets[g + 1]]].astype(np.float64)
            signed.append(0.5 * np.sum(p[:, 0] * np.roll(p[:, 1], -1)
                                       - np.roll(p[:, 0], -1) * p[:, 1]))
        assert m.lx != m.ly and counts.max() >= 2 and min(signed) < 0


@pytest.mark.parametrize("name", ["rect_128x64", "rect_256x512"])
def test_one_iteration_replayed(name):
    m, pts, d, geom, ctx, value = _setup(name)
    ref = oracle.iterate(m, m.value, pts.astype(np.float64), m.n_vertices, 4.0)
    area0, _, _ = ctx.area_error(geom, value)
    rho, pad = ctx.density(geom, value, area0)
    fields, rb = ctx.flux(rho, 4.0)
    stats, _ = ctx.integrate(fields, rb, d, ffb.IntegrateOpts(), replay_h=dev_f64(ref.h))
    area1, err1, mx1 = ctx.area_error(geom, value)
    assert ctx.sync(check=False) == 0
    assert stats_of(stats)["accepted"] == ref.accepted
    np.testing.assert_allclose(to_np(area0), ref.area_before, rtol=1e-12)
    assert to_np(rho).shape == (m.ly, m.lx)
    np.testing.assert_allclose(to_np(rho), ref.rho, rtol=0, atol=1e-11 * np.abs(ref.rho).max())
    dx = np.abs(to_np(d).astype(np.float64) - ref.points).max()
    print(f"[rect] {name} steps={ref.accepted} max|dx|={dx:.3e} "
          f"max err gpu={float(mx1):.6f} oracle={ref.max_err_after:.6f}", flush=True)
    assert dx < 1e-4
    bound = area_bound(m, ref.points[:m.n_vertices], dx) + 1e-12 * np.abs(ref.area_after)
    assert np.all(np.abs(to_np(area1) - ref.area_after) <= bound)


def test_loop_converges_like_the_oracle():
    m, pts, d, geom, ctx, value = _setup("rect_128x64")
    p = pts.astype(np.float64)
    ref_rounds = None
    for k in range(30):
        r = oracle.iterate(m, m.value, p, m.n_vertices, oracle.default_sigma(k))
        p = r.points
        if r.max_err_after < 0.01:
            ref_rounds = k + 1
            break
    area, rounds, mx = None, None, None
    for k in range(30):
        res = ffb.iterate(ctx, geom, value, d, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        if mx < 0.01:
            rounds = k + 1
            break
    assert ctx.sync(check=False) == 0
    print(f"[rect] loop rounds gpu={rounds} oracle={ref_rounds} final={mx:.4f}", flush=True)
    assert ref_rounds is not None and rounds is not None and abs(rounds - ref_rounds) <= 1
    # the final maps agree on their angular distortion to the size of the
    # position differences the rounds accumulate
    stats, _, _ = ctx.distortion(d[m.n_vertices:])
    dref = oracle.distortion(p[m.n_vertices:], m.lx, m.ly)
    s = to_np(stats)
    print(f"[rect] distortion e_a gpu={s[0]:.5f} oracle={dref.e_a:.5f}", flush=True)
    assert s[0] == pytest.approx(dref.e_a, rel=2e-2)


def test_full_size_areas_and_density():
    m = synth.workload("rect_1024x512")
    print(f"[rect] rect_1024x512 E={m.n_entries}", flush=True)
    pts = torch.as_tensor(m.xy.astype(np.float32), device="cuda")
    geom = ffb.Geometry.from_map(m, xy=pts)
    ctx = new_ctx(m.lx, m.ly, m.n_vertices)
    area, _, _ = ctx.area_error(geom, dev_f64(m.value))
    rho, pad = ctx.density(geom, dev_f64(m.value), area)
    ctx.sync()
    a_ref = oracle.region_areas(m)
    np.testing.assert_allclose(to_np(area), a_ref, rtol=1e-11)
    rho_ref, _ = oracle.density(m, m.value, a_ref)
    np.testing.assert_allclose(to_np(rho), rho_ref, rtol=0, atol=1e-11 * np.abs(rho_ref).max())


def test_full_size_loop_converges():
    m, pts, d, geom, ctx, value = _setup("rect_1024x512")
    area, mx = None, None
    for k in range(30):
        res = ffb.iterate(ctx, geom, value, d, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        if mx < 0.01:
            break
    assert ctx.sync(check=False) == 0
    print(f"[rect] rect_1024x512 rounds={k + 1} final={mx:.4f}", flush=True)
    assert mx < 0.01
    # every point stays in the box
    p = to_np(d)
    assert p[:, 0].min() >= 0 and p[:, 0].max() <= m.lx
    assert p[:, 1].min() >= 0 and p[:, 1].max() <= m.ly


def test_backward_matches_oracle_fd():
    sig = [oracle.default_sigma(k) for k in range(3)]
    m = synth.workload("rect_128x64")
    ref = oracle.rounds(m, m.density, sig)
    g_fd = oracle.fd_gradient(m, m.density, sig, ref.schedules, step=1e-4)
    loss, g = gpu_gradient(m, m.density, sig, ref.schedules)
    err = np.max(np.abs(g - g_fd)) / np.max(np.abs(g_fd))
    print(f"[rect] gradient loss gpu={loss:.6e} oracle={ref.loss:.6e} max rel err={err:.3e}",
          flush=True)
    assert abs(loss - ref.loss) <= 1e-3 * ref.loss
    assert err < 1e-3


def test_batch_mixes_rectangular_and_square_maps():
    names = ["rect_128x64", "c4_2", "rect_256x512", "c4_8"]
    maps = [synth.workload(n) for n in names]
    refs = [oracle.iterate(mp, mp.value, mp.xy.astype(np.float64), mp.n_vertices, 4.0)
            for mp in maps]
    offs = np.cumsum([0] + [len(r.h) for r in refs]).astype(np.int32)
    b = ffb.Batch(maps)
    print(f"[rect] batch shapes={b.shapes()}", flush=True)
    b.step(ffb.BatchOpts(use_graph=False),
           replay=(torch.as_tensor(offs, device="cuda"), dev_f64(np.concatenate([r.h for r in refs]))))
    rounds, mx, stats, area = b.results()
    area = to_np(area)
    for k, (mp, r) in enumerate(zip(maps, refs)):
        p = to_np(b.map_points(k)).astype(np.float64)
        dx = np.abs(p - r.points).max()
        print(f"[rect] batch {names[k]} {mp.lx}x{mp.ly} max|dx|={dx:.3e}", flush=True)
        assert dx < 1e-4
        a = area[b.region_offsets[k]:b.region_offsets[k + 1]]
        bound = area_bound(mp, r.points[:mp.n_vertices], dx) + 1e-12 * np.abs(r.area_after)
        assert np.all(np.abs(a - r.area_after) <= bound)
    # and a full run ends like each map's own loop
    b2 = ffb.Batch(maps)
    b2.run(ffb.BatchOpts())
    rounds, mx, _, _ = b2.results()
    for k, mp in enumerate(maps):
        pts = torch.as_tensor(mp.xy.astype(np.float32), device="cuda")
        geom = ffb.Geometry.from_map(mp, xy=pts)
        ctx = new_ctx(mp.lx, mp.ly, pts.shape[0])
        area1, r1, m1 = None, 30, None
        for j in range(30):
            res = ffb.iterate(ctx, geom, dev_f64(mp.value), pts, ffb.default_sigma(j),
                              area_before=area1)
            area1 = res.area_after
            m1 = float(res.max_err_after)
            if m1 < 0.01:
                r1 = j + 1
                break
        print(f"[rect] batch run {names[k]} rounds={rounds[k]} single={r1}", flush=True)
        assert (mx[k] < 0.01) == (m1 < 0.01) and abs(int(rounds[k]) - r1) <= 1
