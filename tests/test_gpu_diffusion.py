"""The diffusion-cartogram variant (SI Appendix, section 2, the diffusion
choice of f_mn) on the device against the oracle.

* Fields rho(t), J(t) at several times from the same FP32 raster: within
  1e-5 of each field's scale (the bar of the FP32 transforms of the main
  method); at t = 0 rho equals the main method's blurred density bit for
  bit (the same forward transform and the same inverse).
* A round with the oracle's accepted steps replayed: positions within the
  stated 1e-4 grid units, areas within dx times the L1 perimeters.
* Whole loops by outcome (rounds to < 1 %, +-1), graph replay against
  direct launches bit for bit, and the error paths.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1802_07625_amd as ffb
import synth
from gpu_util import area_bound, dev_f32, dev_f64, map_points, new_ctx, stats_of, to_np

pytestmark = pytest.mark.gpu


def _interior(fields, lx, ly):
    f = to_np(fields).reshape(ly + 2, lx + 2, 4)[1:-1, 1:-1]
    return f[..., 0].astype(np.float64), f[..., 1].astype(np.float64), f[..., 2].astype(np.float64)


def _raster(m):
    a = oracle.region_areas(m)
    rho, _ = oracle.density(m, m.value, a)
    return rho


@pytest.mark.parametrize("name,sigma", [("c1_L64", 4.0), ("rect_128x64", 2.0), ("c2_L512", 4.0)])
@pytest.mark.parametrize("t", [0.0, 7.5, 400.0, 30000.0])
def test_fields_match_oracle(name, sigma, t):
    m = synth.workload(name)
    rho = _raster(m)
    coef, rb = oracle.coefficients(rho, sigma)
    F = oracle.diffusion_fields(coef, t)
    ctx = new_ctx(m.lx, m.ly)
    print(f"[diffusion] fields {name} sigma={sigma} t={t}", flush=True)
    fields = ctx.diffusion_fields(dev_f64(rho), sigma, t)
    assert ctx.sync(check=False) == 0
    jx, jy, r = _interior(fields, m.lx, m.ly)
    for got, ref, what in ((jx, F.jx, "jx"), (jy, F.jy, "jy"), (r, F.rho_s, "rho")):
        scale = np.abs(ref).max()
        err = np.abs(got - ref).max()
        print(f"[diffusion]   {what} scale={scale:.3e} max err={err:.3e}", flush=True)
        assert err <= 1e-5 * scale


def test_time_zero_density_equals_main_method_full_size():
    """At t = 0 the diffusion density is the blurred density of the main
    method (ffb_flux, FP64 transforms rounded once); the diffusion fields
    come from FP32 transforms, so the two agree to their rounding: 1e-6 of
    the largest density."""
    m = synth.workload("c3_L1024")
    rng = np.random.default_rng(0)
    rho = dev_f64(rng.lognormal(0.0, 1.0, (m.ly, m.lx)))
    ctx = new_ctx(m.lx, m.ly)
    f_ffb, _ = ctx.flux(rho, 4.0)
    f_diff = ctx.diffusion_fields(rho, 4.0, 0.0)
    assert ctx.sync(check=False) == 0
    a = to_np(f_ffb).reshape(m.ly + 2, m.lx + 2, 4)[..., 2].astype(np.float64)
    b = to_np(f_diff).reshape(m.ly + 2, m.lx + 2, 4)[..., 2].astype(np.float64)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-6 * np.abs(a).max())


def _gpu_round(m, pts, sigma, replay=None, opts=None):
    d = torch.as_tensor(pts, device="cuda")
    geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    value = dev_f64(m.value)
    area0, _, _ = ctx.area_error(geom, value)
    rho, _ = ctx.density(geom, value, area0)
    stats, h = ctx.diffusion(rho, sigma, d, opts=opts,
                             replay_h=None if replay is None else dev_f64(replay))
    area1, err1, mx1 = ctx.area_error(geom, value)
    code = ctx.sync(check=False)
    return ctx, d, stats_of(stats), to_np(h), to_np(area1), float(mx1), code


@pytest.mark.parametrize("name", ["c1_L64", "rect_128x64", "c4_8"])
def test_round_replayed_matches_oracle(name):
    m = synth.workload(name)
    pts = map_points(m)
    ref = oracle.iterate_diffusion(m, m.value, pts.astype(np.float64), m.n_vertices, 4.0)
    print(f"[diffusion] round {name} L={m.lx}x{m.ly} P={pts.shape[0]} steps={ref.accepted}",
          flush=True)
    ctx, d, s, h, area1, mx1, code = _gpu_round(m, pts, 4.0, replay=ref.h)
    assert code == 0 and s["status"] == 0 and s["accepted"] == ref.accepted
    dx = np.abs(to_np(d).astype(np.float64) - ref.points).max()
    print(f"[diffusion]   max|dx|={dx:.3e} max err gpu={mx1:.5f} oracle={ref.max_err_after:.5f}",
          flush=True)
    assert dx < 1e-4
    bound = area_bound(m, ref.points[:m.n_vertices], dx) + 1e-12 * np.abs(ref.area_after)
    assert np.all(np.abs(area1 - ref.area_after) <= bound)


def test_adaptive_round_matches_oracle_schedule():
    m = synth.workload("c1_L64")
    pts = map_points(m)
    ref = oracle.iterate_diffusion(m, m.value, pts.astype(np.float64), m.n_vertices, 4.0)
    ctx, d, s, h, area1, mx1, code = _gpu_round(m, pts, 4.0)
    print(f"[diffusion] adaptive accepted gpu={s['accepted']} oracle={ref.accepted} "
          f"rejected {s['rejected']}/{ref.rejected}", flush=True)
    assert code == 0 and s["status"] == 0
    assert abs(s["accepted"] - ref.accepted) <= 1
    assert mx1 == pytest.approx(ref.max_err_after, rel=1e-3)


def test_loop_converges_like_the_oracle():
    m = synth.workload("c1_L64")
    pts = map_points(m)
    p = pts.astype(np.float64)
    ref_rounds = None
    for k in range(30):
        r = oracle.iterate_diffusion(m, m.value, p, m.n_vertices, oracle.default_sigma(k))
        p = r.points
        if r.max_err_after < 0.01:
            ref_rounds = k + 1
            break
    d = torch.as_tensor(pts, device="cuda")
    geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    value = dev_f64(m.value)
    area, rounds, mx = None, None, None
    for k in range(30):
        res = ffb.iterate_diffusion(ctx, geom, value, d, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        if mx < 0.01:
            rounds = k + 1
            break
    assert ctx.sync(check=False) == 0
    print(f"[diffusion] loop rounds gpu={rounds} oracle={ref_rounds} final={mx:.4f}", flush=True)
    assert ref_rounds is not None and rounds is not None and abs(rounds - ref_rounds) <= 1


def test_graph_equals_direct_launches():
    m = synth.workload("rect_128x64")
    pts = map_points(m)
    out = []
    for graph in (1, 0):
        d = torch.as_tensor(pts, device="cuda")
        geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
        ctx = new_ctx(m.lx, m.ly, pts.shape[0])
        ctx.set_option(ffb.OPT_DIFFUSION_GRAPH, graph)
        value = dev_f64(m.value)
        a0, _, _ = ctx.area_error(geom, value)
        rho, _ = ctx.density(geom, value, a0)
        stats, h = ctx.diffusion(rho, 4.0, d)
        assert ctx.sync(check=False) == 0
        out.append((to_np(d), stats_of(stats), to_np(h)))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_repeated_calls_and_ragged_point_counts():
    m = synth.workload("c1_L64")
    rho = dev_f64(_raster(m))
    ctx = new_ctx(m.lx, m.ly, 1000)
    base = map_points(m)
    res, sched = [], None
    for n in (1000, 37, 0, 1000):
        d = torch.as_tensor(base[:n].copy(), device="cuda").reshape(-1, 2)
        replay = sched if n == 37 else None          # the 1000-point run's steps
        stats, h = ctx.diffusion(rho, 4.0, d, replay_h=replay)
        s = stats_of(stats)
        assert ctx.sync(check=False) == 0 and s["status"] == 0
        if sched is None:
            sched = h[:s["accepted"]].clone()
        res.append(to_np(d))
    # the same input gives the same output; points move independently of the
    # others once the steps are fixed
    np.testing.assert_array_equal(res[0], res[3])
    np.testing.assert_array_equal(res[1], res[0][:37])
    assert res[2].shape == (0, 2)


def test_errors():
    m = synth.workload("c1_L64")
    rho = dev_f64(_raster(m))
    ctx = new_ctx(m.lx, m.ly, 100)
    d0 = torch.as_tensor(map_points(m)[:100].copy(), device="cuda")
    # too few attempts: status in stats and the sticky word, points unchanged
    d = d0.clone()
    stats, _ = ctx.diffusion(rho, 4.0, d, opts=ffb.IntegrateOpts(max_attempts=3))
    assert ctx.sync(check=False) == ffb.FFB_E_MAX_ATTEMPTS
    assert stats_of(stats)["status"] == ffb.FFB_E_MAX_ATTEMPTS
    assert torch.equal(d, d0)
    ctx.reset_status()
    # host-side validation
    with pytest.raises(ffb.FFBError):
        ctx.diffusion(rho, 4.0, d, t_end=-1.0)
    with pytest.raises(ffb.FFBError):
        ctx.diffusion(rho, -1.0, d)
    with pytest.raises(ffb.FFBError):
        ctx.diffusion_fields(rho, 4.0, float("nan"))
    # a non-positive density: rho(t) <= 0 somewhere stops the run
    bad = rho.clone()
    bad[10:20, 10:20] = -50.0
    stats, _ = ctx.diffusion(bad, 0.0, d)
    assert ctx.sync(check=False) == ffb.FFB_E_NONPOSITIVE
    assert torch.equal(d, d0)
    ctx.reset_status()
    stats, _ = ctx.diffusion(rho, 4.0, d)
    assert ctx.sync(check=False) == 0 and stats_of(stats)["status"] == 0
