"""GPU parity of whole FFB iterations: every step on the device (areas,
density, flux, advection, areas) against the oracle doing every step in FP64
from the same FP32 input map.

Here the two sides compute their own density grids and fields: the GPU's
density grid and transforms are FP64 and its fields are the FP64 values
rounded once to FP32 (see test_gpu_flux), so the velocities differ from the
oracle's by that rounding and the integration's FP32 arithmetic.  With the
oracle's step schedule replayed, positions (vertices and grid nodes) agree
within the stated 1e-4 grid units.  The stated 1e-6
relative tolerance for areas applies to the area kernel on identical
vertices (test_gpu_geometry, met at 1e-12); after a round the vertices
differ by up to the position difference dx, which moves a region's area by
at most dx times its L1 perimeter, and that derived bound is what the round
is held to.  Full loops are compared on outcomes: both converge below 1 % in
the same number of rounds (+-1)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402


def _setup(name):
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f64, map_points, new_ctx
    import torch
    m = synth.workload(name)
    pts = map_points(m)
    d = torch.as_tensor(pts, device="cuda")
    geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    return m, pts, d, geom, ctx, dev_f64(m.value)


@pytest.mark.parametrize("name", ["c1_L64", "c2_L512"])
def test_one_iteration_replayed(name):
    import paper_1802_07625_amd as ffb
    from gpu_util import area_bound, dev_f64, stats_of, to_np
    m, pts, d, geom, ctx, value = _setup(name)
    print(f"[round] {name} P={pts.shape[0]}", flush=True)
    ref = oracle.iterate(m, m.value, pts.astype(np.float64), m.n_vertices, 4.0)
    area0, _, _ = ctx.area_error(geom, value)
    rho, pad = ctx.density(geom, value, area0)
    fields, rb = ctx.flux(rho, 4.0)
    stats, _ = ctx.integrate(fields, rb, d, ffb.IntegrateOpts(), replay_h=dev_f64(ref.h))
    area1, err1, mx1 = ctx.area_error(geom, value)
    assert ctx.sync(check=False) == 0
    s = stats_of(stats)
    assert s["accepted"] == ref.accepted
    np.testing.assert_allclose(to_np(area0), ref.area_before, rtol=1e-12)
    np.testing.assert_allclose(to_np(rho), ref.rho, rtol=0, atol=1e-11 * np.abs(ref.rho).max())
    assert float(rb) == pytest.approx(ref.fields.rho_bar, rel=1e-6)
    dx = np.abs(to_np(d).astype(np.float64) - ref.points).max()
    de = np.abs(to_np(err1) - ref.err_after).max()
    da = np.abs(to_np(area1) / ref.area_after - 1).max()
    print(f"[round] {name} steps={ref.accepted} max|dx|={dx:.3e} max|d err|={de:.3e} "
          f"max rel d area={da:.3e}", flush=True)
    assert dx < 1e-4
    bound = area_bound(m, ref.points[:m.n_vertices], dx) + 1e-12 * np.abs(ref.area_after)
    assert np.all(np.abs(to_np(area1) - ref.area_after) <= bound)


def test_loop_converges_like_the_oracle():
    import paper_1802_07625_amd as ffb
    m, pts, d, geom, ctx, value = _setup("c1_L64")
    # oracle loop
    p = pts.astype(np.float64)
    ref_rounds = None
    for k in range(20):
        r = oracle.iterate(m, m.value, p, m.n_vertices, oracle.default_sigma(k))
        p = r.points
        if r.max_err_after < 0.01:
            ref_rounds = k + 1
            break
    assert ref_rounds is not None
    # device loop: one host read per round
    area = None
    rounds, mx = None, None
    for k in range(20):
        res = ffb.iterate(ctx, geom, value, d, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        mx = float(res.max_err_after)
        if mx < 0.01:
            rounds = k + 1
            break
    assert ctx.sync(check=False) == 0
    print(f"[loop] c1 rounds gpu={rounds} oracle={ref_rounds} final={mx:.4f}", flush=True)
    assert rounds is not None and abs(rounds - ref_rounds) <= 1
    assert mx < 0.01


def test_c3_round_end_to_end():
    """The headline configuration (L = 1024, 600 regions, 1.0 M vertices +
    1024^2 grid nodes): both sides run a whole round on their own from the
    same FP32 map -- areas, density, flux, integration, areas -- so the
    GPU's field rounding travels through the full C3 flow.  The oracle
    integrates all 2.05 M points with its own adaptive controller; the GPU
    replays the oracle's accepted steps, and every point is compared."""
    import paper_1802_07625_amd as ffb
    from gpu_util import area_bound, dev_f64, stats_of, to_np
    m, pts, d, geom, ctx, value = _setup("c3_L1024")
    V = m.n_vertices
    print(f"[round] c3_L1024 P={pts.shape[0]} (oracle round)", flush=True)
    ref = oracle.iterate(m, m.value, pts.astype(np.float64), V, 4.0)
    print(f"[round] c3 oracle: {ref.accepted} accepted, {ref.rejected} rejected", flush=True)
    area0, _, _ = ctx.area_error(geom, value)
    rho, pad = ctx.density(geom, value, area0)
    fields, rb = ctx.flux(rho, 4.0)
    stats, _ = ctx.integrate(fields, rb, d, ffb.IntegrateOpts(), replay_h=dev_f64(ref.h))
    area1, err1, mx1 = ctx.area_error(geom, value)
    assert ctx.sync(check=False) == 0
    assert stats_of(stats)["accepted"] == ref.accepted
    np.testing.assert_allclose(to_np(area0), ref.area_before, rtol=1e-12)
    np.testing.assert_allclose(to_np(rho), ref.rho, rtol=0, atol=1e-11 * np.abs(ref.rho).max())
    got = to_np(d).astype(np.float64)
    dxv = np.abs(got[:V] - ref.points[:V]).max()
    dxn = np.abs(got[V:] - ref.points[V:]).max()
    da = np.abs(to_np(area1) / ref.area_after - 1).max()
    print(f"[round] c3 steps={ref.accepted} max|dx| vertices={dxv:.3e} nodes={dxn:.3e} "
          f"max rel d area={da:.3e} max err gpu={float(mx1):.6f} oracle={ref.max_err_after:.6f}",
          flush=True)
    assert max(dxv, dxn) < 1e-4
    bound = area_bound(m, ref.points[:V], dxv) + 1e-12 * np.abs(ref.area_after)
    assert np.all(np.abs(to_np(area1) - ref.area_after) <= bound)


def _oracle_loop(m, pts, max_rounds):
    p = pts.astype(np.float64)
    errs, steps = [], []
    for k in range(max_rounds):
        r = oracle.iterate(m, m.value, p, m.n_vertices, oracle.default_sigma(k))
        p = r.points
        errs.append(r.max_err_after)
        steps.append(r.accepted)
        if r.max_err_after < 0.01:
            break
    return errs, steps


def _gpu_loop(m, pts, max_rounds):
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f64, stats_of
    import torch
    d = torch.as_tensor(pts, device="cuda")
    geom = ffb.Geometry.from_map(m, xy=d[:m.n_vertices])
    ctx = ffb.Context(m.lx, m.ly, max_points=pts.shape[0])
    ctx.set_option(ffb.OPT_POINT_ORDER, ffb.POINT_ORDER_KEEP)
    value = dev_f64(m.value)
    area, errs, steps = None, [], []
    for k in range(max_rounds):
        res = ffb.iterate(ctx, geom, value, d, ffb.default_sigma(k), area_before=area)
        area = res.area_after
        errs.append(float(res.max_err_after))
        steps.append(stats_of(res.stats)["accepted"])
        if errs[-1] < 0.01:
            break
    assert ctx.sync(check=False) == 0
    ctx.close()
    return errs, steps


@pytest.mark.parametrize("name", ["c2_L512", "c3_L1024"])
def test_loop_outcome_like_the_oracle(name):
    """The loop to < 1 % on the configurations that ask for it, vertices and
    grid nodes advected, each side with its own adaptive schedules: both
    stop below 1 % within one round of each other, and every round's
    maximum error agrees to the level that schedules differing by O(tol)
    allow.  The accepted-step counts agree within 2 % (at least 2): the
    controller's accept/reject decisions near err = tol flip with last-bit
    rounding (C3's first round takes ~250 accepted and ~20-25 rejected
    attempts), so the counts are an outcome, not a bitwise property."""
    from gpu_util import map_points
    m = synth.workload(name)
    pts = map_points(m)
    print(f"[loop] {name} P={pts.shape[0]}", flush=True)
    ge, gs = _gpu_loop(m, pts, 30)
    print(f"[loop] {name} gpu rounds={len(ge)} steps={gs} errors={np.round(ge, 5).tolist()}",
          flush=True)
    oe, os_ = _oracle_loop(m, pts, 30)
    print(f"[loop] {name} oracle rounds={len(oe)} steps={os_} errors={np.round(oe, 5).tolist()}",
          flush=True)
    assert ge[-1] < 0.01 and oe[-1] < 0.01
    assert abs(len(ge) - len(oe)) <= 1
    n = min(len(ge), len(oe))
    np.testing.assert_allclose(ge[:n], oe[:n], rtol=0.05)
    assert all(abs(a - b) <= max(2, 0.02 * b) for a, b in zip(gs[:n], os_[:n]))


@pytest.mark.parametrize("name", ["c4_3", "c4_6", "c4_5"])
def test_slowly_converging_maps_stall_in_the_oracle_too(name):
    """Batch maps whose smallest regions cover a few grid cells are still
    above 1 % after 30 rounds.  The FP64 oracle's loop ends in the same
    state (not converged, the same final error), so the stall belongs to
    the method at that grid size, not to the FP32 arithmetic."""
    m = synth.workload(name)
    pts = m.xy.astype(np.float32)
    ge, _ = _gpu_loop(m, pts, 30)
    oe, _ = _oracle_loop(m, pts, 30)
    print(f"[stall] {name} L={m.lx} R={m.n_regions} gpu rounds={len(ge)} final={ge[-1]:.5f} "
          f"oracle rounds={len(oe)} final={oe[-1]:.5f}", flush=True)
    assert len(ge) == len(oe) == 30
    assert ge[-1] >= 0.01 and oe[-1] >= 0.01
    np.testing.assert_allclose(ge, oe, rtol=0.02)
