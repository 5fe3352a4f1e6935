"""GPU: the spatial point order of ffb_integrate (FFB_OPT_POINT_ORDER).

The integrator may visit the points sorted by the cell they start in; every
trajectory is independent and the step control takes only a maximum, so
the sorted and unsorted runs must agree bit for bit (positions, step
counts, accepted steps and recorded tapes), for any point count and any
input order, including points outside the box and many points in one cell.
The sorted run is also checked against the oracle on a replayed schedule,
like the unsorted one; the full-size L = 1024 parity test of the integrator
runs the default setting, which sorts there."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402


def _fields(ctx, m):
    from gpu_util import pack_oracle_fields
    rho, _ = oracle.density(m, m.value, oracle.region_areas(m))
    return pack_oracle_fields(ctx, oracle.flux(rho, 4.0))


def _run(ctx, order, fields, rb, pts, replay=None):
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f32, dev_f64, stats_of, to_np
    ctx.set_option(ffb.OPT_POINT_ORDER, order)
    xy = dev_f32(pts)
    rh = None if replay is None else dev_f64(replay)
    stats, h = ctx.integrate(fields, rb, xy, ffb.IntegrateOpts(), replay_h=rh)
    code = ctx.sync(check=False)
    st = stats_of(stats)
    return to_np(xy), st, to_np(h)[:st["accepted"]], code


def _clouds(L, n, seed):
    """Shuffled points: uniform, a dense clump in one cell, a few outside the
    box and on its edges."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.0, L, (n, 2))
    k = n // 4
    p[:k] = rng.uniform(10.2, 10.9, (k, 2))          # many points in one cell
    if n >= 8:
        p[-4:] = [[-2.0, 5.0], [L + 3.0, 7.5], [0.0, 0.0], [L, L]]
    rng.shuffle(p)
    return p.astype(np.float32)


@pytest.mark.parametrize("state_mode", [0, 1, 2])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4099])
def test_sorted_equals_given_order_bitwise(n, state_mode):
    from gpu_util import new_ctx
    m = synth.workload("c1_L64")
    print(f"[order] n={n} state_mode={state_mode}", flush=True)
    ctx = new_ctx(64, mode=state_mode)
    fields, rb, _ = _fields(ctx, m)
    pts = _clouds(64, n, n)
    a, sa, ha, ca = _run(ctx, 0, fields, rb, pts)
    b, sb, hb, cb = _run(ctx, 2, fields, rb, pts)
    assert ca == 0 and cb == 0
    assert sa == sb and sa["accepted"] > 0
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(a, b)


def test_large_shuffled_input_sorted_equals_given_order():
    from gpu_util import map_points, new_ctx
    m = synth.workload("c2_L512")
    pts = map_points(m)
    rng = np.random.default_rng(7)
    pts = pts[rng.permutation(pts.shape[0])]
    print(f"[order] c2 shuffled P={pts.shape[0]}", flush=True)
    ctx = new_ctx(512, max_points=pts.shape[0])
    fields, rb, _ = _fields(ctx, m)
    a, sa, ha, _ = _run(ctx, 0, fields, rb, pts)
    b, sb, hb, _ = _run(ctx, 2, fields, rb, pts)
    assert sa == sb
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(a, b)


def test_sorted_replay_matches_oracle():
    from gpu_util import map_points, new_ctx
    m = synth.workload("c1_L64")
    pts = map_points(m)
    pts = pts[np.random.default_rng(3).permutation(pts.shape[0])]
    ctx = new_ctx(64)
    fields, rb, Fr = _fields(ctx, m)
    ref = oracle.integrate(Fr, pts.astype(np.float64))
    got, st, h, code = _run(ctx, 2, fields, rb, pts, replay=ref.h)
    assert code == 0 and st["accepted"] == ref.accepted and st["rejected"] == 0
    np.testing.assert_array_equal(h, ref.h)
    assert np.abs(got.astype(np.float64) - ref.xy).max() < 1e-4


def test_recorded_tape_is_the_same_in_both_orders():
    import paper_1802_07625_amd as ffb
    import torch
    from gpu_util import dev_f32, new_ctx, stats_of, to_np
    m = synth.workload("c1_L64")
    ctx = new_ctx(64)
    fields, rb, _ = _fields(ctx, m)
    pts = _clouds(64, 3000, 11)
    tape_n, cap = 1700, 256
    out = []
    for order in (0, 2):
        ctx.set_option(ffb.OPT_POINT_ORDER, order)
        xy = dev_f32(pts)
        stats = torch.empty(4, dtype=torch.int32, device="cuda")
        tape = torch.full((cap, tape_n, 4), -7.0, dtype=torch.float32, device="cuda")
        tape_h = torch.zeros(cap, dtype=torch.float64, device="cuda")
        ffb.ffb_integrate_record(ctx.handle, fields, rb, xy, ffb.IntegrateOpts(), stats, tape,
                                 tape_h, tape_n)
        assert ctx.sync(check=False) == 0
        st = stats_of(stats)
        out.append((to_np(xy), st, to_np(tape)[:st["accepted"]], to_np(tape_h)[:st["accepted"]]))
    (a, sa, ta, ha), (b, sb, tb, hb) = out
    assert sa == sb and sa["accepted"] > 0
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(ta, tb)


def test_kept_order_over_rounds_equals_given_order():
    """Mode 3 sorts on the first call and reuses that order while the same
    point array comes back (L = 1024, where mode 1 would sort): three rounds
    over one array give the bits of three rounds in the caller's order."""
    import paper_1802_07625_amd as ffb
    import torch
    from gpu_util import dev_f32, dev_f64, new_ctx, stats_of, to_np
    L, n = 1024, 70000
    ii = (np.arange(L) + 0.5) / L
    rho = 1.0 + 0.6 * np.outer(np.sin(3.1 * ii) ** 2, np.cos(2.3 * ii) ** 2)
    rng = np.random.default_rng(21)
    pts = rng.uniform(0.0, L, (n, 2)).astype(np.float32)
    out = {}
    for order in (ffb.POINT_ORDER_GIVEN, ffb.POINT_ORDER_KEEP):
        ctx = new_ctx(L, max_points=n)
        ctx.set_option(ffb.OPT_POINT_ORDER, order)
        xy = dev_f32(pts)
        rounds = []
        for sigma in (8.0, 4.0, 2.0):
            fields, rb = ctx.flux(dev_f64(rho * (1.0 + sigma / 16.0)), sigma)
            stats, h = ctx.integrate(fields, rb, xy, ffb.IntegrateOpts())
            assert ctx.sync(check=False) == 0
            st = stats_of(stats)
            rounds.append((to_np(xy).copy(), st, to_np(h)[:st["accepted"]]))
        out[order] = rounds
        ctx.close()
    for (a, sa, ha), (b, sb, hb) in zip(out[ffb.POINT_ORDER_GIVEN], out[ffb.POINT_ORDER_KEEP]):
        assert sa == sb and sa["accepted"] > 0
        np.testing.assert_array_equal(ha, hb)
        np.testing.assert_array_equal(a, b)


def test_option_values():
    import paper_1802_07625_amd as ffb
    from gpu_util import new_ctx
    ctx = new_ctx(64)
    for v in (0, 1, 2, 3):
        ctx.set_option(ffb.OPT_POINT_ORDER, v)
    for v in (-1, 4):
        with pytest.raises(ffb.api.FFBError):
            ctx.set_option(ffb.OPT_POINT_ORDER, v)


def test_diffusion_sorted_equals_given_order_bitwise():
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f32, dev_f64, new_ctx, stats_of, to_np
    m = synth.workload("c1_L64")
    rho, _ = oracle.density(m, m.value, oracle.region_areas(m))
    pts = _clouds(64, 5000, 5)
    ctx = new_ctx(64)
    out = []
    for order in (0, 2):
        ctx.set_option(ffb.OPT_POINT_ORDER, order)
        xy = dev_f32(pts)
        stats, h = ctx.diffusion(dev_f64(rho), 4.0, xy)
        assert ctx.sync(check=False) == 0
        st = stats_of(stats)
        out.append((to_np(xy), st, to_np(h)[:st["accepted"]]))
    (a, sa, ha), (b, sb, hb) = out
    assert sa == sb and sa["accepted"] > 0
    np.testing.assert_array_equal(ha, hb)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("order", [0, 2])
def test_workgroup_counts_change_no_bit(order):
    """The points are dealt to the persistent workgroups in 64-slot chunks
    per XCD; any workgroup count (capped by FFB_OPT_ADVECT_BLOCKS, including
    counts that do not divide by the 8 XCDs) must integrate every point
    exactly once and give the same bits."""
    import paper_1802_07625_amd as ffb
    from gpu_util import new_ctx
    m = synth.workload("c1_L64")
    n = 30011
    pts = _clouds(64, n, 17)
    ctx = new_ctx(64, max_points=n)
    fields, rb, _ = _fields(ctx, m)
    ref = None
    for cap in (0, 1, 3, 7, 8, 13, 29, 100):
        print(f"[order] workgroup cap={cap} order={order}", flush=True)
        ctx.set_option(ffb.OPT_ADVECT_BLOCKS, cap)
        got = _run(ctx, order, fields, rb, pts)
        assert got[3] == 0
        if ref is None:
            ref = got
            assert ref[1]["accepted"] > 0
            assert np.abs(ref[0] - pts).max() > 0.01        # the points did move
        else:
            assert got[1] == ref[1]
            np.testing.assert_array_equal(got[2], ref[2])
            np.testing.assert_array_equal(got[0], ref[0])


def test_sorted_nan_point_reports_nonfinite_and_leaves_points():
    """A NaN position sorts into the first cell (its key is clamped) and the
    integration reports a non-finite error as in the caller's order; no
    point is written back."""
    import paper_1802_07625_amd as ffb
    from gpu_util import new_ctx
    m = synth.workload("c1_L64")
    ctx = new_ctx(64)
    fields, rb, _ = _fields(ctx, m)
    pts = _clouds(64, 500, 9)
    pts[123] = [np.nan, 7.0]
    got, st, _, code = _run(ctx, 2, fields, rb, pts)
    assert code == ffb.api.FFB_E_NONFINITE and st["status"] == code
    np.testing.assert_array_equal(got[~np.isnan(pts[:, 0])], pts[~np.isnan(pts[:, 0])])
    ctx.reset_status()
