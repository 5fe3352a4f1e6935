"""GPU parity: ffb_integrate (v = J / rho_t, bilinear lookup, Dormand-Prince
5(4) to t = 1) against the FP64 oracle.

Identical inputs: the oracle's fields rounded to FP32 and packed through
ffb_pack_fields, the same FP32 starting points.  The oracle runs its own
adaptive controller; the GPU replays the oracle's accepted steps, so both
sides take the same steps and positions must agree within 1e-4 grid units
(the stated tolerance).  Unreplayed GPU runs are compared on outcomes (the
schedules differ once an FP32 error estimate lands on the other side of the
tolerance).  At the full C3 size the GPU integrates all 2.05 M points in the
benchmark's launch configuration and sampled points are checked against
the oracle integrating just those points with the same fixed schedule."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402

TOL_POS = 1e-4


def _oracle_fields(m, sigma):
    rho, _ = oracle.density(m, m.value, oracle.region_areas(m))
    return oracle.flux(rho, sigma)


def _gpu_integrate(ctx, fields, rb, pts, opts=None, replay=None):
    from gpu_util import dev_f32, dev_f64, stats_of, to_np
    import paper_1802_07625_amd as ffb
    xy = dev_f32(pts)
    rh = None if replay is None else dev_f64(replay)
    stats, h = ctx.integrate(fields, rb, xy, opts or ffb.IntegrateOpts(), replay_h=rh)
    code = ctx.sync(check=False)
    st = stats_of(stats)
    hh = to_np(h)[:st["accepted"]] if h is not None else None
    return to_np(xy).astype(np.float64), st, hh, code


# where the integrator keeps the point state: 0 device memory, 1 LDS with
# the first-stage velocity carried, 2 LDS with it recomputed
MODES = [0, 1, 2]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["c1_L64", "c4_0", "c2_L512"])
def test_replayed_schedule_parity(name, mode):
    from gpu_util import map_points, new_ctx, pack_oracle_fields
    m = synth.workload(name)
    pts = map_points(m)
    print(f"[integrate] {name} mode={mode} P={pts.shape[0]}", flush=True)
    ctx = new_ctx(m.lx, m.ly, pts.shape[0], mode=mode)
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    ref = oracle.integrate(Fr, pts.astype(np.float64))        # oracle's own control
    got, st, h, code = _gpu_integrate(ctx, fields, rb, pts, replay=ref.h)
    assert code == 0 and st["accepted"] == ref.accepted and st["rejected"] == 0
    np.testing.assert_array_equal(h, ref.h)
    d = np.abs(got - ref.xy).max()
    print(f"[integrate] {name} mode={mode} steps={ref.accepted} max|dx|={d:.3e}", flush=True)
    assert d < TOL_POS


@pytest.mark.parametrize("name", ["c1_L64", "c2_L512"])
def test_adaptive_run_outcome(name):
    from gpu_util import map_points, new_ctx, pack_oracle_fields
    m = synth.workload(name)
    pts = map_points(m)
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    ref = oracle.integrate(Fr, pts.astype(np.float64))
    got, st, h, code = _gpu_integrate(ctx, fields, rb, pts)
    assert code == 0
    assert abs(st["accepted"] - ref.accepted) <= 1
    assert h.sum() == pytest.approx(1.0, abs=1e-12)
    # h0 is exact; later steps follow err^(-1/5) of an error estimate that is
    # a difference of nearly equal sums (err ~ 2e-6 against terms ~ 1e-1 at
    # C2), whose FP32 rounding is ~1e-3 relative, i.e. ~2e-4 on the step
    assert h[0] == ref.h[0]
    np.testing.assert_allclose(h[1:3], ref.h[1:3], rtol=2e-3)
    # each run's local errors are <= tol per accepted step, so two runs with
    # different schedules differ by at most about steps * tol in total
    d = np.abs(got - ref.xy)
    print(f"[integrate] {name} adaptive gpu={st['accepted']}/{st['rejected']} "
          f"oracle={ref.accepted}/{ref.rejected} max|dx|={d.max():.3e} "
          f"p99={np.percentile(d, 99):.3e}", flush=True)
    assert d.max() < ref.accepted * 1e-3
    assert np.percentile(d, 99) < 1e-3


@pytest.mark.parametrize("mode", MODES)
def test_step_control_sees_every_point(mode):
    """300 k copies of one point P and, at index k, one point H in a steeper
    part of the flow.  Copies of P have the same error estimates, so the
    adaptive schedule must be that of the two-point set {P, H}, bit for bit,
    wherever H sits in the array (any lane, wavefront, workgroup or XCD
    share): the error maximum taken per wavefront, per workgroup and over
    the grid covers every point.  P alone takes another schedule, so a
    maximum that missed H would show."""
    from gpu_util import new_ctx, pack_oracle_fields
    L = 64
    rho = np.ones((L, L))
    rho[28:36, 28:36] = 4.0
    F = oracle.flux(rho, 1.0)
    P = np.array([8.3, 9.1], dtype=np.float32)
    H = np.array([27.5, 31.2], dtype=np.float32)

    def run(pts):
        ctx = new_ctx(L, L, pts.shape[0], mode=mode)
        fields, rb, _ = pack_oracle_fields(ctx, F)
        return _gpu_integrate(ctx, fields, rb, pts)

    _, sp, hp, cp = run(P[None, :])
    x2, s2, h2, c2 = run(np.stack([P, H]))
    assert cp == 0 and c2 == 0
    assert hp.shape != h2.shape or not np.array_equal(hp, h2)
    n = 300_000
    for k in (0, 63, 81, 1023, 1029, 70_000, 150_001, n - 1):
        pts = np.tile(P, (n, 1))
        pts[k] = H
        x, s, h, c = run(pts)
        assert c == 0
        assert (s["accepted"], s["rejected"]) == (s2["accepted"], s2["rejected"]), k
        np.testing.assert_array_equal(h, h2)
        np.testing.assert_array_equal(x[k], x2[1])
        np.testing.assert_array_equal(x[k - 1], x2[0])
    print(f"[integrate] mode={mode} P alone {sp['accepted']}/{sp['rejected']}, "
          f"with H {s2['accepted']}/{s2['rejected']}: reproduced with H at 8 positions "
          f"among {n} points", flush=True)


@pytest.mark.parametrize("mode", MODES)
def test_replay_equals_adaptive_bitwise(mode):
    """Rejected attempts (forced by a large first step) leave no trace: the
    adaptive run equals a replay of its accepted steps bit for bit."""
    from gpu_util import map_points, new_ctx, pack_oracle_fields
    m = synth.workload("c1_L64")
    pts = map_points(m)
    ctx = new_ctx(m.lx, m.ly, pts.shape[0], mode=mode)
    fields, rb, _ = pack_oracle_fields(ctx, _oracle_fields(m, 4.0))
    import paper_1802_07625_amd as ffb
    a, sa, ha, _ = _gpu_integrate(ctx, fields, rb, pts, ffb.IntegrateOpts(tol=1e-4, h0=0.5))
    b, sb, hb, _ = _gpu_integrate(ctx, fields, rb, pts, replay=ha)
    assert sa["rejected"] > 0 and sb["accepted"] == sa["accepted"]
    np.testing.assert_array_equal(a, b)


def test_linear_field_exact_solution():
    """Node fields linear in x and y with constant rho_s: bilinear
    interpolation is exact, so the ODE solution is known in closed form."""
    from gpu_util import dev_f32, dev_f64, new_ctx
    L, ax, ay, rs, rbar = 64, 1.2, -0.7, 2.0, 1.0
    i, j = np.meshgrid(np.arange(L) + 0.5, np.arange(L) + 0.5)
    jx, jy = ax * (i - 32), ay * (j - 32)
    ctx = new_ctx(L)
    fields = ctx.pack_fields(dev_f32(jx), dev_f32(jy), dev_f32(np.full((L, L), rs)))
    rng = np.random.default_rng(5)
    p0 = (32 + rng.uniform(-6, 6, (300, 2))).astype(np.float32)
    exact = lambda x0, a: 32 + (x0 - 32) * (rbar / rs) ** (a / (rbar - rs))
    ex = np.stack([exact(p0[:, 0].astype(np.float64), ax), exact(p0[:, 1].astype(np.float64), ay)], 1)
    import paper_1802_07625_amd as ffb
    got, st, h, code = _gpu_integrate(ctx, fields, dev_f64([rbar]), p0, ffb.IntegrateOpts(tol=1e-6))
    assert code == 0
    assert np.abs(got - ex).max() < 2e-5


def test_uniform_field_is_identity_and_edges_stay():
    """J = 0 keeps every point; with a real field, points on the box edges
    stay exactly on them (the normal velocity is exactly zero)."""
    from gpu_util import dev_f32, dev_f64, new_ctx, pack_oracle_fields
    L = 64
    ctx = new_ctx(L)
    z = np.zeros((L, L))
    fields = ctx.pack_fields(dev_f32(z), dev_f32(z), dev_f32(np.full((L, L), 1.5)))
    rng = np.random.default_rng(1)
    p = rng.uniform(0, L, (1000, 2)).astype(np.float32)
    got, st, _, code = _gpu_integrate(ctx, fields, dev_f64([1.5]), p)
    assert code == 0
    np.testing.assert_array_equal(got, p.astype(np.float64))

    m = synth.workload("c1_L64")
    fields, rb, _ = pack_oracle_fields(ctx, _oracle_fields(m, 4.0))
    s = np.linspace(0, L, 65)[:-1]
    ring = np.concatenate([np.stack([s, 0 * s], 1), np.stack([0 * s + L, s], 1),
                           np.stack([L - s, 0 * s + L], 1), np.stack([0 * s, L - s], 1)]).astype(np.float32)
    q, st, _, code = _gpu_integrate(ctx, fields, rb, ring)
    assert code == 0
    assert np.all(q[:64, 1] == 0) and np.all(q[64:128, 0] == L)
    assert np.all(q[128:192, 1] == L) and np.all(q[192:, 0] == 0)


@pytest.mark.parametrize("n", [0, 1, 255, 257, 1000])
def test_ragged_point_counts(n):
    from gpu_util import new_ctx, pack_oracle_fields
    m = synth.workload("c1_L64")
    ctx = new_ctx(64)
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    rng = np.random.default_rng(n)
    p = rng.uniform(0.0, 64.0, (n, 2)).astype(np.float32)
    # schedule from the oracle on a reference cloud, replayed on both sides
    sched = oracle.integrate(Fr, rng.uniform(0, 64, (500, 2))).h
    got, st, _, code = _gpu_integrate(ctx, fields, rb, p, replay=sched)
    assert code == 0 and st["accepted"] == len(sched)
    if n:
        ref = oracle.integrate(Fr, p.astype(np.float64), replay_h=sched)
        assert np.abs(got - ref.xy).max() < TOL_POS


def test_points_outside_box_and_errors():
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f32, dev_f64, new_ctx, pack_oracle_fields
    m = synth.workload("c1_L64")
    ctx = new_ctx(64)
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    # points outside the box: lookups clamp, like the oracle
    p = np.array([[-3.0, 10.0], [70.0, 20.5], [30.0, -1.0], [12.0, 99.0]], np.float32)
    sched = np.full(8, 1.0 / 8)
    got, st, _, code = _gpu_integrate(ctx, fields, rb, p, replay=sched)
    ref = oracle.integrate(Fr, p.astype(np.float64), replay_h=sched)
    assert code == 0 and np.abs(got - ref.xy).max() < TOL_POS
    # NaN point -> NONFINITE, positions left untouched
    pn = np.array([[10.0, 10.0], [np.nan, 5.0]], np.float32)
    got, st, _, code = _gpu_integrate(ctx, fields, rb, pn)
    assert code == ffb.api.FFB_E_NONFINITE and st["status"] == code
    assert got[0, 0] == 10.0
    ctx.reset_status()
    # step underflow and attempt cap
    q = np.array([[20.0, 30.0]], np.float32)
    _, st, _, code = _gpu_integrate(ctx, fields, rb, q, ffb.IntegrateOpts(tol=1e-30, h_min=1e-3))
    assert code == ffb.api.FFB_E_STEP_UNDERFLOW
    ctx.reset_status()
    _, st, _, code = _gpu_integrate(ctx, fields, rb, q, ffb.IntegrateOpts(max_attempts=2))
    assert code == ffb.api.FFB_E_MAX_ATTEMPTS
    ctx.reset_status()
    # a sticky status from an earlier call stops the integration untouched
    bad = np.ones((64, 64))
    bad[:8, :8] = -50
    ctx.flux(dev_f64(bad), 0.0)
    got, st, _, code = _gpu_integrate(ctx, fields, rb, q)
    assert code == ffb.api.FFB_E_NONPOSITIVE
    np.testing.assert_array_equal(got, q.astype(np.float64))


@pytest.mark.parametrize("mode", MODES)
def test_full_size_sampled_points(mode):
    """C3 (L = 1024, 1.0 M vertices + 1024^2 grid nodes) in one launch with a
    fixed schedule of 32 equal steps; 3000 sampled points against the
    oracle integrating only those points."""
    from gpu_util import map_points, new_ctx, pack_oracle_fields
    m = synth.workload("c3_L1024")
    pts = map_points(m)
    print(f"[integrate] c3_L1024 mode={mode} P={pts.shape[0]}", flush=True)
    ctx = new_ctx(m.lx, m.ly, pts.shape[0], mode=mode)
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    sched = np.full(32, 1.0 / 32)
    got, st, _, code = _gpu_integrate(ctx, fields, rb, pts, replay=sched)
    assert code == 0 and st["accepted"] == 32
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(m.n_vertices, 1500, replace=False),
                          m.n_vertices + rng.choice(m.lx * m.ly, 1500, replace=False)])
    ref = oracle.integrate(Fr, pts[idx].astype(np.float64), replay_h=sched)
    d = np.abs(got[idx] - ref.xy).max()
    print(f"[integrate] c3 sampled max|dx|={d:.3e}", flush=True)
    assert d < TOL_POS


def test_beyond_lds_capacity_falls_back_to_device_state():
    """2.8 M points at L = 1024 (more than one workgroup per CU can hold in
    LDS): the default state mode falls back to device-memory state, the
    points are still sorted by cell, and sampled points agree with the
    oracle.  The schedule is the oracle's own adaptive one for the sampled
    points, replayed on the GPU for all of them (equal steps as coarse as
    1/16 leave this flow unresolved by up to 49 cells, where rounding
    differences between FP32 and FP64 grow past the tolerance)."""
    from gpu_util import map_points, new_ctx, pack_oracle_fields
    m = synth.workload("c3_L1024")
    base = map_points(m)
    rng = np.random.default_rng(31)
    extra = rng.uniform(0.0, 1024.0, (2_800_000 - base.shape[0], 2)).astype(np.float32)
    pts = np.concatenate([base, extra])
    print(f"[integrate] beyond LDS P={pts.shape[0]}", flush=True)
    ctx = new_ctx(m.lx, m.ly, pts.shape[0])
    F = _oracle_fields(m, 4.0)
    fields, rb, Fr = pack_oracle_fields(ctx, F)
    idx = np.concatenate([rng.choice(base.shape[0], 1500, replace=False),
                          base.shape[0] + rng.choice(extra.shape[0], 1500, replace=False)])
    ref = oracle.integrate(Fr, pts[idx].astype(np.float64))
    got, st, _, code = _gpu_integrate(ctx, fields, rb, pts, replay=ref.h)
    assert code == 0 and st["accepted"] == ref.accepted
    d = np.abs(got[idx] - ref.xy).max()
    print(f"[integrate] beyond LDS sampled max|dx|={d:.3e}", flush=True)
    assert d < TOL_POS
