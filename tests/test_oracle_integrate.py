"""Pins of the oracle's time integration and of whole rounds.

* The Dormand-Prince 5(4) coefficients are held against the Butcher order
  conditions (a mistyped coefficient breaks one of them).
* The integrator is held against the exact solution of a linear velocity
  field (exactly representable by bilinear interpolation): fixed-step
  replays converge at order 5, adaptive runs land within the tolerance.
* A density that varies only in x has the closed-form map
  X(x) = (1/rho_bar) * integral_0^x rho_0 (flux conservation along a 1D
  flow); the oracle's round converges to it at first order in 1/L.
* Uniform density gives the identity map; the box edges map onto
  themselves (total area is conserved); replaying a recorded schedule
  reproduces the adaptive run bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth

PI = np.pi


# ------------------------------------------------------------------ tableau
def test_dormand_prince_order_conditions():
    c, a, b, bs = oracle.tableau()
    A = np.zeros((7, 7))
    A[:, :6] = a
    # row sums give the nodes
    np.testing.assert_allclose(A.sum(1), c, atol=1e-15)
    # FSAL: the last stage row is the order-5 weight vector, evaluated at t+h
    np.testing.assert_allclose(A[6], b, atol=1e-16)
    assert c[6] == 1.0

    def conds(w, order):
        out = []
        Ac = A @ c
        Ac2 = A @ c ** 2
        AAc = A @ Ac
        if order >= 1:
            out.append((w.sum(), 1.0))
        if order >= 2:
            out.append((w @ c, 1 / 2))
        if order >= 3:
            out += [(w @ c ** 2, 1 / 3), (w @ Ac, 1 / 6)]
        if order >= 4:
            out += [(w @ c ** 3, 1 / 4), (w @ (c * Ac), 1 / 8), (w @ Ac2, 1 / 12),
                    (w @ AAc, 1 / 24)]
        if order >= 5:
            out += [(w @ c ** 4, 1 / 5), (w @ (c ** 2 * Ac), 1 / 10),
                    (w @ (Ac * Ac), 1 / 20), (w @ (c * Ac2), 1 / 15),
                    (w @ (c * AAc), 1 / 30), (w @ (A @ c ** 3), 1 / 20),
                    (w @ (A @ (c * Ac)), 1 / 40), (w @ (A @ Ac2), 1 / 60),
                    (w @ (A @ AAc), 1 / 120)]
        return out

    for got, want in conds(b, 5):
        assert got == pytest.approx(want, abs=1e-14)
    for got, want in conds(bs, 4):
        assert got == pytest.approx(want, abs=1e-14)
    # the embedded pair is genuinely of order 4: some order-5 condition fails
    assert any(abs(g - w) > 1e-6 for g, w in conds(bs, 5)[8:])


# ------------------------------------------------------- linear velocity
def linear_fields(L=64, ax=1.2, ay=-0.7, rho_s=2.0, rho_bar=1.0):
    i, j = np.meshgrid(np.arange(L) + 0.5, np.arange(L) + 0.5)
    c = L / 2
    return oracle.Fields(L, L, np.full((L, L), rho_s), ax * (i - c), ay * (j - c), rho_bar)


def linear_exact(x0, a, c, rho_s, rho_bar):
    """dx/dt = a (x - c) / ((1-t) rho_s + t rho_bar) integrated to t = 1."""
    return c + (x0 - c) * (rho_bar / rho_s) ** (a / (rho_bar - rho_s))


def linear_case():
    L, ax, ay = 64, 1.2, -0.7
    F = linear_fields(L, ax, ay)
    rng = np.random.default_rng(5)
    p0 = 32 + rng.uniform(-6, 6, (50, 2))
    ex = np.stack([linear_exact(p0[:, 0], ax, 32, 2.0, 1.0),
                   linear_exact(p0[:, 1], ay, 32, 2.0, 1.0)], 1)
    assert np.all((ex > 4) & (ex < L - 4))
    return F, p0, ex


def test_fixed_step_convergence_is_order_five():
    F, p0, ex = linear_case()
    errs = []
    for N in (4, 8, 16):
        r = oracle.integrate(F, p0, replay_h=np.full(N, 1.0 / N))
        assert r.accepted == N
        errs.append(np.abs(r.xy - ex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 4.5) and np.all(rates < 6.0), (errs, rates)


@pytest.mark.parametrize("tol", [1e-4, 1e-7])
def test_adaptive_run_meets_tolerance(tol):
    F, p0, ex = linear_case()
    r = oracle.integrate(F, p0, oracle.IntegrateOpts(tol=tol))
    assert np.abs(r.xy - ex).max() < 10 * tol
    assert r.h.sum() == pytest.approx(1.0, abs=1e-15)


def test_replay_reproduces_adaptive_run_exactly():
    m = synth.workload("c1_L64")
    area = oracle.region_areas(m)
    rho, _ = oracle.density(m, m.value, area)
    F = oracle.flux(rho, 4.0)
    pts = np.concatenate([m.xy, synth.grid_nodes(64, 64)]).astype(np.float64)
    r1 = oracle.integrate(F, pts, oracle.IntegrateOpts(tol=1e-4))
    r2 = oracle.integrate(F, pts, replay_h=r1.h)
    assert r1.rejected >= 0 and r1.accepted == r2.accepted
    np.testing.assert_array_equal(r1.xy, r2.xy)


def test_step_underflow_and_attempt_cap():
    F, p0, _ = linear_case()
    with pytest.raises(oracle.OracleError) as ei:
        oracle.integrate(F, p0, oracle.IntegrateOpts(tol=1e-30, h_min=1e-3))
    assert ei.value.code == oracle.E_STEP_UNDERFLOW
    with pytest.raises(oracle.OracleError) as ei:
        oracle.integrate(F, p0, oracle.IntegrateOpts(max_attempts=2))
    assert ei.value.code == oracle.E_MAX_ATTEMPTS


# ------------------------------------------------------- whole rounds
def strip_map(L, profile):
    """A map whose regions are full-height vertical strips one cell wide
    (cell-aligned, so the raster is exact) with densities ``profile``."""
    from types import SimpleNamespace
    xy, vidx, off = [], [], [0]
    for i in range(L):
        base = len(xy)
        xy += [(i, 0.0), (i + 1.0, 0.0), (i + 1.0, float(L)), (i, float(L))]
        vidx += [base, base + 1, base + 2, base + 3]
        off.append(len(vidx))
    return SimpleNamespace(lx=L, ly=L, xy=np.array(xy), ring_offsets=np.array(off, np.int32),
                           ring_vidx=np.array(vidx, np.int32),
                           ring_region=np.arange(L, dtype=np.int32), n_regions=L,
                           value=np.asarray(profile, dtype=np.float64) * L)


def one_d_error(L):
    x = np.arange(L) + 0.5
    prof = 1.0 + 0.6 * np.cos(PI * x / L)         # cell averages differ from
    m = strip_map(L, prof)                         # point values by O(1/L^2)
    rho, pad = oracle.density(m, m.value, oracle.region_areas(m))
    F = oracle.flux(rho, 0.0)
    xs = np.linspace(0.0, L, 4 * L + 1)
    pts = np.stack([xs, np.full_like(xs, L / 2 + 0.25)], 1)
    r = oracle.integrate(F, pts, oracle.IntegrateOpts(tol=1e-10))
    # closed form: rho_bar * X = G(x0) = integral_0^x0 rho_0, with the cell
    # averages of rho_0 integrated exactly (piecewise constant in x)
    edges = np.concatenate([[0.0], np.cumsum(rho[0])])
    G = np.interp(xs, np.arange(L + 1.0), edges)
    X = G / F.rho_bar
    assert np.abs(r.xy[:, 1] - pts[:, 1]).max() < 1e-12        # no y motion
    return np.abs(r.xy[:, 0] - X).max()


def test_one_dimensional_closed_form():
    e32, e64 = one_d_error(32), one_d_error(64)
    assert e64 < 0.01
    assert 1.6 < e32 / e64 < 2.5          # first order in 1/L (grid units)


def test_uniform_density_is_identity():
    m = synth.workload("c1_L64")
    value = 1.7 * oracle.region_areas(m)       # every region at one density
    pts = np.concatenate([m.xy, synth.grid_nodes(64, 64)]).astype(np.float64)
    r = oracle.iterate(m, value, pts, m.n_vertices, 4.0)
    assert np.abs(r.fields.jx).max() < 1e-12 and np.abs(r.fields.jy).max() < 1e-12
    assert np.abs(r.points - pts).max() < 1e-10
    assert r.max_err_after < 1e-12


def test_box_maps_onto_itself():
    """Points on the box edges stay on them, and corners stay fixed, so the
    advected box boundary still encloses area L^2 (total area conserved)."""
    m = synth.workload("c1_L64")
    L = 64
    area = oracle.region_areas(m)
    rho, _ = oracle.density(m, m.value, area)
    F = oracle.flux(rho, 4.0)
    s = np.linspace(0, L, 65)[:-1]
    ring = np.concatenate([np.stack([s, 0 * s], 1), np.stack([0 * s + L, s], 1),
                           np.stack([L - s, 0 * s + L], 1), np.stack([0 * s, L - s], 1)])
    r = oracle.integrate(F, ring)
    q = r.xy
    assert np.all(q[:64, 1] == 0) and np.all(q[64:128, 0] == L)
    assert np.all(q[128:192, 1] == L) and np.all(q[192:, 0] == 0)
    x, y = q[:, 0], q[:, 1]
    shoelace = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
    assert shoelace == pytest.approx(L * L, rel=1e-13)
    assert np.all(np.diff(q[:64, 0]) > 0)                       # order kept


def test_c1_round_shrinks_errors_and_keeps_the_grid_unfolded():
    m = synth.workload("c1_L64")
    L = 64
    pts = np.concatenate([m.xy, synth.grid_nodes(L, L)]).astype(np.float64)
    e0, mx0 = oracle.area_error(m.value, oracle.region_areas(m))
    r = oracle.iterate(m, m.value, pts, m.n_vertices, oracle.default_sigma(0))
    assert r.max_err_after < 0.8 * mx0
    g = r.points[m.n_vertices:].reshape(L, L, 2)
    # signed area of every advected grid quadrilateral stays positive
    a, b = g[:-1, :-1], g[:-1, 1:]
    c, d = g[1:, 1:], g[1:, :-1]
    cross = lambda p, q: p[..., 0] * q[..., 1] - p[..., 1] * q[..., 0]
    quad = 0.5 * (cross(a, b) + cross(b, c) + cross(c, d) + cross(d, a))
    assert quad.min() > 0
    # sum of region areas changes only by blur leakage across the map edge
    assert abs(r.area_after.sum() / r.area_before.sum() - 1) < 0.05


def test_c1_loop_converges_below_one_percent():
    m = synth.workload("c1_L64")
    L = 64
    pts = np.concatenate([m.xy, synth.grid_nodes(L, L)]).astype(np.float64)
    for k in range(20):
        r = oracle.iterate(m, m.value, pts, m.n_vertices, oracle.default_sigma(k))
        pts = r.points
        if r.max_err_after < 0.01:
            break
    assert r.max_err_after < 0.01, (k, r.max_err_after)


def test_nonfinite_points_are_an_error():
    F, p0, _ = linear_case()
    p = p0.copy()
    p[3, 1] = np.nan
    with pytest.raises(oracle.OracleError) as ei:
        oracle.integrate(F, p)
    assert ei.value.code == oracle.E_NONFINITE
