"""Pins of the oracle's reverse-mode gradient (oracle.adjoint_gradient and
the per-step adjoints it chains), each against the oracle's own forward by
directional derivatives, so that a dropped term, a wrong sign or a swapped
index in any adjoint fails here:

* areas: the shoelace sum is quadratic in the coordinates, so the central
  difference along a direction is exact up to rounding;
* raster: central differences of density() along random directions in
  (value, area, vertices), the clipping-based coverage being smooth while
  no vertex crosses a grid line;
* flux: linear in rho, so <flux(rho), lam> = <rho, flux_adj(lam)> exactly
  (the forward series themselves are pinned in test_oracle_flux.py);
* integration (steps replayed): central differences of integrate() along
  directions in the start points and in each field;
* the whole K-round gradient: against fd_gradient, whose truncation error
  falls as O(step^2), and the Euler relation sum_r d_r dL/dd_r = 0 of the
  scale-invariant loss, which the reverse mode meets to rounding.
"""
import numpy as np
import pytest

import oracle
import synth

SIGMAS = [oracle.default_sigma(k) for k in range(3)]


@pytest.fixture(scope="module")
def c1():
    m = synth.workload("c1_L64")
    ref = oracle.rounds(m, m.density, SIGMAS)
    return m, ref


def _value_area(m, xy=None):
    area = oracle.region_areas(m, xy)
    return m.density * area, area


def test_area_adj_matches_central_differences(c1):
    m, _ = c1
    rng = np.random.default_rng(3)
    lam = rng.standard_normal(m.n_regions)
    g = oracle.area_adj(m, lam)
    for _ in range(3):
        d = rng.standard_normal(m.xy.shape)
        eps = 1e-3
        fp = float(lam @ oracle.region_areas(m, m.xy + eps * d))
        fm = float(lam @ oracle.region_areas(m, m.xy - eps * d))
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - float(np.sum(g * d))) <= 1e-9 * max(1.0, abs(fd)), (fd, np.sum(g * d))


def test_density_adj_matches_central_differences(c1):
    """At the vertices after one round (the synthetic map's own borders
    partly run along grid lines, where the coverage has a kink: moving such
    an edge adds the cell on one side and removes the other's)."""
    m, _ = c1
    xy = oracle.rounds(m, m.density, SIGMAS[:1]).points[:m.n_vertices]
    rng = np.random.default_rng(5)
    value, area = _value_area(m, xy)
    lam = rng.standard_normal((m.ly, m.lx))
    lv, la, lxy = oracle.density_adj(m, value, area, lam, xy=xy)

    def f(v, a, x):
        rho, _ = oracle.density(m, v, a, xy=x)
        return float(np.sum(lam * rho))

    eps = 1e-6
    dv = rng.standard_normal(value.shape) * value
    fd = (f(value + eps * dv, area, xy) - f(value - eps * dv, area, xy)) / (2 * eps)
    assert abs(fd - lv @ dv) <= 1e-6 * abs(fd), (fd, lv @ dv)
    da = rng.standard_normal(area.shape) * area
    fd = (f(value, area + eps * da, xy) - f(value, area - eps * da, xy)) / (2 * eps)
    assert abs(fd - la @ da) <= 1e-6 * abs(fd), (fd, la @ da)
    for _ in range(2):
        dx = rng.standard_normal(xy.shape)
        fd = (f(value, area, xy + eps * dx) - f(value, area, xy - eps * dx)) / (2 * eps)
        an = float(np.sum(lxy * dx))
        assert abs(fd - an) <= 1e-5 * abs(fd), (fd, an)


@pytest.mark.parametrize("lx,ly,sigma", [(16, 16, 0.0), (32, 16, 2.0), (8, 32, 4.0)])
def test_flux_adj_is_the_transpose_of_flux(lx, ly, sigma):
    rng = np.random.default_rng(lx + 3 * ly)
    rho = 1.0 + rng.random((ly, lx))
    F = oracle.flux(rho, sigma)
    lrs, ljx, ljy = (rng.standard_normal((ly, lx)) for _ in range(3))
    lrb = float(rng.standard_normal())
    lam_rho = oracle.flux_adj(lrs, ljx, ljy, lrb, sigma)
    lhs = float(np.sum(F.rho_s * lrs) + np.sum(F.jx * ljx) + np.sum(F.jy * ljy)) + F.rho_bar * lrb
    rhs = float(np.sum(rho * lam_rho))
    scale = float(np.sum(np.abs(F.rho_s * lrs)) + np.sum(np.abs(F.jx * ljx)) +
                  np.sum(np.abs(F.jy * ljy)))
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)


def test_integrate_adj_matches_central_differences(c1):
    m, ref = c1
    rng = np.random.default_rng(7)
    value, area = _value_area(m)
    rho, _ = oracle.density(m, value, area)
    F = oracle.flux(rho, SIGMAS[0])
    h = ref.schedules[0]
    pts = m.xy
    lam_end = rng.standard_normal(pts.shape)
    lam0, lrs, ljx, ljy, lrb = oracle.integrate_adj(F, pts, h, lam_end)

    def f(pts_, rs=F.rho_s, jx=F.jx, jy=F.jy, rb=F.rho_bar):
        G = oracle.Fields(F.lx, F.ly, rs, jx, jy, rb, None)
        return float(np.sum(lam_end * oracle.integrate(G, pts_, replay_h=h).xy))

    eps = 1e-6
    d = rng.standard_normal(pts.shape)
    fd = (f(pts + eps * d) - f(pts - eps * d)) / (2 * eps)
    assert abs(fd - np.sum(lam0 * d)) <= 1e-6 * abs(fd), (fd, np.sum(lam0 * d))
    for name, lam_f, base in (("rho_s", lrs, F.rho_s), ("jx", ljx, F.jx), ("jy", ljy, F.jy)):
        d = rng.standard_normal(base.shape) * np.abs(base).mean()
        kw = {{"rho_s": "rs"}.get(name, name): base + eps * d}
        km = {{"rho_s": "rs"}.get(name, name): base - eps * d}
        fd = (f(pts, **kw) - f(pts, **km)) / (2 * eps)
        assert abs(fd - np.sum(lam_f * d)) <= 1e-6 * abs(fd), (name, fd, np.sum(lam_f * d))
    fd = (f(pts, rb=F.rho_bar * (1 + eps)) - f(pts, rb=F.rho_bar * (1 - eps))) / (2 * eps)
    assert abs(fd - lrb * F.rho_bar) <= 1e-6 * abs(fd), (fd, lrb * F.rho_bar)


def test_adjoint_gradient_matches_fd_to_its_truncation(c1):
    """The difference to the central differences falls as the step does
    (O(step^2) truncation): below 1e-6 of max|g| at step 1e-5."""
    m, ref = c1
    loss, g = oracle.adjoint_gradient(m, m.density, SIGMAS, ref.schedules)
    assert loss == ref.loss
    errs = []
    for step in (1e-3, 1e-4, 1e-5):
        gfd = oracle.fd_gradient(m, m.density, SIGMAS, ref.schedules, step=step)
        errs.append(np.max(np.abs(g - gfd)) / np.max(np.abs(gfd)))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 1e-6, errs


def test_adjoint_gradient_euler_relation(c1):
    m, ref = c1
    _, g = oracle.adjoint_gradient(m, m.density, SIGMAS, ref.schedules)
    assert abs(np.dot(m.density, g)) <= 1e-12 * np.sum(np.abs(m.density * g))


def test_adjoint_gradient_with_grid_points_is_unchanged(c1):
    """Grid nodes advected beside the vertices do not enter the loss."""
    m, ref = c1
    nodes = synth.grid_nodes(m.lx, m.ly).astype(np.float64)
    pts = np.concatenate([m.xy, nodes])
    r2 = oracle.rounds(m, m.density, SIGMAS, points=pts, schedules=ref.schedules)
    _, g0 = oracle.adjoint_gradient(m, m.density, SIGMAS, ref.schedules)
    loss, g1 = oracle.adjoint_gradient(m, m.density, SIGMAS, ref.schedules, points=pts)
    assert loss == r2.loss
    assert np.max(np.abs(g0 - g1)) <= 1e-12 * np.max(np.abs(g0))
