"""Pins of the oracle's diffusion variant (SI Appendix, section 2: the
diffusion choice f_mn(t) = exp(-(m^2/Lx^2 + n^2/Ly^2) t) and its flux
coefficients m/(pi Lx) rho~_mn f_mn, n/(pi Ly) rho~_mn f_mn).

* A single cosine mode on the cell centres has one nonzero coefficient, so
  rho(t) and J(t) on the nodes have closed forms: the mode times
  exp(-lambda t), and J = -(1/pi^2) grad rho (the diffusion constant that the
  printed f_mn implies).  A dropped normalisation, a swapped m/n, a wrong
  sign or a wrong decay rate fails these.
* At t = 0, f_mn = 1: rho(0) is the blurred density of the fast flow-based
  fields.
* In one dimension the density-equalising map is unique: x(inf) solves
  int_0^x(inf) rho_bar = int_0^x0 rho_0, which for rho_0 = rho_bar +
  A cos(pi x / L) is x0 + (A L / (pi rho_bar)) sin(pi x0 / L).  The
  integration reaches it up to the bilinear interpolation of v between the
  nodes: |v - I v| <= (1/8)(pi/L)^2 |v| for one mode, accumulated along a
  monotone path of length |x(inf) - x0|; a factor 2 covers the curvature
  that 1/rho adds.
* At t_end = 12 max(Lx, Ly)^2 every non-constant mode has decayed by at
  least exp(-12).
"""
import numpy as np
import pytest

import oracle


def _mode_density(lx, ly, modes, rho_bar=2.0):
    i = np.arange(lx) + 0.5
    j = np.arange(ly) + 0.5
    rho = np.full((ly, lx), rho_bar)
    for (m, n, A) in modes:
        rho += A * np.outer(np.cos(np.pi * n * j / ly), np.cos(np.pi * m * i / lx))
    return rho


def _closed_form(lx, ly, modes, t, rho_bar=2.0):
    x = np.arange(lx) + 0.5
    y = np.arange(ly) + 0.5
    rho = np.full((ly, lx), rho_bar)
    jx = np.zeros((ly, lx))
    jy = np.zeros((ly, lx))
    for (m, n, A) in modes:
        lam = (m / lx) ** 2 + (n / ly) ** 2
        d = A * np.exp(-lam * t)
        cx, sx = np.cos(np.pi * m * x / lx), np.sin(np.pi * m * x / lx)
        cy, sy = np.cos(np.pi * n * y / ly), np.sin(np.pi * n * y / ly)
        rho += d * np.outer(cy, cx)
        # J = -(1/pi^2) grad rho
        jx += d * (m / (np.pi * lx)) * np.outer(cy, sx)
        jy += d * (n / (np.pi * ly)) * np.outer(sy, cx)
    return rho, jx, jy


@pytest.mark.parametrize("lx,ly,modes", [
    (16, 16, [(1, 0, 0.5)]),
    (16, 16, [(0, 3, 0.4)]),
    (32, 8, [(5, 2, 0.3)]),
    (8, 32, [(2, 7, -0.2), (3, 0, 0.1), (0, 1, 0.25)]),
])
@pytest.mark.parametrize("t", [0.0, 3.0, 250.0])
def test_single_modes_closed_form(lx, ly, modes, t):
    rho0 = _mode_density(lx, ly, modes)
    coef, rb = oracle.coefficients(rho0, 0.0)
    F = oracle.diffusion_fields(coef, t)
    r, jx, jy = _closed_form(lx, ly, modes, t)
    scale = 1.0 + sum(abs(A) for *_, A in modes)
    np.testing.assert_allclose(F.rho_s, r, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(F.jx, jx, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(F.jy, jy, rtol=0, atol=1e-12 * scale)
    assert rb == pytest.approx(2.0, rel=1e-14)


def test_uniform_density_has_no_flux():
    coef, _ = oracle.coefficients(np.full((16, 32), 3.5), 0.0)
    F = oracle.diffusion_fields(coef, 7.0)
    np.testing.assert_allclose(F.rho_s, 3.5, rtol=1e-14)
    assert np.abs(F.jx).max() < 1e-13 and np.abs(F.jy).max() < 1e-13


def test_time_zero_is_the_blurred_density():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 3.0, (24, 40))
    coef, rb = oracle.coefficients(rho, 1.5)
    F = oracle.diffusion_fields(coef, 0.0)
    ffb = oracle.flux(rho, 1.5)
    np.testing.assert_allclose(F.rho_s, ffb.rho_s, rtol=1e-12)
    assert rb == pytest.approx(ffb.rho_bar, rel=1e-14)


@pytest.mark.parametrize("A", [0.3, 0.6])
def test_one_dimensional_equalisation(A):
    L, Ly, rho_bar = 64, 16, 1.0
    rho = _mode_density(L, Ly, [(1, 0, A)], rho_bar)
    coef, _ = oracle.coefficients(rho, 0.0)
    x0 = np.linspace(0.0, L, 41)
    pts = np.stack([x0, np.full_like(x0, 5.3)], 1)
    r = oracle.diffusion_integrate(coef, pts, oracle.diffusion_t_end(L, Ly))
    x_inf = x0 + A * L / (np.pi * rho_bar) * np.sin(np.pi * x0 / L)
    bound = 2.0 * (np.pi / L) ** 2 / 8.0 * np.abs(x_inf - x0).max() + 1e-4
    assert np.abs(r.xy[:, 0] - x_inf).max() <= bound
    assert np.all(r.xy[:, 1] == 5.3)           # no flux across rows: v_y = 0 exactly
    assert r.xy[0, 0] == 0.0 and r.xy[-1, 0] == L


def test_end_time_leaves_the_density_uniform():
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.5, 3.0, (16, 32))
    coef, rb = oracle.coefficients(rho, 0.0)
    te = oracle.diffusion_t_end(32, 16)
    F = oracle.diffusion_fields(coef, te)
    rest = np.abs(coef).sum() - abs(coef[0, 0])
    assert np.abs(F.rho_s - rb).max() <= np.exp(-oracle.DIFF_K) * rest / (32 * 16) + 1e-14
