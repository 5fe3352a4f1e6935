"""Pins of the oracle's K-round area loss and its central-difference gradient
(the reference the device adjoint is checked against).

* Homogeneity: scaling every density by 2 scales value, rho, rho_bar and the
  flux exactly, so velocities, schedules and the loss are bit-identical;
  hence sum_r d_r dL/dd_r = 0 (Euler), which the differences must satisfy to
  their truncation error.
* Uniform densities: no flow and a zero loss, i.e. a minimum with zero
  gradient.
* No-flow limit: with a very wide blur only the mean survives, the flux is
  zero and the areas stay A0, so L(d) = sum_r (S/(d_r A) - 1)^2 with
  S = sum_q d_q A0_q, A = sum_q A0_q, whose gradient is written out below.
* The differences at h = 1e-4 and 1e-5 agree (O(h^2) truncation).
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


def test_loss_is_scale_invariant_bit_for_bit(c1):
    m, ref = c1
    r2 = oracle.rounds(m, 2.0 * m.density, SIGMAS)
    assert r2.loss == ref.loss
    assert all(np.array_equal(a, b) for a, b in zip(r2.schedules, ref.schedules))


def test_fd_gradient_satisfies_euler_relation(c1):
    m, ref = c1
    g = oracle.fd_gradient(m, m.density, SIGMAS, ref.schedules, step=1e-4)
    s = float(np.dot(m.density, g))
    assert abs(s) < 1e-6 * float(np.sum(np.abs(m.density * g))), s


def test_fd_gradient_step_convergence(c1):
    m, ref = c1
    g4 = oracle.fd_gradient(m, m.density, SIGMAS, ref.schedules, step=1e-4)
    g5 = oracle.fd_gradient(m, m.density, SIGMAS, ref.schedules, step=1e-5)
    assert np.max(np.abs(g4 - g5)) < 1e-5 * np.max(np.abs(g4))


def test_uniform_density_is_a_minimum():
    m = synth.workload("c1_L64")
    d = np.full(m.n_regions, 1.7)
    r = oracle.rounds(m, d, SIGMAS)
    assert r.loss < 1e-20
    g = oracle.fd_gradient(m, d, SIGMAS, r.schedules, step=1e-4)
    assert np.max(np.abs(g)) < 1e-8


def test_no_flow_limit_closed_form():
    m = synth.workload("c1_L64")
    wide = [400.0]                       # exp(-pi^2 s^2 / (2 L^2)) underflows for every mode > 0
    rng = np.random.default_rng(3)
    d = m.density * np.exp(0.1 * rng.standard_normal(m.n_regions))
    r = oracle.rounds(m, d, wide)
    a0 = oracle.region_areas(m)
    np.testing.assert_allclose(r.areas[-1], a0, rtol=0, atol=1e-9)
    A, S = a0.sum(), float(np.dot(d, a0))
    q = S / (d * A)                      # A_r / T_r
    assert r.loss == pytest.approx(float(np.sum((q - 1) ** 2)), rel=1e-9)
    # dL/dd_k = sum_r 2 (q_r - 1) dq_r/dd_k,  dq_r/dd_k = a0_k/(d_r A) - delta_rk S/(d_r^2 A)
    g_cf = 2 * (np.sum((q - 1) / (d * A)) * a0 - (q - 1) * S / (d * d * A))
    g = oracle.fd_gradient(m, d, wide, r.schedules, step=1e-5)
    np.testing.assert_allclose(g, g_cf, rtol=1e-6, atol=1e-9 * np.max(np.abs(g_cf)))
