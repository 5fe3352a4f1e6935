"""Pins of the oracle's angular-distortion measures (main text, section
"Measures of distortion"; SI Appendix section 3).

* identity and similarity maps (rotation + scale + shift) are conformal:
  a = b, e = e~ = 0 everywhere;
* an affine map x -> A x + c has grad T = A on every square (the bilinear
  differences of an affine map are exact), so a, b are A's singular values,
  written out here in closed form (independent of the SVD the oracle uses);
* a one-dimensional map (x, y) -> (f(x), y) has grad T = diag(f'_h, 1) with
  f'_h the node difference of f, so e = |ln f'_h|;
* e~ = 2 arcsin(tanh(e / 2)) holds identically, since
  (a - b)/(a + b) = tanh(ln(a/b)/2);
* a folded square (det < 0) is counted.
"""
import numpy as np
import pytest

import oracle


def _nodes(lx, ly):
    x, y = np.meshgrid(np.arange(lx) + 0.5, np.arange(ly) + 0.5)
    return np.stack([x, y], -1).reshape(-1, 2)


def test_identity_and_similarity_are_conformal():
    lx, ly = 16, 8
    p = _nodes(lx, ly)
    d = oracle.distortion(p, lx, ly)
    assert d.e_inf == 0.0 and d.e_tilde_inf == 0.0 and d.folded == 0
    th, s = 0.7, 1.9
    R = s * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    d = oracle.distortion(p @ R.T + [3.0, -2.0], lx, ly)
    assert d.e_inf < 1e-12 and d.e_tilde_inf < 1e-12


def test_affine_map_closed_form():
    lx, ly = 12, 10
    A = np.array([[1.7, 0.4], [-0.3, 0.6]])
    d = oracle.distortion(_nodes(lx, ly) @ A.T + [1.0, 2.0], lx, ly)
    # singular values of [[p, q], [r, s]]: Q +- R with
    # Q = |((p + s), (r - q))| / 2, R = |((p - s), (r + q))| / 2
    p_, q_, r_, s_ = A[0, 0], A[0, 1], A[1, 0], A[1, 1]
    Q = 0.5 * np.hypot(p_ + s_, r_ - q_)
    R = 0.5 * np.hypot(p_ - s_, r_ + q_)
    a, b = Q + R, abs(Q - R)
    np.testing.assert_allclose(d.e, np.log(a / b), rtol=1e-12)
    np.testing.assert_allclose(d.e_tilde, 2 * np.arcsin((a - b) / (a + b)), rtol=1e-12)
    assert d.e_a == pytest.approx(np.log(a / b), rel=1e-12)


def test_one_dimensional_map():
    lx, ly = 32, 6
    p = _nodes(lx, ly)
    f = lambda x: x + 3.0 * np.sin(np.pi * x / lx) ** 2
    q = np.stack([f(p[:, 0]), p[:, 1]], -1)
    d = oracle.distortion(q, lx, ly)
    xs = np.arange(lx) + 0.5
    fh = f(xs[1:]) - f(xs[:-1])                       # node differences along x
    np.testing.assert_allclose(d.e, np.broadcast_to(np.abs(np.log(fh)), d.e.shape), rtol=1e-12)


def test_etilde_identity_and_folding():
    rng = np.random.default_rng(4)
    lx, ly = 20, 20
    p = _nodes(lx, ly) + 0.2 * rng.standard_normal((lx * ly, 2))
    d = oracle.distortion(p, lx, ly)
    np.testing.assert_allclose(d.e_tilde, 2 * np.arcsin(np.tanh(d.e / 2)), rtol=1e-12, atol=1e-15)
    q = _nodes(lx, ly)
    q[5 * lx + 7, 0] += 2.5                           # push one node past its neighbour
    assert oracle.distortion(q, lx, ly).folded > 0
