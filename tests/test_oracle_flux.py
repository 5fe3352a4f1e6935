"""Pins of the oracle's transform, blur, flux and velocity-lookup steps.

The oracle computes every sum directly.  Here it is held against library
transforms (scipy.fft's DCT/DST, a test-only use), closed forms of single
cosine modes, the Poisson/continuity and curl-free identities the flux must
satisfy (SI Appendix, section 2), and the boundary behaviour of the
interpolated velocity.
"""
import numpy as np
import pytest
import scipy.fft as sf

import oracle

PI = np.pi


def mode(lx, ly, m, n):
    i = np.arange(lx) + 0.5
    j = np.arange(ly) + 0.5
    return np.cos(PI * n * j / ly)[:, None] * np.cos(PI * m * i / lx)[None, :]


@pytest.mark.parametrize("lx,ly", [(8, 8), (12, 6), (16, 32)])
def test_dct2_matches_library(lx, ly):
    rng = np.random.default_rng(lx * 100 + ly)
    rho = rng.uniform(0.1, 3.0, (ly, lx))
    S = oracle.dct2(rho)
    # scipy's unnormalised DCT-II carries a factor 2 per axis
    ref = sf.dctn(rho, type=2) / 4.0
    np.testing.assert_allclose(S, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_single_mode_gives_single_coefficient():
    lx, ly = 16, 8
    m0, n0 = 3, 2
    S = oracle.dct2(mode(lx, ly, m0, n0))
    expect = np.zeros((ly, lx))
    expect[n0, m0] = lx * ly / 4.0
    np.testing.assert_allclose(S, expect, atol=1e-12)


def test_zero_mode_is_mean():
    """rho~_00 = rho_bar * lx * ly (SI, the constant term of the series)."""
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, (16, 24))
    F = oracle.flux(rho, 0.0, keep_coef=True)
    assert F.coef[0, 0] == pytest.approx(rho.mean() * rho.size, rel=1e-14)
    assert F.rho_bar == pytest.approx(rho.mean(), rel=1e-14)


def test_round_trip_without_blur():
    """The backward cosine series (SI) inverts Eq. 7's midpoint coefficients."""
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.5, 2.0, (16, 24))
    F = oracle.flux(rho, 0.0)
    np.testing.assert_allclose(F.rho_s, rho, atol=1e-13)


@pytest.mark.parametrize("sigma", [0.0, 0.7, 4.0])
def test_blur_scales_a_mode_and_keeps_the_mean(sigma):
    lx, ly, m0, n0 = 32, 16, 5, 3
    rho = 2.0 + 0.5 * mode(lx, ly, m0, n0)
    F = oracle.flux(rho, sigma)
    g = np.exp(-PI ** 2 * sigma ** 2 * (m0 ** 2 / lx ** 2 + n0 ** 2 / ly ** 2) / 2)
    np.testing.assert_allclose(F.rho_s, 2.0 + 0.5 * g * mode(lx, ly, m0, n0), atol=1e-13)
    assert F.rho_bar == pytest.approx(2.0, rel=1e-14)


def test_blur_is_heat_kernel_in_physical_space():
    """A blurred cosine mode equals the mode convolved with a Gaussian of
    standard deviation sigma on the mirror-extended line (a 1D check in x)."""
    lx, ly, sigma, m0 = 64, 4, 3.0, 4
    rho = 1.0 + 0.3 * mode(lx, ly, m0, 0)
    F = oracle.flux(rho, sigma)
    x = np.arange(lx) + 0.5
    s = np.linspace(-8 * sigma, 8 * sigma, 4001)
    w = np.exp(-s ** 2 / (2 * sigma ** 2))
    w /= w.sum()
    conv = 1.0 + 0.3 * (np.cos(PI * m0 * (x[:, None] + s[None, :]) / lx) * w).sum(1)
    np.testing.assert_allclose(F.rho_s[0], conv, atol=1e-10)


def poisson_flux(lx, ly, m, n, a):
    """Exact flux for rho = rho_bar + a cos(pi m x/lx) cos(pi n y/ly): J is the
    gradient of the Neumann solution phi of lap(phi) = rho - rho_bar,
    phi = -a cos cos / k^2, k^2 = pi^2 (m^2/lx^2 + n^2/ly^2), at the nodes."""
    k2 = PI ** 2 * (m ** 2 / lx ** 2 + n ** 2 / ly ** 2)
    i = np.arange(lx) + 0.5
    j = np.arange(ly) + 0.5
    X, Y = np.meshgrid(i, j)
    jx = a * (PI * m / lx) / k2 * np.sin(PI * m * X / lx) * np.cos(PI * n * Y / ly)
    jy = a * (PI * n / ly) / k2 * np.cos(PI * m * X / lx) * np.sin(PI * n * Y / ly)
    return jx, jy


@pytest.mark.parametrize("lx,ly,m,n", [(16, 16, 1, 0), (32, 16, 3, 2), (24, 40, 0, 5), (16, 16, 7, 9)])
def test_single_mode_flux_is_poisson_gradient(lx, ly, m, n):
    a = 0.4
    rho = 1.5 + a * mode(lx, ly, m, n)
    F = oracle.flux(rho, 0.0)
    jx, jy = poisson_flux(lx, ly, m, n, a)
    np.testing.assert_allclose(F.jx, jx, atol=1e-13)
    np.testing.assert_allclose(F.jy, jy, atol=1e-13)


def sine_coeffs(f, axis):
    """s_m, m = 1..L, with f = sum_m s_m sin(pi m (k+1/2)/L) along ``axis``,
    from the library DST-II (unnormalised: y_k = 2 sum f sin(pi (k+1)(2n+1)/2L))."""
    L = f.shape[axis]
    y = sf.dst(f, type=2, axis=axis)
    y = np.moveaxis(y, axis, -1) / L
    y[..., L - 1] *= 0.5
    return y          # index m-1 <-> frequency m


def eval_cos(c, L, axis_len_nodes):
    """sum_m c_m cos(pi m (k+1/2)/L) on the nodes, frequencies m = 1..L."""
    k = np.arange(axis_len_nodes) + 0.5
    m = np.arange(1, L + 1)
    M = np.cos(PI * m[:, None] * k[None, :] / L)
    return c @ M


def spectral_divergence(F):
    """div J from the node values: J_x is a sine series in x (cosine in y),
    J_y a sine series in y; d/dx sin(pi m x/L) = (pi m/L) cos(pi m x/L)."""
    ly, lx = F.jx.shape
    sx = sine_coeffs(F.jx, axis=1)                       # [ly, lx]
    dx = eval_cos(sx * (PI * np.arange(1, lx + 1) / lx), lx, lx)
    sy = sine_coeffs(F.jy, axis=0)                       # [lx, ly]
    dy = eval_cos(sy * (PI * np.arange(1, ly + 1) / ly), ly, ly).T
    return dx + dy


def test_flux_divergence_equals_density_excess():
    """Continuity with Eq. 4 (SI continuity equation, linear f_mn):
    d rho/dt = rho_bar - rho_0 = -div J, i.e. div J = rho_s - rho_bar, for a
    band-limited density whose highest modes are below the Nyquist edge."""
    lx = ly = 32
    rng = np.random.default_rng(9)
    rho = np.full((ly, lx), 2.0)
    for _ in range(12):
        m, n = rng.integers(0, 12, 2)
        rho += rng.uniform(-0.1, 0.1) * mode(lx, ly, m, n)
    F = oracle.flux(rho, 1.5)
    div = spectral_divergence(F)
    np.testing.assert_allclose(div, F.rho_s - F.rho_bar, atol=1e-12)


def test_flux_is_curl_free():
    """SI no-vortex condition dJx/dy = dJy/dx, checked on the coefficients:
    the x-sine/y-cosine coefficients of J_x times (pi n/ly) equal the
    x-cosine/y-sine coefficients of J_y times (pi m/lx)."""
    lx, ly = 32, 16
    rng = np.random.default_rng(10)
    rho = rng.uniform(0.5, 2.0, (ly, lx))
    F = oracle.flux(rho, 2.0)
    # exact discrete coefficients (type-II transforms of node values)
    cx = sf.dct(sf.dst(F.jx, type=2, axis=1), type=2, axis=0)      # [n, m-1]
    cy = sf.dst(sf.dct(F.jy, type=2, axis=1), type=2, axis=0)      # [n-1, m]
    m = np.arange(1, lx)
    n = np.arange(1, ly)
    lhs = cx[1:, :lx - 1] * (PI * n[:, None] / ly)
    rhs = cy[:ly - 1, 1:] * (PI * m[None, :] / lx)
    np.testing.assert_allclose(lhs, rhs, atol=1e-10 * np.abs(lhs).max())


def test_flux_symmetries():
    """Mirroring the density in x flips J_x and keeps J_y; transposing a
    square density swaps J_x and J_y."""
    rng = np.random.default_rng(12)
    rho = rng.uniform(0.5, 2.0, (16, 16))
    F = oracle.flux(rho, 1.0)
    Fm = oracle.flux(rho[:, ::-1], 1.0)
    np.testing.assert_allclose(Fm.jx, -F.jx[:, ::-1], atol=1e-13)
    np.testing.assert_allclose(Fm.jy, F.jy[:, ::-1], atol=1e-13)
    Ft = oracle.flux(rho.T, 1.0)
    np.testing.assert_allclose(Ft.jx, F.jy.T, atol=1e-13)
    np.testing.assert_allclose(Ft.jy, F.jx.T, atol=1e-13)


def test_uniform_density_has_zero_flux():
    F = oracle.flux(np.full((16, 16), 3.0), 2.0)
    assert np.abs(F.jx).max() < 1e-14 and np.abs(F.jy).max() < 1e-14
    np.testing.assert_allclose(F.rho_s, 3.0, atol=1e-14)


def test_nonpositive_blurred_density_is_an_error():
    rho = np.full((16, 16), 1.0)
    rho[4:8, 4:8] = -5.0
    with pytest.raises(oracle.OracleError) as ei:
        oracle.flux(rho, 0.0)
    assert ei.value.code == oracle.E_NONPOSITIVE


# ---------------------------------------------------------------- velocity
def fields_random(lx=16, ly=12, seed=0):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, (ly, lx))
    return oracle.flux(rho, 1.0)


def test_velocity_at_nodes_and_time_limits():
    F = fields_random()
    i, j = np.meshgrid(np.arange(F.lx) + 0.5, np.arange(F.ly) + 0.5)
    q = np.stack([i.ravel(), j.ravel()], 1)
    v0 = oracle.velocity(F, 0.0, q)
    v1 = oracle.velocity(F, 1.0, q)
    vh = oracle.velocity(F, 0.25, q)
    np.testing.assert_allclose(v0[:, 0], (F.jx / F.rho_s).ravel(), rtol=1e-15)
    np.testing.assert_allclose(v0[:, 1], (F.jy / F.rho_s).ravel(), rtol=1e-15)
    np.testing.assert_allclose(v1[:, 0], (F.jx / F.rho_bar).ravel(), rtol=1e-15)
    rt = 0.75 * F.rho_s + 0.25 * F.rho_bar          # Eq. 4
    np.testing.assert_allclose(vh[:, 1], (F.jy / rt).ravel(), rtol=1e-14)


def test_velocity_is_bilinear_between_nodes():
    F = fields_random(seed=1)
    t = 0.3
    # the centre of four nodes is their average; a point on a node row is the
    # linear blend of its two neighbours
    q = np.array([[3.0, 4.0], [3.25, 4.5]])
    v = oracle.velocity(F, t, q)
    nodes = lambda pts: oracle.velocity(F, t, np.array(pts, dtype=float))
    c = nodes([[2.5, 3.5], [3.5, 3.5], [2.5, 4.5], [3.5, 4.5]])
    np.testing.assert_allclose(v[0], c.mean(0), rtol=1e-14)
    e = nodes([[2.5, 4.5], [3.5, 4.5]])
    np.testing.assert_allclose(v[1], 0.25 * e[0] + 0.75 * e[1], rtol=1e-14)


def test_velocity_normal_component_vanishes_on_edges():
    F = fields_random(seed=2)
    ys = np.linspace(0, F.ly, 37)
    xs = np.linspace(0, F.lx, 41)
    for t in (0.0, 0.6, 1.0):
        left = oracle.velocity(F, t, np.stack([np.zeros_like(ys), ys], 1))
        right = oracle.velocity(F, t, np.stack([np.full_like(ys, F.lx), ys], 1))
        bottom = oracle.velocity(F, t, np.stack([xs, np.zeros_like(xs)], 1))
        top = oracle.velocity(F, t, np.stack([xs, np.full_like(xs, F.ly)], 1))
        assert np.all(left[:, 0] == 0) and np.all(right[:, 0] == 0)
        assert np.all(bottom[:, 1] == 0) and np.all(top[:, 1] == 0)


def test_velocity_lookup_clamps_to_box():
    F = fields_random(seed=3)
    q = np.array([[-1.0, 3.3], [F.lx + 2.0, 5.1], [4.2, -0.5], [7.7, F.ly + 9]])
    qc = np.clip(q, 0, [F.lx, F.ly])
    np.testing.assert_array_equal(oracle.velocity(F, 0.4, q), oracle.velocity(F, 0.4, qc))


# ------------------------------------------- series extension at the ghosts
MODES = [(1, 0, 0.21), (0, 1, -0.17), (2, 3, 0.11), (3, 1, 0.13), (1, 2, -0.09)]


def band_limited(lx, ly):
    """rho = 2 + sum a cos(pi m x/lx) cos(pi n y/ly) on the cell centres."""
    rho = np.full((ly, lx), 2.0)
    for m, n, a in MODES:
        rho += a * mode(lx, ly, m, n)
    return rho


def exact_series(lx, ly, x, y):
    """Closed-form density and flux of ``band_limited`` at any (x, y), the
    mirrored centres outside the box included: per mode, J is the gradient of
    the Neumann solution of lap(phi) = rho - rho_bar (SI Appendix, section 2:
    J_x is a sine series in x and a cosine series in y, J_y the mirror
    image).  Nothing here uses the oracle's sums or its ghost rule."""
    rho = np.full(np.broadcast(x, y).shape, 2.0)
    jx = np.zeros_like(rho)
    jy = np.zeros_like(rho)
    for m, n, a in MODES:
        k2 = PI ** 2 * (m ** 2 / lx ** 2 + n ** 2 / ly ** 2)
        cx, sx = np.cos(PI * m * x / lx), np.sin(PI * m * x / lx)
        cy, sy = np.cos(PI * n * y / ly), np.sin(PI * n * y / ly)
        rho = rho + a * cx * cy
        jx = jx + a * (PI * m / lx) / k2 * sx * cy
        jy = jy + a * (PI * n / ly) / k2 * cx * sy
    return rho, jx, jy


@pytest.mark.parametrize("lx,ly", [(16, 16), (24, 12)])
@pytest.mark.parametrize("t", [0.0, 0.35, 1.0])
def test_velocity_ghosts_are_the_series_at_mirrored_centres(lx, ly, t):
    """In the half-cell bands along the edges the lookup blends real nodes
    with ghost nodes.  The ghosts must carry what the series take at the
    mirrored cell centres x = -1/2, lx + 1/2 (and likewise in y): the normal
    component odd, the tangential component even, the density even.  The
    expected velocity is bilinear in the exact node velocities of an
    (lx + 2) x (ly + 2) lattice of centres, ghosts included."""
    F = oracle.flux(band_limited(lx, ly), 0.0)
    xc = np.arange(-1, lx + 1) + 0.5
    yc = np.arange(-1, ly + 1) + 0.5
    X, Y = np.meshgrid(xc, yc)
    r, jx, jy = exact_series(lx, ly, X, Y)
    rt = (1 - t) * r + t * F.rho_bar
    vx, vy = jx / rt, jy / rt                 # [ly + 2, lx + 2]
    rng = np.random.default_rng(lx + ly)
    bands = [
        np.stack([rng.uniform(0, 0.5, 64), rng.uniform(0, ly, 64)], 1),        # x = 0
        np.stack([rng.uniform(lx - 0.5, lx, 64), rng.uniform(0, ly, 64)], 1),  # x = lx
        np.stack([rng.uniform(0, lx, 64), rng.uniform(0, 0.5, 64)], 1),        # y = 0
        np.stack([rng.uniform(0, lx, 64), rng.uniform(ly - 0.5, ly, 64)], 1),  # y = ly
        np.array([[0.1, 0.2], [lx - 0.2, 0.3], [0.4, ly - 0.1], [lx - 0.3, ly - 0.45]]),
    ]
    q = np.concatenate(bands)
    v = oracle.velocity(F, t, q)
    u, w = q[:, 0] + 0.5, q[:, 1] + 0.5       # lattice coordinates (ghost row 0)
    i0, j0 = np.floor(u).astype(int), np.floor(w).astype(int)
    a, b = u - i0, w - j0
    for comp, grid in ((0, vx), (1, vy)):
        g00, g10 = grid[j0, i0], grid[j0, i0 + 1]
        g01, g11 = grid[j0 + 1, i0], grid[j0 + 1, i0 + 1]
        ref = (1 - b) * ((1 - a) * g00 + a * g10) + b * ((1 - a) * g01 + a * g11)
        np.testing.assert_allclose(v[:, comp], ref, rtol=0, atol=1e-12)
    # the tangential component is not trivially zero in these bands
    assert np.abs(v[:64, 1]).max() > 1e-3 and np.abs(v[128:192, 0]).max() > 1e-3


@pytest.mark.parametrize("lx,ly", [(16, 16), (24, 12)])
def test_flux_nodes_match_closed_form(lx, ly):
    """The node-by-node full double sums give the closed-form flux and
    density of a band-limited map at every node."""
    F = oracle.flux(band_limited(lx, ly), 0.0, keep_coef=True)
    jj, ii = np.meshgrid(np.arange(ly), np.arange(lx), indexing="ij")
    out = oracle.flux_nodes(F.coef, ii.ravel(), jj.ravel())
    r, jx, jy = exact_series(lx, ly, ii.ravel() + 0.5, jj.ravel() + 0.5)
    np.testing.assert_allclose(out[:, 0], jx, atol=1e-13)
    np.testing.assert_allclose(out[:, 1], jy, atol=1e-13)
    np.testing.assert_allclose(out[:, 2], r, atol=1e-13)


@pytest.mark.parametrize("lx,ly,sigma", [(16, 16, 1.3), (32, 8, 0.0), (12, 20, 2.5)])
def test_flux_nodes_equal_separable_sums(lx, ly, sigma):
    """The full double sums at chosen nodes agree with the separable sums of
    the whole-grid flux on a random (not band-limited) density."""
    rng = np.random.default_rng(lx * ly)
    rho = rng.uniform(0.3, 3.0, (ly, lx))
    F = oracle.flux(rho, sigma, keep_coef=True)
    jj, ii = np.meshgrid(np.arange(ly), np.arange(lx), indexing="ij")
    out = oracle.flux_nodes(F.coef, ii.ravel(), jj.ravel())
    scale = max(np.abs(F.jx).max(), np.abs(F.jy).max())
    np.testing.assert_allclose(out[:, 0], F.jx.ravel(), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(out[:, 1], F.jy.ravel(), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(out[:, 2], F.rho_s.ravel(), rtol=0, atol=1e-12 * rho.max())
