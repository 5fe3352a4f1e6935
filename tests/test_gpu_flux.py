"""GPU parity: ffb_flux (Eq. 7 coefficients, blur, SI flux series on the
nodes) against the FP64 oracle on identical FP64 density grids.

The device transforms run in FP64 and round each field value to FP32 once,
so the bar is that rounding: |gpu - oracle| <= 2^-23 |oracle| (one FP32
ulp: half an ulp of rounding plus slack for the FP64 transform error,
~log2(L) 1e-16 of the field's largest magnitude, which the absolute term
1e-12 max|field| also covers).  rho_bar within 1e-12 relative (FP64 mean of
the same grid), ghosts exactly mirrored.  At L = 1024 the oracle's direct
sums are evaluated at sampled nodes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402


RTOL = 2.0 ** -23


def _close(got, ref, scale=None):
    scale = np.abs(ref).max() if scale is None else scale
    np.testing.assert_allclose(got, ref, rtol=RTOL, atol=1e-12 * scale)


def _density_grid(name):
    m = synth.workload(name)
    rho, _ = oracle.density(m, m.value, oracle.region_areas(m))
    return rho


def _check_ghosts(f):
    """Ghost border: J_x odd / J_y even across x edges, J_x even / J_y odd
    across y edges, rho_s even, w = 0."""
    lx, ly = f.shape[1] - 2, f.shape[0] - 2
    inner = f[1:-1, 1:-1]
    np.testing.assert_array_equal(f[1:-1, 0, 0], -inner[:, 0, 0])
    np.testing.assert_array_equal(f[1:-1, 0, 1:3], inner[:, 0, 1:3])
    np.testing.assert_array_equal(f[1:-1, -1, 0], -inner[:, -1, 0])
    np.testing.assert_array_equal(f[1:-1, -1, 1:3], inner[:, -1, 1:3])
    np.testing.assert_array_equal(f[0, 1:-1, 1], -inner[0, :, 1])
    np.testing.assert_array_equal(f[0, 1:-1, 0], inner[0, :, 0])
    np.testing.assert_array_equal(f[-1, 1:-1, 1], -inner[-1, :, 1])
    np.testing.assert_array_equal(f[-1, 1:-1, 2], inner[-1, :, 2])
    np.testing.assert_array_equal(f[0, 0, :2], -inner[0, 0, :2])
    np.testing.assert_array_equal(f[-1, -1, :2], -inner[-1, -1, :2])
    assert np.all(f[..., 3] == 0)


def _run(rho, sigma):
    from gpu_util import dev_f64, new_ctx, to_np
    ly, lx = rho.shape
    ctx = new_ctx(lx, ly)
    fields, rb = ctx.flux(dev_f64(rho), sigma)
    ctx.sync()
    return to_np(fields), float(rb)


@pytest.mark.parametrize("L,sigma", [(8, 0.0), (16, 1.0), (64, 4.0), (128, 2.0), (256, 4.0)])
def test_flux_parity_random(L, sigma):
    rng = np.random.default_rng(L)
    rho = rng.lognormal(0.0, 1.0, (L, L))
    print(f"[flux] random L={L} sigma={sigma}", flush=True)
    f, rb = _run(rho, sigma)
    F = oracle.flux(rho, sigma)
    assert rb == pytest.approx(rho.mean(), rel=1e-12)
    assert rb == pytest.approx(F.rho_bar, rel=1e-12)
    for c, ref in ((0, F.jx), (1, F.jy), (2, F.rho_s)):
        _close(f[1:-1, 1:-1, c], ref)
    _check_ghosts(f)


@pytest.mark.parametrize("lx,ly", [(64, 16), (16, 128), (256, 32)])
def test_flux_parity_rectangular(lx, ly):
    rng = np.random.default_rng(lx + 7 * ly)
    rho = rng.uniform(0.2, 5.0, (ly, lx))
    f, rb = _run(rho, 1.5)
    F = oracle.flux(rho, 1.5)
    for c, ref in ((0, F.jx), (1, F.jy), (2, F.rho_s)):
        _close(f[1:-1, 1:-1, c], ref)
    _check_ghosts(f)


@pytest.mark.parametrize("name,sigma", [("c1_L64", 4.0), ("c2_L512", 4.0), ("c2_L512", 0.5)])
def test_flux_parity_voronoi(name, sigma):
    rho = _density_grid(name)
    print(f"[flux] {name} sigma={sigma}", flush=True)
    f, rb = _run(rho, sigma)
    F = oracle.flux(rho, sigma)
    for c, ref in ((0, F.jx), (1, F.jy), (2, F.rho_s)):
        _close(f[1:-1, 1:-1, c], ref)
    _check_ghosts(f)


def test_flux_full_size_sampled_nodes():
    """C3 density (L = 1024, Pareto densities) at sampled nodes."""
    rho = _density_grid("c3_L1024")
    print("[flux] c3_L1024 sampled", flush=True)
    f, rb = _run(rho, 4.0)
    coef, rbo = oracle.coefficients(rho, 4.0)
    assert rb == pytest.approx(rbo, rel=1e-12)
    rng = np.random.default_rng(0)
    ii = np.concatenate([rng.integers(0, 1024, 60), [0, 1023, 0, 1023, 511]])
    jj = np.concatenate([rng.integers(0, 1024, 60), [0, 0, 1023, 1023, 512]])
    ref = oracle.flux_nodes(coef, ii, jj)
    got = f[jj + 1, ii + 1, :3]
    # the absolute term uses the samples' largest magnitude (an oracle value)
    for c in range(3):
        _close(got[:, c], ref[:, c], max(np.abs(ref[:, c]).max(), 1e-30))
    _check_ghosts(f)
    # mean of the blurred density is preserved (property at any size)
    assert f[1:-1, 1:-1, 2].astype(np.float64).mean() == pytest.approx(rbo, rel=1e-6)


def test_uniform_density_gives_zero_flux():
    rho = np.full((32, 32), 2.5)
    f, rb = _run(rho, 3.0)
    assert np.abs(f[..., :2]).max() < 1e-12
    np.testing.assert_allclose(f[..., 2], 2.5, rtol=1e-6)
    assert rb == 2.5


def test_nonpositive_blurred_density_sets_status():
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f64, new_ctx
    rho = np.ones((16, 16))
    rho[3:9, 3:9] = -10.0
    ctx = new_ctx(16)
    ctx.flux(dev_f64(rho), 0.0)
    assert ctx.sync(check=False) == ffb.api.FFB_E_NONPOSITIVE


def test_pack_fields_layout():
    from gpu_util import dev_f32, new_ctx, to_np
    rng = np.random.default_rng(5)
    jx, jy, rs = (rng.standard_normal((8, 16)).astype(np.float32) for _ in range(3))
    ctx = new_ctx(16, 8)
    f = to_np(ctx.pack_fields(dev_f32(jx), dev_f32(jy), dev_f32(rs)))
    ctx.sync()
    np.testing.assert_array_equal(f[1:-1, 1:-1, 0], jx)
    np.testing.assert_array_equal(f[1:-1, 1:-1, 1], jy)
    np.testing.assert_array_equal(f[1:-1, 1:-1, 2], rs)
    _check_ghosts(f)
