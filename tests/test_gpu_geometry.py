"""GPU parity: ffb_area_error and ffb_density against the FP64 oracle on
identical FP32 vertices (the seeded synthetic maps), plus edge cases.

Bars: areas and area errors within 1e-6 relative (the stated tolerance for
area errors; FP64 sums of exact FP32 products reach ~1e-12); densities
within 1e-5 of the largest cell value (FP64 accumulation, FP32 output)."""
from types import SimpleNamespace

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402

MAPS = ["c1_L64", "c4_0", "c4_1", "c2_L512"]


def _geom_and_ctx(m, xy=None):
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f32, new_ctx
    xy_d = dev_f32(m.xy if xy is None else xy)
    return ffb.Geometry.from_map(m, xy=xy_d), new_ctx(m.lx, m.ly)


@pytest.mark.parametrize("name", MAPS)
def test_area_error_parity(name):
    from gpu_util import dev_f64, to_np
    m = synth.workload(name)
    print(f"[area] {name} V={m.n_vertices} G={m.n_rings}", flush=True)
    geom, ctx = _geom_and_ctx(m)
    value = m.value * np.linspace(0.7, 1.3, m.n_regions)   # non-trivial errors
    area, err, mx = ctx.area_error(geom, dev_f64(value))
    ctx.sync()
    a_ref = oracle.region_areas(m)
    e_ref, mx_ref = oracle.area_error(value, a_ref)
    np.testing.assert_allclose(to_np(area), a_ref, rtol=1e-12)
    np.testing.assert_allclose(to_np(err), e_ref, rtol=1e-6, atol=1e-12)
    assert float(mx) == pytest.approx(mx_ref, rel=1e-10)


@pytest.mark.parametrize("name", MAPS)
def test_density_parity(name):
    from gpu_util import dev_f64, to_np
    m = synth.workload(name)
    print(f"[density] {name} L={m.lx} E={m.n_entries}", flush=True)
    geom, ctx = _geom_and_ctx(m)
    area, _, _ = ctx.area_error(geom, dev_f64(m.value))
    rho, pad = ctx.density(geom, dev_f64(m.value), area)
    ctx.sync()
    a_ref = oracle.region_areas(m)
    rho_ref, pad_ref = oracle.density(m, m.value, a_ref)
    assert float(pad) == pytest.approx(pad_ref, rel=1e-13)
    r = to_np(rho)
    # FP64 grid: edge deposits and row prefix sums against polygon clipping
    np.testing.assert_allclose(r, rho_ref, rtol=0, atol=1e-11 * np.abs(rho_ref).max())
    # mass: sum of rho equals rho_pad * L^2
    assert r.sum() == pytest.approx(pad_ref * m.lx * m.ly, rel=1e-12)


def test_density_pareto_contrast_full_size():
    """C3 map (L = 1024, 600 regions, Pareto densities up to 1e3): sampled
    rows of the density grid against the oracle's clipping raster."""
    from gpu_util import dev_f64, to_np
    m = synth.workload("c3_L1024")
    print(f"[density] c3_L1024 E={m.n_entries}", flush=True)
    geom, ctx = _geom_and_ctx(m)
    area, _, _ = ctx.area_error(geom, dev_f64(m.value))
    rho, pad = ctx.density(geom, dev_f64(m.value), area)
    ctx.sync()
    a_ref = oracle.region_areas(m)
    np.testing.assert_allclose(to_np(area), a_ref, rtol=1e-11)
    rho_ref, pad_ref = oracle.density(m, m.value, a_ref)
    r = to_np(rho)
    np.testing.assert_allclose(r, rho_ref, rtol=0, atol=1e-11 * np.abs(rho_ref).max())
    rel = np.abs(r - rho_ref) / np.abs(rho_ref)
    assert rel.max() < 1e-10


def rings_map(rings, values, L=16, regions=None):
    xy, vidx, off = [], [], [0]
    for ring in rings:
        for p in ring:
            vidx.append(len(xy))
            xy.append(p)
        off.append(len(vidx))
    reg = list(range(len(rings))) if regions is None else regions
    return SimpleNamespace(lx=L, ly=L, xy=np.array(xy, np.float32),
                           ring_offsets=np.array(off, np.int32),
                           ring_vidx=np.array(vidx, np.int32),
                           ring_region=np.array(reg, np.int32), n_regions=max(reg) + 1,
                           n_vertices=len(xy), value=np.array(values, np.float64))


def test_holes_long_edges_and_box_edges():
    """A region with a hole, edges many cells long, vertices on the box edges
    and at cell corners, a triangle: GPU density equals the oracle's."""
    from gpu_util import dev_f64, to_np
    L = 16
    outer = [(0.0, 0.0), (9.0, 0.0), (9.0, 16.0), (0.0, 16.0)]
    hole = [(2.5, 3.25), (2.5, 11.0), (6.75, 11.0), (6.75, 3.25)]          # clockwise
    tri = [(9.0, 0.0), (16.0, 0.0), (12.3, 13.7)]
    sliver = [(9.0, 16.0), (13.1, 14.05), (16.0, 16.0)]
    m = rings_map([outer, hole, tri, sliver], [50.0, 3.0, 7.0], L, regions=[0, 0, 1, 2])
    geom, ctx = _geom_and_ctx(m)
    area, _, _ = ctx.area_error(geom, dev_f64(m.value))
    rho, pad = ctx.density(geom, dev_f64(m.value), area)
    assert ctx.sync(check=False) == 0
    a_ref = oracle.region_areas(m)
    np.testing.assert_allclose(to_np(area), a_ref, rtol=1e-13)
    rho_ref, pad_ref = oracle.density(m, m.value, a_ref)
    np.testing.assert_allclose(to_np(rho), rho_ref, rtol=1e-12, atol=1e-12)


def test_device_errors_are_sticky_status():
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f64
    L = 16
    sq = [(2.0, 2.0), (6.0, 2.0), (6.0, 6.0), (2.0, 6.0)]
    out = [(2.0, 2.0), (17.0, 2.0), (6.0, 6.0)]
    # vertex outside the box -> DOMAIN
    m = rings_map([sq, out], [1.0, 2.0], L)
    geom, ctx = _geom_and_ctx(m)
    area, _, _ = ctx.area_error(geom, dev_f64(m.value))
    ctx.density(geom, dev_f64(m.value), area)
    assert ctx.sync(check=False) == ffb.api.FFB_E_DOMAIN
    ctx.reset_status()
    assert ctx.sync(check=False) == 0
    # non-positive value -> NONPOSITIVE
    m2 = rings_map([sq], [0.0], L)
    geom2, ctx2 = _geom_and_ctx(m2)
    ctx2.area_error(geom2, dev_f64(m2.value))
    assert ctx2.sync(check=False) == ffb.api.FFB_E_NONPOSITIVE
    # NaN coordinate -> NONFINITE
    xy = m2.xy.copy()
    xy[1, 0] = np.nan
    geom3, ctx3 = _geom_and_ctx(m2, xy=xy)
    ctx3.area_error(geom3, dev_f64([1.0]))
    assert ctx3.sync(check=False) == ffb.api.FFB_E_NONFINITE
    # vertex index out of range -> INVALID (no memory access beyond xy)
    m4 = rings_map([sq], [1.0], L)
    m4.ring_vidx = np.array([0, 1, 2, 9], np.int32)
    geom4, ctx4 = _geom_and_ctx(m4)
    ctx4.area_error(geom4, dev_f64(m4.value))
    assert ctx4.sync(check=False) == ffb.api.FFB_E_INVALID


def test_host_validation_rejects_before_launch():
    import paper_1802_07625_amd as ffb
    from gpu_util import dev_f64
    m = rings_map([[(2.0, 2.0), (6.0, 2.0), (6.0, 6.0)]], [1.0], 16)
    geom, ctx = _geom_and_ctx(m)
    import torch
    with pytest.raises(ValueError):          # marshalling: wrong dtype
        ctx.area_error(geom, dev_f64(m.value).to(dtype=torch.float32))
    with pytest.raises(ffb.FFBError) as ei:  # C ABI: sigma < 0
        ffb.ffb_flux(ctx.handle, dev_f64(np.ones(256)), -1.0, ctx.new_fields(), dev_f64([0.0]),
                     16, 16)
    assert ei.value.code == 1
