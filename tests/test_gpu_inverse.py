"""Inverse of the piecewise-linear T on the device against the oracle
(Conclusion: the graticule of the inverse transformation).

Both sides decide containment with the same plain-FP64 orientation signs
on the same FP32 inputs and take the lowest-numbered containing triangle,
so the triangle index is compared exactly; the preimages are the same FP64
barycentric sums (1e-12 absolute).  At L = 1024 a sample of queries is
checked against the oracle's brute force, and every query by the round trip
through the forward piecewise-linear map.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1802_07625_amd as ffb
import synth
from gpu_util import new_ctx, to_np
from test_oracle_inverse import _forward_pl

pytestmark = pytest.mark.gpu


def _gpu(nodes, lx, ly, q):
    ctx = new_ctx(8, 8)
    print(f"[inverse] lx={lx} ly={ly} queries={len(q)}", flush=True)
    tri, pre = ctx.inverse(torch.as_tensor(np.asarray(nodes, np.float32), device="cuda"),
                           torch.as_tensor(np.asarray(q, np.float32), device="cuda"), lx, ly)
    assert ctx.sync(check=False) == 0
    out = to_np(tri), to_np(pre)
    ctx.close()
    return out


def _compare(nodes, lx, ly, q, tag):
    t_ref, p_ref = oracle.inverse(nodes, lx, ly, q)
    t, p = _gpu(nodes, lx, ly, q)
    print(f"[inverse] {tag}: found {np.sum(t >= 0)}/{len(t)}", flush=True)
    np.testing.assert_array_equal(t, t_ref)
    np.testing.assert_allclose(p, p_ref, rtol=0, atol=1e-12)
    return t, p


def _random_queries(lx, ly, n, seed, margin=1.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-margin, [lx + margin, ly + margin], (n, 2)).astype(np.float32)


@pytest.mark.parametrize("lx,ly,seed,amp", [(64, 64, 1, 0.3), (96, 40, 2, 0.4), (33, 65, 3, 0.2)])
def test_warped_maps(lx, ly, seed, amp):
    nodes = synth.warped_nodes(lx, ly, seed, amp=amp)
    _compare(nodes, lx, ly, _random_queries(lx, ly, 5000, seed), f"warp {lx}x{ly}")


def test_cartogram_after_oracle_rounds_graticule():
    m = synth.workload("c1_L64")
    L = m.lx
    pts = np.concatenate([m.xy, synth.grid_nodes(L, L)])
    rr = oracle.rounds(m, m.density, [oracle.default_sigma(k) for k in range(3)], points=pts)
    nodes = rr.points[m.n_vertices:].astype(np.float32)
    s = np.arange(0.0, L + 1e-9, 0.25)
    q = np.stack(np.meshgrid(s, s, indexing="xy"), -1).reshape(-1, 2).astype(np.float32)
    t, p = _compare(nodes, L, L, q, "c1 after 3 rounds, graticule")
    ok = t >= 0
    back = _forward_pl(nodes, L, L, p[ok])
    np.testing.assert_allclose(back, q[ok].astype(np.float64), rtol=0, atol=1e-9)


def test_folded_map_takes_lowest_triangle():
    nodes = synth.warped_nodes(128, 128, 4, amp=2.5)
    assert oracle.distortion(nodes.astype(np.float64), 128, 128).folded > 0
    _compare(nodes, 128, 128, _random_queries(128, 128, 20000, 5), "folded")


def test_edge_inputs():
    L = 16
    nodes = synth.grid_nodes(L, L)
    q = np.array([[np.nan, 3.0], [np.inf, 2.0], [-1e30, 5.0], [0.5, 0.5], [15.5, 15.5],
                  [8.0, 8.0], [0.49, 3.0]], np.float32)
    t, p = _compare(nodes, L, L, q, "edge inputs")
    assert list(t[:3]) == [-1, -1, -1] and t[-1] == -1
    np.testing.assert_allclose(p[3:6], q[3:6].astype(np.float64), atol=1e-12)
    # no queries; then a smaller call after a larger one on the same context
    ctx = new_ctx(8, 8)
    dn = torch.as_tensor(nodes, device="cuda")
    tri, pre = ctx.inverse(dn, torch.empty((0, 2), dtype=torch.float32, device="cuda"), L, L)
    assert tri.numel() == 0
    big = _random_queries(L, L, 3000, 7)
    t1, p1 = ctx.inverse(dn, torch.as_tensor(big, device="cuda"), L, L)
    t2, p2 = ctx.inverse(dn, torch.as_tensor(big[:77], device="cuda"), L, L)
    assert ctx.sync(check=False) == 0
    np.testing.assert_array_equal(to_np(t2), to_np(t1)[:77])
    np.testing.assert_array_equal(to_np(p2), to_np(p1)[:77])
    with pytest.raises(ffb.FFBError):
        ctx.inverse(dn, torch.as_tensor(big, device="cuda"), 1, L)


def test_full_size_sampled_and_round_trip():
    L = 1024
    nodes = synth.warped_nodes(L, L, 6, amp=0.4)
    # the graticule of the inverse at 1/2-cell sampling: about 4.2 M queries
    s = np.arange(0.25, L, 0.5)
    q = np.stack(np.meshgrid(s, s, indexing="xy"), -1).reshape(-1, 2).astype(np.float32)
    t, p = _gpu(nodes, L, L, q)
    ok = t >= 0
    print(f"[inverse] full size: found {ok.sum()}/{len(t)}", flush=True)
    assert ok.mean() > 0.99
    back = _forward_pl(nodes, L, L, p[ok])
    np.testing.assert_allclose(back, q[ok].astype(np.float64), rtol=0, atol=1e-8)
    rng = np.random.default_rng(8)
    idx = rng.choice(len(q), 512, replace=False)
    t_ref, p_ref = oracle.inverse(nodes, L, L, q[idx])
    np.testing.assert_array_equal(t[idx], t_ref)
    np.testing.assert_allclose(p[idx], p_ref, rtol=0, atol=1e-12)


def test_graticule_helper_on_identity_and_warp():
    L = 32
    ctx = new_ctx(L, L)
    g = torch.as_tensor(synth.grid_nodes(L, L), device="cuda")
    vert, horz = ctx.graticule(g, spacing=8.0, samples=2)
    v, h = to_np(vert), to_np(horz)
    assert v.shape == (3, 2 * L + 1, 2) and h.shape == (3, 2 * L + 1, 2)
    inside = (np.abs(v[..., 1] - L / 2) <= L / 2 - 0.5)
    # the identity map: the line x = 8 k maps to itself
    np.testing.assert_allclose(v[..., 0][inside], np.repeat([8.0, 16.0, 24.0], inside.sum(1)),
                               atol=1e-12)
    assert np.all(np.isnan(v[~inside]))
    # a warped map: every sample inside the hull maps back onto its line
    nodes = synth.warped_nodes(L, L, 9, amp=0.3)
    vert, _ = ctx.graticule(torch.as_tensor(nodes, device="cuda"), spacing=8.0, samples=2)
    v = to_np(vert)
    ok = ~np.isnan(v[..., 0])
    back = _forward_pl(nodes, L, L, v[ok])
    np.testing.assert_allclose(back[:, 0], np.repeat([8.0, 16.0, 24.0], ok.sum(1)), atol=1e-9)
    ctx.close()
