"""Angular distortion of the map given by the grid nodes (main text, section
"Measures of distortion"; SI Appendix section 3) against the oracle.

Both sides read the same FP32 node positions (from the oracle's rounds, or a
seeded smooth deformation), so the per-square Jacobians agree to FP64
rounding.  The device takes the singular values in closed form, the oracle
from LAPACK's SVD; the smaller one loses about eps * a / b to cancellation in
the closed form, so per-square e and e~ (FP32 outputs) agree to 2e-6
absolute plus 2e-6 relative and the FP64 summaries to 1e-9 relative
(the maps here have a / b below 1e3).  The folded-square counts are integers
decided by the sign of the same FP64 determinant: equal.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1802_07625_amd as ffb
import synth
from gpu_util import to_np

pytestmark = pytest.mark.gpu


def _gpu(nodes32, lx, ly, per_square=True):
    ctx = ffb.Context(8, 8, max_points=0)
    print(f"[distortion] gpu lx={lx} ly={ly} per_square={per_square}", flush=True)
    stats, e, et = ctx.distortion(torch.as_tensor(nodes32, device="cuda"), per_square, lx, ly)
    ctx.sync()
    out = to_np(stats), (None if e is None else to_np(e)), (None if et is None else to_np(et))
    ctx.close()
    return out


def _compare(nodes32, lx, ly, tag):
    ref = oracle.distortion(nodes32.astype(np.float64), lx, ly)
    stats, e, et = _gpu(nodes32, lx, ly)
    print(f"[distortion] {tag} lx={lx} ly={ly} e_a={stats[0]:.6e} e_inf={stats[1]:.6e} "
          f"e~_a={stats[2]:.6e} e~_inf={stats[3]:.6e} folded={int(stats[4])} "
          f"oracle e_a={ref.e_a:.6e} e_inf={ref.e_inf:.6e} folded={ref.folded}", flush=True)
    assert e.shape == (ly - 1, lx - 1)
    np.testing.assert_allclose(e, ref.e, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(et, ref.e_tilde, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(stats[:4], [ref.e_a, ref.e_inf, ref.e_tilde_a, ref.e_tilde_inf],
                               rtol=1e-9, atol=1e-15)
    assert int(stats[4]) == ref.folded
    return stats, ref


def test_nodes_after_oracle_rounds_c1():
    m = synth.workload("c1_L64")
    L = m.lx
    pts = np.concatenate([m.xy, synth.grid_nodes(L, L)])
    rr = oracle.rounds(m, m.density, [ffb.default_sigma(k) for k in range(3)], points=pts)
    nodes = rr.points[m.n_vertices:].astype(np.float32)
    stats, _ = _compare(nodes, L, L, "c1 after 3 oracle rounds")
    assert stats[0] > 1e-3          # the cartogram does distort the grid


@pytest.mark.parametrize("lx,ly,seed", [(64, 64, 1), (96, 40, 2), (1024, 1024, 3)])
def test_smooth_deformation(lx, ly, seed):
    nodes = synth.warped_nodes(lx, ly, seed, amp=0.3)
    _compare(nodes, lx, ly, f"warp seed={seed}")


def test_partly_folded_map():
    # displacement gradients above 1 fold part of the grid
    nodes = synth.warped_nodes(128, 128, 4, amp=2.5)
    stats, ref = _compare(nodes, 128, 128, "warp folded")
    assert 0 < ref.folded < 127 * 127


def test_conformal_and_folded_maps():
    L = 64
    g = synth.grid_nodes(L, L)
    # rotation by 30 degrees and scaling by 1.7: conformal, e = e~ = 0 up to
    # the FP32 rounding of the node positions (half an ulp of ~110 per
    # coordinate moves a / b by at most ~2e-5)
    c, s = 1.7 * np.cos(np.pi / 6), 1.7 * np.sin(np.pi / 6)
    rot = synth.warped_nodes(L, L, 0, amp=0.0, linear=((c, -s), (s, c)))
    stats, e, et = _gpu(rot, L, L)
    assert np.abs(stats[:4]).max() < 5e-5 and int(stats[4]) == 0
    # a reflection is conformal but flips orientation: every square folded
    ref = g.copy()
    ref[:, 0] = L - ref[:, 0]
    stats, _, _ = _gpu(ref, L, L)
    assert np.abs(stats[:4]).max() == 0.0 and int(stats[4]) == (L - 1) ** 2
    # the shear x -> x + k y (positions exact in FP32): singular values
    # a = (sqrt(k^2 + 4) + k) / 2 and b = 1 / a on every square
    sh = synth.warped_nodes(L, L, 0, amp=0.0, linear=((1.0, 0.5), (0.0, 1.0)))
    stats, e, _ = _gpu(sh, L, L)
    k = 0.5
    a = 0.5 * (np.sqrt(k * k + 4) + k)            # singular values of [[1, k], [0, 1]]
    b = 1.0 / a
    np.testing.assert_allclose(e, np.log(a / b), rtol=1e-6)
    np.testing.assert_allclose(stats[0], np.log(a / b), rtol=1e-9)


def test_stats_only_and_small_grids():
    for lx, ly in [(2, 2), (2, 17), (33, 3), (257, 129)]:
        nodes = synth.warped_nodes(lx, ly, 7, amp=0.1)
        ref = oracle.distortion(nodes.astype(np.float64), lx, ly)
        stats, e, et = _gpu(nodes, lx, ly, per_square=False)
        assert e is None and et is None
        np.testing.assert_allclose(stats[:4], [ref.e_a, ref.e_inf, ref.e_tilde_a,
                                               ref.e_tilde_inf], rtol=1e-9, atol=1e-15)
        assert int(stats[4]) == ref.folded


def test_collapsed_square_is_undefined_on_both_sides():
    # four nodes on one point: grad T = 0 there, e and e~ are 0 / 0 (NaN) on
    # both sides, the means and maxima carry the NaN, and the square counts
    # as folded (det = 0)
    L = 32
    nodes = synth.warped_nodes(L, L, 5, amp=0.1)
    g = nodes.reshape(L, L, 2)
    g[10:12, 20:22] = g[10, 20]
    _compare(nodes, L, L, "collapsed square")
