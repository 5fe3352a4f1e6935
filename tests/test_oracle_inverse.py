"""Pins of the oracle's inverse of the piecewise-linear T (Conclusion: the
graticule of the inverse transformation; T approximated as piecewise linear
and inverted).

* Identity and affine maps: a piecewise-linear map reproduces an affine map
  exactly, so the preimage is A^-1 (q - b) (FP64 rounding), and the query
  is outside every triangle beyond the hull of the nodes.
* A query at the centroid of a triangle's image is found in that triangle.
* Round trip on a warped map: the forward piecewise-linear map, written out
  here on its own (cell of the preimage, the diagonal test, barycentric
  weights in the original cell applied to the images), takes each preimage
  back to its query.
* A reflection (every image triangle clockwise) is inverted as well, and
  where two image triangles overlap the lower-numbered one is taken.
"""
import numpy as np
import pytest

import oracle
import synth


def _affine_nodes(lx, ly, A, b):
    g = synth.grid_nodes(lx, ly).astype(np.float64)
    return (g @ np.asarray(A, dtype=np.float64).T + np.asarray(b)).astype(np.float32)


def _forward_pl(nodes, lx, ly, p):
    """T_PL(p) from the images of the cell centres, for p in the node hull."""
    T = np.asarray(nodes, dtype=np.float64).reshape(ly, lx, 2)
    u, v = p[:, 0] - 0.5, p[:, 1] - 0.5
    i = np.clip(np.floor(u).astype(int), 0, lx - 2)
    j = np.clip(np.floor(v).astype(int), 0, ly - 2)
    a, b = u - i, v - j
    lower = a >= b          # below the (i,j)-(i+1,j+1) diagonal: corners 00, 10, 11
    out = np.empty_like(p)
    t00, t10, t11, t01 = T[j, i], T[j, i + 1], T[j + 1, i + 1], T[j + 1, i]
    lo = (1 - a)[:, None] * t00 + (a - b)[:, None] * t10 + b[:, None] * t11
    up = (1 - b)[:, None] * t00 + (b - a)[:, None] * t01 + a[:, None] * t11
    out[:] = np.where(lower[:, None], lo, up)
    return out


def test_identity_map():
    L = 16
    nodes = synth.grid_nodes(L, L)
    rng = np.random.default_rng(0)
    q = rng.uniform(0.5, L - 0.5, (300, 2)).astype(np.float32)
    tri, pre = oracle.inverse(nodes, L, L, q)
    assert np.all(tri >= 0)
    np.testing.assert_allclose(pre, q.astype(np.float64), rtol=0, atol=1e-12)
    # outside the hull of the nodes: no triangle
    out = np.array([[0.2, 5.0], [L - 0.3, 5.0], [5.0, 0.1], [-3.0, -3.0]], np.float32)
    tri, pre = oracle.inverse(nodes, L, L, out)
    assert np.all(tri == -1) and np.all(np.isnan(pre))


@pytest.mark.parametrize("A,b", [(((2.0, 0.5), (0.25, 1.5)), (3.0, -1.0)),
                                 (((0.0, -1.0), (1.0, 0.0)), (20.0, 0.0)),
                                 (((1.3, 0.2), (-0.4, 0.9)), (0.7, 4.1))])
def test_affine_maps(A, b):
    lx, ly = 12, 9
    nodes = _affine_nodes(lx, ly, A, b)
    rng = np.random.default_rng(1)
    p = rng.uniform(0.6, [lx - 0.6, ly - 0.6], (400, 2))
    q = (p @ np.asarray(A).T + np.asarray(b)).astype(np.float32)
    tri, pre = oracle.inverse(nodes, lx, ly, q)
    assert np.all(tri >= 0)
    expect = np.linalg.solve(np.asarray(A), (q.astype(np.float64) - np.asarray(b)).T).T
    # the FP32 images of the nodes make the map affine only to ~1e-6 cells
    np.testing.assert_allclose(pre, expect, rtol=0, atol=2e-5)


def test_centroids_are_found_in_their_triangle():
    lx, ly = 10, 7
    nodes = synth.warped_nodes(lx, ly, 3, amp=0.2).astype(np.float64).reshape(ly, lx, 2)
    qs, want = [], []
    for t in range(0, 2 * (lx - 1) * (ly - 1), 7):
        c = t >> 1
        i, j = c % (lx - 1), c // (lx - 1)
        if t & 1 == 0:
            corners = [nodes[j, i], nodes[j, i + 1], nodes[j + 1, i + 1]]
        else:
            corners = [nodes[j, i], nodes[j + 1, i + 1], nodes[j + 1, i]]
        qs.append(np.mean(corners, axis=0))
        want.append(t)
    tri, _ = oracle.inverse(nodes.reshape(-1, 2), lx, ly, np.array(qs))
    np.testing.assert_array_equal(tri, want)


def test_round_trip_on_a_warped_map():
    lx, ly = 40, 24
    nodes = synth.warped_nodes(lx, ly, 4, amp=0.35)
    rng = np.random.default_rng(2)
    p0 = rng.uniform(1.0, [lx - 1.0, ly - 1.0], (500, 2))
    q = _forward_pl(nodes, lx, ly, p0).astype(np.float32)
    tri, pre = oracle.inverse(nodes, lx, ly, q)
    assert np.all(tri >= 0)
    back = _forward_pl(nodes, lx, ly, pre)
    np.testing.assert_allclose(back, q.astype(np.float64), rtol=0, atol=1e-9)
    # and (no fold here) the preimage is the original point up to the FP32
    # rounding of the queries
    np.testing.assert_allclose(pre, p0, rtol=0, atol=1e-3)


def test_reflection_and_overlaps():
    L = 8
    g = synth.grid_nodes(L, L)
    ref = g.copy()
    ref[:, 0] = L - ref[:, 0]
    q = np.array([[2.3, 3.7], [6.1, 1.2]], np.float32)
    tri, pre = oracle.inverse(ref, L, L, q)
    np.testing.assert_allclose(pre, np.stack([L - q[:, 0], q[:, 1]], 1), atol=1e-12)
    # fold one node over its neighbour: image triangles overlap near it; a
    # query inside several is assigned to the lowest-numbered one
    nodes = g.copy().reshape(L, L, 2)
    nodes[3, 3] = (5.2, 3.5)                     # pulled across the node (4, 3)
    flat = nodes.reshape(-1, 2)

    def cross(u, v):
        return u[0] * v[1] - u[1] * v[0]

    def hits(q):
        out = []
        for t in range(2 * (L - 1) ** 2):
            c = t >> 1
            i, j = c % (L - 1), c // (L - 1)
            idx = [(j, i), (j, i + 1), (j + 1, i + 1)] if t % 2 == 0 else \
                  [(j, i), (j + 1, i + 1), (j + 1, i)]
            P = [nodes[a, b].astype(np.float64) for a, b in idx]
            o = cross(P[1] - P[0], P[2] - P[0])
            d = [cross(P[(k + 1) % 3] - P[k], q - P[k]) for k in range(3)]
            if o != 0 and (all(x >= 0 for x in d) if o > 0 else all(x <= 0 for x in d)):
                out.append(t)
        return out

    rng = np.random.default_rng(3)
    cand = rng.uniform(3.0, 6.0, (400, 2)).astype(np.float32)
    multi = [(q, h) for q in cand for h in [hits(q.astype(np.float64))] if len(h) >= 2][:10]
    assert len(multi) >= 3
    tri, _ = oracle.inverse(flat, L, L, np.array([q for q, _ in multi]))
    np.testing.assert_array_equal(tri, [min(h) for _, h in multi])
