"""Seeded bounded-Voronoi maps standing in for the paper's country maps.

A map is a set of regions inside an Lx x Ly box [0, Lx] x [0, Ly] (the paper places the
mapped area in a rectangular box with reflecting edges and fills the space
around it with the mean density; main text, section "Flow-based cartogram
with linear equalization" and the benchmarking section).  Regions are the
Voronoi cells of seeds drawn uniformly in an inner rectangle, clipped to it.

Construction (all FP64, then vertex coordinates rounded once to FP32):

* every cell is built by clipping the inner rectangle with the bisector
  half-planes of the other seeds, nearest first, stopping once no remaining
  seed can reach the cell;
* every polygon corner carries the pair of constraint lines that meet there,
  so a corner shared by neighbouring cells gets one canonical key and one
  coordinate computed from that key (shared vertices are bit-identical and
  stored once);
* every edge is split into ceil(length / s) equal parts along its canonical
  direction, so both cells that share an edge reference the same
  subdivision vertices;
* rings are counter-clockwise, one ring per region (convex cells), unless
  enclaves (a region inside another, which then has a clockwise hole ring on
  the same vertices) or merged cells (one region, two rings) are asked for.

The statistic of region r is value_r = d_r * A_r, where d_r is the drawn
target density and A_r the area of the cell's FP32 polygon (evaluated here
with a triangle fan in FP64, purely to synthesise a statistic whose density
has the requested distribution).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["CartogramMap", "make_map", "workload", "grid_nodes", "WORKLOADS"]


@dataclass
class CartogramMap:
    """Polygon geometry in CSR-ring form plus per-region statistics."""

    lx: int
    ly: int
    xy: np.ndarray            # float32 [V, 2], box coordinates
    ring_offsets: np.ndarray  # int32 [n_rings + 1]
    ring_vidx: np.ndarray     # int32 [E]
    ring_region: np.ndarray   # int32 [n_rings]
    n_regions: int
    density: np.ndarray       # float64 [R], drawn target density d_r
    value: np.ndarray         # float64 [R], statistic d_r * A_r
    seeds: np.ndarray = field(repr=False, default=None)
    name: str = ""

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_rings(self) -> int:
        return int(self.ring_region.shape[0])

    @property
    def n_entries(self) -> int:
        return int(self.ring_vidx.shape[0])


def grid_nodes(lx: int, ly: int) -> np.ndarray:
    """Cell centres (i + 1/2, j + 1/2), row-major with x fastest, float32."""
    jj, ii = np.meshgrid(np.arange(ly, dtype=np.float64),
                         np.arange(lx, dtype=np.float64), indexing="ij")
    out = np.empty((lx * ly, 2), dtype=np.float32)
    out[:, 0] = (ii + 0.5).ravel()
    out[:, 1] = (jj + 0.5).ravel()
    return out


def warped_nodes(lx: int, ly: int, seed: int, amp: float = 0.3, modes: int = 6,
                 linear=((1.0, 0.0), (0.0, 1.0))) -> np.ndarray:
    """Grid nodes moved by a seeded smooth displacement, float32 [ly*lx, 2]:
    a linear part (rows of ``linear``) applied to the cell centres plus a sum
    of ``modes`` random sinusoids per axis, each of amplitude ``amp`` grid
    units and wavelength between 8 cells and the grid size (at least 8).  Stands in for
    the positions of the grid nodes after the rounds of a cartogram."""
    rng = np.random.default_rng(seed)
    g = grid_nodes(lx, ly).astype(np.float64)
    A = np.asarray(linear, dtype=np.float64)
    out = g @ A.T
    n = max(lx, ly, 8)
    for axis in range(2):
        for _ in range(modes):
            kx, ky = rng.uniform(-1.0, 1.0, 2) * 2.0 * np.pi / rng.uniform(8.0, n)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            out[:, axis] += amp * np.sin(kx * g[:, 0] + ky * g[:, 1] + ph)
    return out.astype(np.float32)


# --------------------------------------------------------------------------
# Voronoi construction with labelled constraint lines
# --------------------------------------------------------------------------
# Edge labels: ("B", side) for the inner rectangle's sides 0=bottom, 1=right,
# 2=top, 3=left; ("S", i, j) with i < j for the bisector of seeds i and j.
# The inner rectangle is box = (x0, x1, y0, y1).


def _line_of(label, seeds, box):
    """Return (n, c) with the line n . p = c for a constraint label."""
    if label[0] == "B":
        side = label[1]
        x0, x1, y0, y1 = box
        if side == 0:
            return np.array([0.0, 1.0]), y0
        if side == 1:
            return np.array([1.0, 0.0]), x1
        if side == 2:
            return np.array([0.0, 1.0]), y1
        return np.array([1.0, 0.0]), x0
    _, i, j = label
    si, sj = seeds[i], seeds[j]
    n = sj - si
    c = 0.5 * float(np.dot(sj, sj) - np.dot(si, si))
    return n, c


def _intersect(l1, l2, seeds, box):
    n1, c1 = _line_of(l1, seeds, box)
    n2, c2 = _line_of(l2, seeds, box)
    det = n1[0] * n2[1] - n1[1] * n2[0]
    x = (c1 * n2[1] - c2 * n1[1]) / det
    y = (n1[0] * c2 - n2[0] * c1) / det
    return np.array([x, y])


def _vertex_key(l_in, l_out):
    """Canonical key of the corner where two constraint lines meet."""
    a, b = l_in, l_out
    if a[0] == "S" and b[0] == "S":
        return ("V",) + tuple(sorted(set(a[1:]) | set(b[1:])))
    if a[0] == "B" and b[0] == "B":
        return ("C",) + tuple(sorted((a[1], b[1])))
    s = a if a[0] == "S" else b
    e = b if a[0] == "S" else a
    return ("E", s[1], s[2], e[1])


def _key_point(key, seeds, box):
    """Coordinates of a canonical corner, computed from its key only."""
    if key[0] == "V":
        i, j, k = key[1:]
        return _intersect(("S", i, j), ("S", i, k), seeds, box)
    if key[0] == "C":
        return _intersect(("B", key[1]), ("B", key[2]), seeds, box)
    _, i, j, side = key
    return _intersect(("S", i, j), ("B", side), seeds, box)


def _voronoi_cells(seeds: np.ndarray, box):
    """List of cells; each cell is a list of (point, outgoing label)."""
    n = seeds.shape[0]
    x0, x1, y0, y1 = box
    cells = []
    for i in range(n):
        si = seeds[i]
        poly = [(np.array([x0, y0]), ("B", 0)), (np.array([x1, y0]), ("B", 1)),
                (np.array([x1, y1]), ("B", 2)), (np.array([x0, y1]), ("B", 3))]
        d = np.hypot(seeds[:, 0] - si[0], seeds[:, 1] - si[1])
        order = np.argsort(d, kind="stable")
        for j in order:
            if j == i:
                continue
            reach = max(np.hypot(p[0] - si[0], p[1] - si[1]) for p, _ in poly)
            if 0.5 * d[j] > reach:
                break
            lab = ("S", min(i, j), max(i, j))
            nrm = seeds[j] - si
            c = 0.5 * float(np.dot(seeds[j], seeds[j]) - np.dot(si, si))
            out = []
            m = len(poly)
            for k in range(m):
                p, lp = poly[k]
                q, _ = poly[(k + 1) % m]
                fp = float(np.dot(nrm, p)) - c
                fq = float(np.dot(nrm, q)) - c
                pin, qin = fp <= 0.0, fq <= 0.0
                if pin:
                    out.append((p, lp))
                if pin != qin:
                    w = fp / (fp - fq)
                    ip = p + w * (q - p)
                    out.append((ip, lab if pin else lp))
            poly = out
        cells.append(poly)
    return cells


def _cell_area(pts: np.ndarray) -> float:
    """Signed area (counter-clockwise positive) of a simple polygon by a
    triangle fan from its first corner."""
    o = pts[0]
    a = 0.0
    for k in range(1, len(pts) - 1):
        u = pts[k] - o
        v = pts[k + 1] - o
        a += 0.5 * (u[0] * v[1] - u[1] * v[0])
    return a


def _draw_density(rng, kind: str, n: int) -> np.ndarray:
    if kind == "loguniform":
        return np.exp(rng.uniform(math.log(0.2), math.log(5.0), n))
    if kind == "lognormal":
        return rng.lognormal(0.0, 1.0, n)
    if kind == "pareto":
        return np.minimum(rng.pareto(1.2, n) + 1.0, 1.0e3)
    raise ValueError(f"unknown density law {kind!r}")


def make_map(L: int, n_seeds: int, seed: int, density: str,
             inner: tuple[float, float] | None = None,
             target_vertices: int | None = None,
             spacing: float | None = None, name: str = "",
             ly: int | None = None, inner_y: tuple[float, float] | None = None,
             enclaves: int = 0, merges: int = 0) -> CartogramMap:
    """Build one seeded Voronoi map in an L x ly box (ly defaults to L).

    Exactly one of ``target_vertices`` (total unique edge length divided by
    this count gives the subdivision spacing s) or ``spacing`` (s itself)
    sets the edge subdivision.  ``inner`` and ``inner_y`` bound the seeds
    and the cells along x and y (default: the middle two thirds of each
    side).  ``enclaves`` cells each get a region inside them (their seed's
    cell scaled by 0.45 about the seed) that the host region surrounds as a
    hole: a second, clockwise ring of the host on the same vertices.
    ``merges`` pairs of cells become one region with two rings
    (multipolygons).  Region densities are drawn per region.
    """
    Ly = L if ly is None else int(ly)
    if inner is None:
        inner = (L / 6.0, 5.0 * L / 6.0)
    if inner_y is None:
        inner_y = inner if Ly == L else (Ly / 6.0, 5.0 * Ly / 6.0)
    lo, hi = float(inner[0]), float(inner[1])
    box = (lo, hi, float(inner_y[0]), float(inner_y[1]))
    rng = np.random.default_rng(seed)
    if box[2:] == box[:2]:
        seeds = rng.uniform(lo, hi, size=(n_seeds, 2))
    else:
        seeds = rng.uniform((box[0], box[2]), (box[1], box[3]), size=(n_seeds, 2))
    dens = _draw_density(rng, density, n_seeds)

    cells = _voronoi_cells(seeds, box)

    # canonical corners
    key_id: dict = {}
    key_pts: list = []
    cell_keys = []
    for poly in cells:
        m = len(poly)
        ks = []
        for k in range(m):
            lin = poly[k - 1][1]
            lout = poly[k][1]
            key = _vertex_key(lin, lout)
            if key not in key_id:
                key_id[key] = len(key_pts)
                key_pts.append(_key_point(key, seeds, box))
            ks.append(key_id[key])
        # drop repeated consecutive corners (degenerate zero-length edges)
        ks2 = [ks[k] for k in range(len(ks)) if ks[k] != ks[k - 1]]
        cell_keys.append(ks2)
    corners = np.array(key_pts, dtype=np.float64)

    # unique edges and spacing
    edges = {}
    for ks in cell_keys:
        for k in range(len(ks)):
            a, b = ks[k], ks[(k + 1) % len(ks)]
            e = (min(a, b), max(a, b))
            if e not in edges:
                edges[e] = float(np.hypot(*(corners[e[1]] - corners[e[0]])))
    total_len = sum(edges.values())
    if spacing is None:
        if target_vertices is None:
            spacing = math.inf
        else:
            spacing = total_len / float(target_vertices)

    # vertices in ring-traversal order (spatial locality along borders)
    vert_of_corner = -np.ones(len(corners), dtype=np.int64)
    edge_inner: dict = {}
    xy_list: list = []

    n_xy = [0]

    def corner_vid(c):
        if vert_of_corner[c] < 0:
            vert_of_corner[c] = n_xy[0]
            xy_list.append(corners[c][None, :])
            n_xy[0] += 1
        return int(vert_of_corner[c])

    ring_vidx = []
    ring_offsets = [0]
    for ks in cell_keys:
        ring = []
        for k in range(len(ks)):
            a, b = ks[k], ks[(k + 1) % len(ks)]
            ring.append(np.array([corner_vid(a)], dtype=np.int64))
            e = (min(a, b), max(a, b))
            if e not in edge_inner:
                nseg = max(1, int(math.ceil(edges[e] / spacing))) if math.isfinite(spacing) else 1
                p0, p1 = corners[e[0]], corners[e[1]]
                w = np.arange(1, nseg, dtype=np.float64)[:, None] / nseg
                first = n_xy[0]
                if nseg > 1:
                    xy_list.append(p0[None, :] + w * (p1 - p0)[None, :])
                    n_xy[0] += nseg - 1
                edge_inner[e] = np.arange(first, first + nseg - 1, dtype=np.int64)
            ids = edge_inner[e]
            ring.append(ids if a == e[0] else ids[::-1])
        ring = np.concatenate(ring)
        ring_vidx.append(ring)
        ring_offsets.append(ring_offsets[-1] + ring.shape[0])

    ring_region = list(range(n_seeds))
    if enclaves or merges:
        pick = rng.permutation(n_seeds)
        hosts = pick[:enclaves]
        pairs = pick[enclaves:enclaves + 2 * merges].reshape(-1, 2)
        region_of_cell = np.arange(n_seeds)
        for a, b in pairs:
            region_of_cell[b] = region_of_cell[a]
        ring_region = [int(region_of_cell[c]) for c in range(n_seeds)]
        next_region = n_seeds
        for c in hosts:
            # enclave corners: the cell's corners pulled towards its seed
            ks = cell_keys[c]
            pts = seeds[c][None, :] + 0.45 * (corners[ks] - seeds[c][None, :])
            ring = []
            for k in range(len(ks)):
                p0, p1 = pts[k], pts[(k + 1) % len(ks)]
                length = float(np.hypot(*(p1 - p0)))
                nseg = max(1, int(math.ceil(length / spacing))) if math.isfinite(spacing) else 1
                w = np.arange(0, nseg, dtype=np.float64)[:, None] / nseg
                xy_list.append(p0[None, :] + w * (p1 - p0)[None, :])
                ring.append(np.arange(n_xy[0], n_xy[0] + nseg, dtype=np.int64))
                n_xy[0] += nseg
            ring = np.concatenate(ring)
            # the host's hole (clockwise), then the enclave (counter-clockwise)
            for rr, reg in ((ring[::-1], ring_region[c]), (ring, next_region)):
                ring_vidx.append(rr)
                ring_offsets.append(ring_offsets[-1] + rr.shape[0])
                ring_region.append(reg)
            next_region += 1
        # compact region ids in order of first appearance
        ids = {}
        ring_region = [ids.setdefault(r, len(ids)) for r in ring_region]
    n_regions = max(ring_region) + 1
    if n_regions != n_seeds:
        dens = np.concatenate([dens, _draw_density(rng, density, max(0, n_regions - n_seeds))])
        dens = dens[:n_regions]

    xy = np.concatenate(xy_list, axis=0).astype(np.float32)
    ring_offsets_a = np.array(ring_offsets, dtype=np.int32)
    ring_vidx_a = np.concatenate(ring_vidx).astype(np.int32)
    ring_region_a = np.array(ring_region, dtype=np.int32)

    areas = np.zeros(n_regions)
    for g in range(ring_region_a.shape[0]):
        pts = xy[ring_vidx_a[ring_offsets_a[g]:ring_offsets_a[g + 1]]].astype(np.float64)
        areas[ring_region_a[g]] += _cell_area(pts)
    value = dens * areas
    return CartogramMap(lx=L, ly=Ly, xy=xy, ring_offsets=ring_offsets_a,
                        ring_vidx=ring_vidx_a, ring_region=ring_region_a,
                        n_regions=n_regions, density=dens, value=value,
                        seeds=seeds, name=name)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    # L = 64, 16 seeds in the inner 48 x 48 square (8-cell padding),
    # log-uniform densities in [0.2, 5], about 2k vertices.
    "c1_L64": dict(L=64, n_seeds=16, seed=1, density="loguniform",
                   inner=(8.0, 56.0), target_vertices=2000),
    # L = 512, 50 seeds, lognormal(sigma = 1), about 100k vertices.
    "c2_L512": dict(L=512, n_seeds=50, seed=2, density="lognormal",
                    target_vertices=100_000),
    # L = 1024, 600 seeds, Pareto(alpha = 1.2) clipped at 1e3, about 1M vertices.
    "c3_L1024": dict(L=1024, n_seeds=600, seed=3, density="pareto",
                     target_vertices=1_000_000),
    # L = 512, 50 seeds, lognormal: the differentiation workload.
    "c5_L512": dict(L=512, n_seeds=50, seed=5, density="lognormal",
                    target_vertices=100_000),
    # Rectangular boxes with holes and multipolygons: enclaves inside their
    # host regions (the host has a clockwise ring around each) and pairs of
    # cells merged into one region with two rings.
    "rect_128x64": dict(L=128, ly=64, n_seeds=24, seed=6, density="loguniform",
                        inner=(16.0, 112.0), inner_y=(8.0, 56.0), target_vertices=4000,
                        enclaves=3, merges=2),
    "rect_256x512": dict(L=256, ly=512, n_seeds=60, seed=7, density="lognormal",
                         spacing=0.5, enclaves=4, merges=3),
    "rect_1024x512": dict(L=1024, ly=512, n_seeds=300, seed=8, density="lognormal",
                          target_vertices=500_000, enclaves=20, merges=10),
}


def workload(name: str) -> CartogramMap:
    """Build a named workload (see ``WORKLOADS``)."""
    if name.startswith("c4_"):
        # c4_<m>: map m of the batched set: L from {128, 256, 512},
        # 20-200 regions, lognormal densities, edge spacing 0.5 cells.
        m = int(name.split("_")[1])
        rng = np.random.default_rng(4000 + m)
        L = int(rng.choice([128, 256, 512]))
        n = int(rng.integers(20, 201))
        return make_map(L, n, 4000 + m, "lognormal", spacing=0.5, name=name)
    kw = dict(WORKLOADS[name])
    return make_map(name=name, **kw)
