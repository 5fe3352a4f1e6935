"""Helpers for the GPU parity tests: move seeded inputs to the device, and
pack oracle fields into the library's field layout through the C ABI."""
import numpy as np
import torch

import paper_1802_07625_amd as ffb
import synth

DEV = "cuda"


def dev_f64(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=DEV)


def dev_f32(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device=DEV).contiguous()


def to_np(t):
    return t.detach().cpu().numpy()


def map_points(m, with_grid=True):
    """Vertices first, then (optionally) every grid node; float32."""
    parts = [m.xy.astype(np.float32)]
    if with_grid:
        parts.append(synth.grid_nodes(m.lx, m.ly))
    return np.concatenate(parts).astype(np.float32)


def pack_oracle_fields(ctx, F):
    """Oracle fields (FP64 node arrays) rounded to FP32 and packed into the
    ghosted layout by the library's own pack entry point; returns
    (fields tensor, rho_bar tensor, the FP32-rounded oracle Fields)."""
    Fr = F.rounded_f32()
    fields = ctx.pack_fields(dev_f32(Fr.jx), dev_f32(Fr.jy), dev_f32(Fr.rho_s))
    return fields, dev_f64([F.rho_bar]), Fr


def stats_of(stats):
    s = to_np(stats)
    return dict(accepted=int(s[0]), rejected=int(s[1]), attempts=int(s[2]), status=int(s[3]))


def new_ctx(lx, ly=None, max_points=0, mode=None):
    ctx = ffb.Context(lx, lx if ly is None else ly, max_points=max_points)
    if mode is not None:
        ctx.set_option(ffb.OPT_ADVECT_STATE, mode)
    return ctx


def l1_perimeters(m, xy):
    """Per-region sum over its ring edges of |dx| + |dy| (FP64)."""
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    per = np.zeros(m.n_regions)
    for g in range(len(m.ring_region)):
        idx = m.ring_vidx[m.ring_offsets[g]:m.ring_offsets[g + 1]]
        p = xy[idx]
        per[m.ring_region[g]] += np.abs(np.roll(p, -1, axis=0) - p).sum()
    return per


def area_bound(m, xy_ref, dx):
    """Largest |A_r - A_r(ref)| when every vertex is within dx (max norm) of
    the reference: the shoelace sum changes at first order by at most
    dx * sum over edges (|dx_e| + |dy_e|); 1 % covers the second order, and
    1e-12 relative the FP64 sums."""
    return 1.01 * dx * l1_perimeters(m, xy_ref)


def gpu_gradient(m, density, sigmas, schedules=None, with_grid=False, max_steps=512):
    """dL/dd on the device through FFBFunction and torch autograd."""
    V = m.n_vertices
    pts_np = m.xy.astype(np.float32)
    if with_grid:
        pts_np = np.concatenate([pts_np, synth.grid_nodes(m.lx, m.ly)])
    pts = dev_f32(pts_np).reshape(-1, 2)
    ctx = new_ctx(m.lx, m.ly, max_points=pts.shape[0])
    geom = ffb.Geometry.from_map(m, pts[:V])
    a0, _, _ = ctx.area_error(geom, dev_f64(np.ones(m.n_regions)))
    d = dev_f64(density).requires_grad_(True)
    value = d * a0
    replay = None if schedules is None else [dev_f64(s) for s in schedules]
    area = ffb.FFBFunction.apply(value, ctx, geom, pts, sigmas, None, max_steps, replay)
    T = value * area.sum() / value.sum()
    e = area / T - 1.0
    loss = (e * e).sum()
    loss.backward()
    assert ctx.sync(check=False) == 0
    return float(loss.detach()), to_np(d.grad)
