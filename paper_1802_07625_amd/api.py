"""Thin Python binding of the libffb C ABI (include/ffb.h).

Only argument marshalling happens here: torch tensors supply device memory,
``torch.cuda.current_stream()`` supplies the HIP stream, and every step of
the method runs in the HIP kernels behind the C ABI.  There is no CPU
fallback: if the library is not built, importing the binding fails.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffb.so")

FFB_OK = 0
STATUS = {
    0: "FFB_OK", 1: "FFB_E_INVALID", 2: "FFB_E_NOMEM", 3: "FFB_E_DEVICE",
    4: "FFB_E_NONPOSITIVE", 5: "FFB_E_DOMAIN", 6: "FFB_E_STEP_UNDERFLOW",
    7: "FFB_E_NONFINITE", 8: "FFB_E_NO_TAPE", 9: "FFB_E_MAX_ATTEMPTS",
    10: "FFB_E_TOO_LARGE",
}
globals().update({name: code for code, name in STATUS.items()})


class FFBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class FFBGeometry(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("xy", ctypes.c_void_p),
                ("n_rings", ctypes.c_int32), ("ring_offsets", ctypes.c_void_p),
                ("ring_vidx", ctypes.c_void_p), ("ring_region", ctypes.c_void_p),
                ("n_regions", ctypes.c_int32), ("n_entries", ctypes.c_int64)]


class FFBIntegrateOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("h0", ctypes.c_double),
                ("safety", ctypes.c_double), ("fac_min", ctypes.c_double),
                ("fac_max", ctypes.c_double), ("h_min", ctypes.c_double),
                ("max_attempts", ctypes.c_int32), ("n_replay", ctypes.c_int32),
                ("replay_h", ctypes.c_void_p)]


class FFBBatchDesc(ctypes.Structure):
    _fields_ = [("n_maps", ctypes.c_int32), ("lx", ctypes.c_void_p), ("ly", ctypes.c_void_p),
                ("point_offsets", ctypes.c_void_p), ("n_vertices", ctypes.c_void_p),
                ("ring_offsets_map", ctypes.c_void_p), ("region_offsets", ctypes.c_void_p),
                ("geometry", FFBGeometry), ("points", ctypes.c_void_p), ("value", ctypes.c_void_p)]


class FFBBatchOpts(ctypes.Structure):
    _fields_ = [("stop_err", ctypes.c_double), ("max_rounds", ctypes.c_int32),
                ("sigma0", ctypes.c_double), ("integrate", FFBIntegrateOpts),
                ("use_graph", ctypes.c_int32)]


_lib = None

# Contexts and batches still open when the interpreter exits are closed by
# an exit hook, while the HIP runtime, torch and any profiler attached to the
# process are all still up; otherwise their streams, graph executables and
# device memory would be released by __del__ during interpreter teardown, in
# whatever order the collector picks, or not at all before the runtime's own
# teardown at exit().
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live():
    live = list(_LIVE)
    if not live:
        return
    try:
        torch.cuda.synchronize()
    except Exception:
        pass
    for obj in live:
        try:
            obj.close()
        except Exception:
            pass


def lib():
    """Load libffb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.ffb_create.argtypes = [ctypes.POINTER(vp), i32, i32, i64, vp]
        L.ffb_destroy.argtypes = [vp]
        L.ffb_sync.argtypes = [vp]
        L.ffb_reset_status.argtypes = [vp]
        L.ffb_last_error.argtypes = [vp]
        L.ffb_last_error.restype = ctypes.c_char_p
        G = ctypes.POINTER(FFBGeometry)
        L.ffb_area_error.argtypes = [vp, G, vp, vp, vp, vp]
        L.ffb_density.argtypes = [vp, G, vp, vp, vp, vp]
        L.ffb_flux.argtypes = [vp, vp, ctypes.c_float, vp, vp]
        L.ffb_flux_noalloc.argtypes = [i32, i32, vp, ctypes.c_float, vp, vp, vp, vp]
        L.ffb_pack_fields.argtypes = [vp, vp, vp, vp, vp]
        L.ffb_integrate.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(FFBIntegrateOpts),
                                    vp, vp, i32]
        L.ffb_set_option.argtypes = [vp, i32, i32]
        L.ffb_distortion.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp]
        L.ffb_diffusion_fields.argtypes = [vp, vp, ctypes.c_float, ctypes.c_double, vp]
        L.ffb_inverse.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, i64, vp, vp]
        L.ffb_diffusion.argtypes = [vp, vp, ctypes.c_float, ctypes.c_double, vp, i64,
                                    ctypes.POINTER(FFBIntegrateOpts), vp, vp, ctypes.c_int32]
        L.ffb_area_adj.argtypes = [vp, G, vp, vp]
        L.ffb_density_adj.argtypes = [vp, G, vp, vp, vp, vp, vp, vp]
        L.ffb_flux_adj.argtypes = [vp, ctypes.c_float, vp, vp, vp]
        L.ffb_integrate_record.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(FFBIntegrateOpts),
                                           vp, vp, i64, i32, vp]
        L.ffb_integrate_adj.argtypes = [vp, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp]
        L.ffb_tape_begin.argtypes = [vp, i32]
        L.ffb_tape_end.argtypes = [vp]
        L.ffb_tape_clear.argtypes = [vp]
        L.ffb_backward.argtypes = [vp, vp, vp, vp]
        L.ffb_tape_generation.argtypes = [vp, ctypes.POINTER(i64)]
        L.ffb_tape_check.argtypes = [vp, i64]
        B, BO = ctypes.POINTER(FFBBatchDesc), ctypes.POINTER(FFBBatchOpts)
        L.ffb_batch_create.argtypes = [ctypes.POINTER(vp), B, vp]
        L.ffb_batch_destroy.argtypes = [vp]
        L.ffb_batch_last_error.argtypes = [vp]
        L.ffb_batch_last_error.restype = ctypes.c_char_p
        L.ffb_batch_set_shapes.argtypes = [vp, i32, i32]
        L.ffb_batch_get_shapes.argtypes = [vp, vp, vp, vp, vp]
        L.ffb_batch_autotune.argtypes = [vp, BO]
        L.ffb_batch_reset.argtypes = [vp]
        L.ffb_batch_step.argtypes = [vp, BO, vp, vp]
        L.ffb_batch_run.argtypes = [vp, BO, vp]
        L.ffb_batch_results.argtypes = [vp, vp, vp, vp, vp]
        for f in ("ffb_create", "ffb_destroy", "ffb_sync", "ffb_reset_status", "ffb_area_error",
                  "ffb_density", "ffb_flux", "ffb_pack_fields", "ffb_integrate", "ffb_set_option",
                  "ffb_distortion", "ffb_diffusion_fields", "ffb_diffusion", "ffb_inverse", "ffb_area_adj", "ffb_density_adj", "ffb_flux_adj", "ffb_integrate_record",
                  "ffb_integrate_adj", "ffb_tape_begin", "ffb_tape_end", "ffb_tape_clear",
                  "ffb_backward", "ffb_tape_generation", "ffb_tape_check", "ffb_batch_create", "ffb_batch_destroy", "ffb_batch_set_shapes",
                  "ffb_batch_get_shapes", "ffb_batch_autotune", "ffb_batch_reset",
                  "ffb_batch_step", "ffb_batch_run", "ffb_batch_results"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


# ------------------------------------------------------------ marshalling
def _ptr(t: torch.Tensor | None, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs at least {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, code: int, what: str):
    if code != FFB_OK:
        detail = lib().ffb_last_error(ctx).decode() if ctx else ""
        raise FFBError(code, f"{what}: {detail}")


@dataclass
class Geometry:
    """CSR rings over unique vertices, all device tensors."""
    xy: torch.Tensor            # float32 [V, 2] (may be a view into a points tensor)
    ring_offsets: torch.Tensor  # int32 [G + 1]
    ring_vidx: torch.Tensor     # int32 [E]
    ring_region: torch.Tensor   # int32 [G]
    n_regions: int

    @classmethod
    def from_map(cls, m, xy: torch.Tensor | None = None, device="cuda"):
        """From a synthetic map (host arrays) with vertices ``xy`` (device)."""
        if xy is None:
            xy = torch.as_tensor(m.xy, dtype=torch.float32, device=device)
        t = lambda a: torch.as_tensor(a, dtype=torch.int32, device=device).contiguous()
        return cls(xy, t(m.ring_offsets), t(m.ring_vidx), t(m.ring_region), int(m.n_regions))

    def struct(self) -> FFBGeometry:
        return FFBGeometry(
            n_vertices=self.xy.shape[0], xy=_ptr(self.xy, torch.float32, name="xy"),
            n_rings=self.ring_region.numel(),
            ring_offsets=_ptr(self.ring_offsets, torch.int32, name="ring_offsets"),
            ring_vidx=_ptr(self.ring_vidx, torch.int32, name="ring_vidx"),
            ring_region=_ptr(self.ring_region, torch.int32, name="ring_region"),
            n_regions=self.n_regions, n_entries=self.ring_vidx.numel())


@dataclass
class IntegrateOpts:
    tol: float = 1e-3
    h0: float = 1e-2
    safety: float = 0.9
    fac_min: float = 0.2
    fac_max: float = 5.0
    h_min: float = 1e-7
    max_attempts: int = 4096

    def struct(self, replay_h: torch.Tensor | None = None) -> FFBIntegrateOpts:
        n = 0 if replay_h is None else replay_h.numel()
        return FFBIntegrateOpts(self.tol, self.h0, self.safety, self.fac_min, self.fac_max,
                                self.h_min, self.max_attempts, n,
                                _ptr(replay_h, torch.float64, name="replay_h"))


# ------------------------------------------------------- C-ABI functions
def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def ffb_create(lx: int, ly: int, max_points: int = 0, stream=None):
    ctx = ctypes.c_void_p()
    code = lib().ffb_create(ctypes.byref(ctx), int(lx), int(ly), int(max_points),
                            _stream_handle(stream))
    if code != FFB_OK:
        raise FFBError(code, f"ffb_create(lx={lx}, ly={ly}, max_points={max_points})")
    return ctx


def ffb_destroy(ctx) -> None:
    _check(None, lib().ffb_destroy(ctx), "ffb_destroy")


def ffb_sync(ctx) -> int:
    return int(lib().ffb_sync(ctx))


def ffb_reset_status(ctx) -> None:
    _check(ctx, lib().ffb_reset_status(ctx), "ffb_reset_status")


def ffb_last_error(ctx) -> str:
    return lib().ffb_last_error(ctx).decode()


OPT_ADVECT_STATE, OPT_ADVECT_BLOCKS, OPT_DIFFUSION_GRAPH, OPT_POINT_ORDER = 1, 2, 3, 4
# values of OPT_POINT_ORDER
POINT_ORDER_GIVEN, POINT_ORDER_AUTO, POINT_ORDER_ALWAYS, POINT_ORDER_KEEP = 0, 1, 2, 3


def ffb_set_option(ctx, option: int, value: int) -> None:
    _check(ctx, lib().ffb_set_option(ctx, int(option), int(value)), "ffb_set_option")


def ffb_area_error(ctx, geom: Geometry, value, area, err, max_abs_err) -> None:
    R = geom.n_regions
    g = geom.struct()
    _check(ctx, lib().ffb_area_error(ctx, ctypes.byref(g), _ptr(value, torch.float64, R, "value"),
                                     _ptr(area, torch.float64, R, "area"),
                                     _ptr(err, torch.float64, R, "err"),
                                     _ptr(max_abs_err, torch.float64, 1, "max_abs_err")),
           "ffb_area_error")


def ffb_density(ctx, geom: Geometry, value, area, rho, rho_pad, lx: int, ly: int) -> None:
    R = geom.n_regions
    g = geom.struct()
    _check(ctx, lib().ffb_density(ctx, ctypes.byref(g), _ptr(value, torch.float64, R, "value"),
                                  _ptr(area, torch.float64, R, "area"),
                                  _ptr(rho, torch.float64, lx * ly, "rho"),
                                  _ptr(rho_pad, torch.float64, 1, "rho_pad")), "ffb_density")


def ffb_flux(ctx, rho, sigma: float, fields, rho_bar, lx: int, ly: int) -> None:
    _check(ctx, lib().ffb_flux(ctx, _ptr(rho, torch.float64, lx * ly, "rho"), float(sigma),
                               _ptr(fields, torch.float32, 4 * (lx + 2) * (ly + 2), "fields"),
                               _ptr(rho_bar, torch.float64, 1, "rho_bar")), "ffb_flux")


def ffb_pack_fields(ctx, jx, jy, rho_s, fields, lx: int, ly: int) -> None:
    n = lx * ly
    _check(ctx, lib().ffb_pack_fields(ctx, _ptr(jx, torch.float32, n, "jx"),
                                      _ptr(jy, torch.float32, n, "jy"),
                                      _ptr(rho_s, torch.float32, n, "rho_s"),
                                      _ptr(fields, torch.float32, 4 * (lx + 2) * (ly + 2),
                                           "fields")), "ffb_pack_fields")


def ffb_integrate(ctx, fields, rho_bar, xy, opts: IntegrateOpts, stats, h_out=None,
                  replay_h=None) -> None:
    n = xy.shape[0]
    o = opts.struct(replay_h)
    _check(ctx, lib().ffb_integrate(ctx, _ptr(fields, torch.float32, name="fields"),
                                    _ptr(rho_bar, torch.float64, 1, "rho_bar"),
                                    _ptr(xy, torch.float32, 2 * n, "xy"), n, ctypes.byref(o),
                                    _ptr(stats, torch.int32, 4, "stats"),
                                    _ptr(h_out, torch.float64, name="h_out"),
                                    0 if h_out is None else h_out.numel()), "ffb_integrate")


def ffb_diffusion_fields(ctx, rho, sigma: float, t: float, fields, lx: int, ly: int) -> None:
    _check(ctx, lib().ffb_diffusion_fields(ctx, _ptr(rho, torch.float64, lx * ly, "rho"),
                                           float(sigma), float(t),
                                           _ptr(fields, torch.float32, 4 * (lx + 2) * (ly + 2),
                                                "fields")), "ffb_diffusion_fields")


def ffb_diffusion(ctx, rho, sigma: float, t_end: float, xy, opts: IntegrateOpts, stats,
                  h_out=None, replay_h=None, lx: int = 0, ly: int = 0) -> None:
    n = xy.shape[0]
    o = opts.struct(replay_h)
    _check(ctx, lib().ffb_diffusion(ctx, _ptr(rho, torch.float64, lx * ly, "rho"), float(sigma),
                                    float(t_end), _ptr(xy, torch.float32, 2 * n, "xy"), n,
                                    ctypes.byref(o), _ptr(stats, torch.int32, 4, "stats"),
                                    _ptr(h_out, torch.float64, name="h_out"),
                                    0 if h_out is None else h_out.numel()), "ffb_diffusion")


def ffb_inverse(ctx, lx: int, ly: int, nodes, queries, tri, pre) -> None:
    nq = queries.shape[0]
    _check(ctx, lib().ffb_inverse(ctx, lx, ly, _ptr(nodes, torch.float32, 2 * lx * ly, "nodes"),
                                  _ptr(queries, torch.float32, 2 * nq, "queries"), nq,
                                  _ptr(tri, torch.int32, nq, "tri"),
                                  _ptr(pre, torch.float64, 2 * nq, "pre")), "ffb_inverse")


def ffb_distortion(ctx, lx: int, ly: int, nodes, stats, e=None, e_tilde=None) -> None:
    n = max(lx - 1, 0) * max(ly - 1, 0)
    _check(ctx, lib().ffb_distortion(ctx, lx, ly, _ptr(nodes, torch.float32, 2 * lx * ly, "nodes"),
                                     _ptr(stats, torch.float64, 5, "stats"),
                                     _ptr(e, torch.float32, n, "e"),
                                     _ptr(e_tilde, torch.float32, n, "e_tilde")), "ffb_distortion")


def ffb_area_adj(ctx, geom: Geometry, lam_area, lam_xy) -> None:
    g = geom.struct()
    _check(ctx, lib().ffb_area_adj(ctx, ctypes.byref(g),
                                   _ptr(lam_area, torch.float64, geom.n_regions, "lam_area"),
                                   _ptr(lam_xy, torch.float64, 2 * g.n_vertices, "lam_xy")),
           "ffb_area_adj")


def ffb_density_adj(ctx, geom: Geometry, value, area, lam_rho, lam_value, lam_area, lam_xy,
                    lx: int, ly: int) -> None:
    R = geom.n_regions
    g = geom.struct()
    _check(ctx, lib().ffb_density_adj(
        ctx, ctypes.byref(g), _ptr(value, torch.float64, R, "value"),
        _ptr(area, torch.float64, R, "area"), _ptr(lam_rho, torch.float32, lx * ly, "lam_rho"),
        _ptr(lam_value, torch.float64, R, "lam_value"),
        _ptr(lam_area, torch.float64, R, "lam_area"),
        _ptr(lam_xy, torch.float64, 2 * g.n_vertices, "lam_xy")), "ffb_density_adj")


def ffb_flux_adj(ctx, sigma: float, lam_fields, lam_rho_bar, lam_rho, lx: int, ly: int) -> None:
    _check(ctx, lib().ffb_flux_adj(
        ctx, float(sigma), _ptr(lam_fields, torch.float32, 4 * (lx + 2) * (ly + 2), "lam_fields"),
        _ptr(lam_rho_bar, torch.float64, 1, "lam_rho_bar"),
        _ptr(lam_rho, torch.float32, lx * ly, "lam_rho")), "ffb_flux_adj")


def ffb_integrate_record(ctx, fields, rho_bar, xy, opts: IntegrateOpts, stats, tape_states,
                         tape_h, tape_n: int, replay_h=None) -> None:
    n = xy.shape[0]
    cap = tape_h.numel()
    o = opts.struct(replay_h)
    _check(ctx, lib().ffb_integrate_record(
        ctx, _ptr(fields, torch.float32, name="fields"), _ptr(rho_bar, torch.float64, 1, "rho_bar"),
        _ptr(xy, torch.float32, 2 * n, "xy"), n, ctypes.byref(o),
        _ptr(stats, torch.int32, 4, "stats"),
        _ptr(tape_states, torch.float32, 4 * cap * tape_n, "tape_states"), int(tape_n), cap,
        _ptr(tape_h, torch.float64, cap, "tape_h")), "ffb_integrate_record")


def ffb_integrate_adj(ctx, fields, rho_bar, stats, tape_states, tape_h, tape_n: int, lam_xy,
                      lam_fields, lam_rho_bar) -> None:
    cap = tape_h.numel()
    _check(ctx, lib().ffb_integrate_adj(
        ctx, _ptr(fields, torch.float32, name="fields"), _ptr(rho_bar, torch.float64, 1, "rho_bar"),
        _ptr(stats, torch.int32, 4, "stats"),
        _ptr(tape_states, torch.float32, 4 * cap * tape_n, "tape_states"), int(tape_n), cap,
        _ptr(tape_h, torch.float64, cap, "tape_h"),
        _ptr(lam_xy, torch.float64, 2 * tape_n, "lam_xy"),
        _ptr(lam_fields, torch.float32, name="lam_fields"),
        _ptr(lam_rho_bar, torch.float64, 1, "lam_rho_bar")), "ffb_integrate_adj")


def ffb_tape_begin(ctx, max_steps: int) -> None:
    _check(ctx, lib().ffb_tape_begin(ctx, int(max_steps)), "ffb_tape_begin")


def ffb_tape_end(ctx) -> None:
    _check(ctx, lib().ffb_tape_end(ctx), "ffb_tape_end")


def ffb_tape_clear(ctx) -> None:
    _check(ctx, lib().ffb_tape_clear(ctx), "ffb_tape_clear")


def ffb_tape_generation(ctx) -> int:
    g = ctypes.c_int64()
    _check(ctx, lib().ffb_tape_generation(ctx, ctypes.byref(g)), "ffb_tape_generation")
    return g.value


def ffb_tape_check(ctx, generation: int) -> None:
    _check(ctx, lib().ffb_tape_check(ctx, int(generation)), "ffb_tape_check")


def ffb_backward(ctx, dL_darea, dL_dvalue, dL_dxy0=None) -> None:
    R = dL_darea.numel()
    _check(ctx, lib().ffb_backward(ctx, _ptr(dL_darea, torch.float64, R, "dL_darea"),
                                   _ptr(dL_dvalue, torch.float64, R, "dL_dvalue"),
                                   _ptr(dL_dxy0, torch.float64, name="dL_dxy0")), "ffb_backward")


# ------------------------------------------------------------ convenience
class Context:
    """An ffb context bound to the current torch stream, with output
    allocation helpers.  Every method only enqueues work."""

    def __init__(self, lx: int, ly: int, max_points: int = 0, stream=None, device="cuda"):
        self.lx, self.ly = int(lx), int(ly)
        self.device = torch.device(device)
        self.handle = ffb_create(lx, ly, max_points, stream)
        _LIVE.add(self)
        # the record references the ring arrays of the geometries it saw
        # (the library keeps pointers, not copies): hold them while it exists
        self._recording = False
        self._tape_refs = []

    def close(self):
        if self.handle is not None:
            ffb_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, check: bool = True) -> int:
        code = ffb_sync(self.handle)
        if check and code != FFB_OK:
            raise FFBError(code, "device status after sync")
        return code

    def reset_status(self):
        ffb_reset_status(self.handle)

    def set_option(self, option: int, value: int):
        ffb_set_option(self.handle, option, value)

    def _f64(self, *shape):
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def area_error(self, geom: Geometry, value):
        R = geom.n_regions
        area, err, mx = self._f64(R), self._f64(R), self._f64(1)
        ffb_area_error(self.handle, geom, value, area, err, mx)
        self._hold(geom)
        return area, err, mx

    def density(self, geom: Geometry, value, area):
        rho = torch.empty((self.ly, self.lx), dtype=torch.float64, device=self.device)
        pad = self._f64(1)
        ffb_density(self.handle, geom, value, area, rho, pad, self.lx, self.ly)
        self._hold(geom)
        return rho, pad

    def new_fields(self):
        return torch.empty((self.ly + 2, self.lx + 2, 4), dtype=torch.float32, device=self.device)

    def flux(self, rho, sigma: float, fields=None, rho_bar=None):
        fields = self.new_fields() if fields is None else fields
        rho_bar = self._f64(1) if rho_bar is None else rho_bar
        ffb_flux(self.handle, rho, sigma, fields, rho_bar, self.lx, self.ly)
        return fields, rho_bar

    def pack_fields(self, jx, jy, rho_s, fields=None):
        fields = self.new_fields() if fields is None else fields
        ffb_pack_fields(self.handle, jx, jy, rho_s, fields, self.lx, self.ly)
        return fields

    def integrate(self, fields, rho_bar, xy, opts: IntegrateOpts | None = None,
                  replay_h=None, h_cap: int | None = None, stats=None, h_out=None):
        opts = opts or IntegrateOpts()
        stats = torch.empty(4, dtype=torch.int32, device=self.device) if stats is None else stats
        if h_out is None and (h_cap is None or h_cap > 0):
            h_out = self._f64(opts.max_attempts if h_cap is None else h_cap)
        ffb_integrate(self.handle, fields, rho_bar, xy, opts, stats, h_out, replay_h)
        return stats, h_out

    def diffusion_fields(self, rho, sigma: float, t: float, fields=None):
        """Fields (J_x, J_y, rho(t)) of the diffusion variant at time t."""
        fields = self.new_fields() if fields is None else fields
        ffb_diffusion_fields(self.handle, rho, sigma, t, fields, self.lx, self.ly)
        return fields

    def diffusion(self, rho, sigma: float, xy, t_end: float | None = None,
                  opts: IntegrateOpts | None = None, replay_h=None, h_cap: int | None = None):
        """Advect xy with the diffusion variant to t_end (default
        diffusion_t_end); returns (stats, accepted steps).  Waits for the
        integration to end."""
        opts = opts or IntegrateOpts()
        te = diffusion_t_end(self.lx, self.ly) if t_end is None else t_end
        stats = torch.empty(4, dtype=torch.int32, device=self.device)
        h_out = None
        if h_cap is None or h_cap > 0:
            h_out = self._f64(opts.max_attempts if h_cap is None else h_cap)
        ffb_diffusion(self.handle, rho, sigma, te, xy, opts, stats, h_out, replay_h,
                      self.lx, self.ly)
        return stats, h_out

    def inverse(self, nodes, queries, lx: int | None = None, ly: int | None = None):
        """Preimages of cartogram points under the piecewise-linear T given by
        the images of the nodes of an lx x ly grid: (triangle [Q] int32, -1
        outside; preimage [Q, 2] FP64, NaN outside)."""
        lx = self.lx if lx is None else lx
        ly = self.ly if ly is None else ly
        q = queries.reshape(-1, 2).contiguous()
        tri = torch.empty(q.shape[0], dtype=torch.int32, device=self.device)
        pre = torch.empty((q.shape[0], 2), dtype=torch.float64, device=self.device)
        ffb_inverse(self.handle, lx, ly, nodes.contiguous(), q, tri, pre)
        return tri, pre

    def graticule(self, nodes, spacing: float = 8.0, samples: int = 4, lx: int | None = None,
                  ly: int | None = None):
        """The graticule of the inverse transformation: the lines x = k
        spacing and y = k spacing of the cartogram box, sampled `samples`
        times per unit length, mapped back to the original map.  Returns
        (vertical, horizontal) preimage polylines as [lines, points, 2]
        FP64 tensors (NaN where a sample lies outside the node hull)."""
        lx = self.lx if lx is None else lx
        ly = self.ly if ly is None else ly
        xs = torch.arange(spacing, lx, spacing, dtype=torch.float64)
        ys = torch.arange(spacing, ly, spacing, dtype=torch.float64)
        tx = torch.linspace(0.0, float(lx), int(lx * samples) + 1, dtype=torch.float64)
        ty = torch.linspace(0.0, float(ly), int(ly * samples) + 1, dtype=torch.float64)
        vert = torch.stack(torch.broadcast_tensors(xs[:, None], ty[None, :]), -1)
        horz = torch.stack(torch.broadcast_tensors(tx[None, :], ys[:, None]), -1)
        q = torch.cat([vert.reshape(-1, 2), horz.reshape(-1, 2)]).to(torch.float32)
        _, pre = self.inverse(nodes, q.to(self.device), lx, ly)
        nv = vert.shape[0] * vert.shape[1]
        return pre[:nv].reshape(vert.shape), pre[nv:].reshape(horz.shape)

    def distortion(self, nodes, per_square: bool = False, lx: int | None = None,
                   ly: int | None = None):
        """Angular distortion of the map given by the images of the nodes of
        an lx x ly grid (default: the context's): (stats [5] = e_a, e_inf,
        e~_a, e~_inf, folded; per-square e; per-square e~)."""
        lx = self.lx if lx is None else lx
        ly = self.ly if ly is None else ly
        stats = self._f64(5)
        e = et = None
        if per_square:
            shape = (max(ly - 1, 0), max(lx - 1, 0))
            e = torch.empty(shape, dtype=torch.float32, device=self.device)
            et = torch.empty(shape, dtype=torch.float32, device=self.device)
        ffb_distortion(self.handle, lx, ly, nodes.contiguous(), stats, e, et)
        return stats, e, et

    # adjoints
    def _hold(self, geom):
        if self._recording and not any(g is geom for g in self._tape_refs):
            self._tape_refs.append(geom)

    def tape_begin(self, max_steps: int = 512):
        ffb_tape_begin(self.handle, max_steps)
        self._recording = True
        self._tape_refs = []

    def tape_end(self):
        ffb_tape_end(self.handle)
        self._recording = False

    def tape_clear(self):
        ffb_tape_clear(self.handle)
        self._recording = False
        self._tape_refs = []

    def tape_generation(self) -> int:
        return ffb_tape_generation(self.handle)

    def backward(self, dL_darea, n_vertices: int | None = None, generation: int | None = None):
        """Reverse pass over the recorded rounds: (dL/dvalue, dL/dxy0 or None).
        With ``generation`` (from tape_generation() after tape_begin) the
        call fails with FFB_E_NO_TAPE if the record was replaced since."""
        if generation is not None:
            ffb_tape_check(self.handle, generation)
        dval = torch.empty_like(dL_darea)
        dxy = None if n_vertices is None else self._f64(n_vertices, 2)
        ffb_backward(self.handle, dL_darea.contiguous(), dval, dxy)
        self._recording = False
        return dval, dxy


def default_sigma(k: int) -> float:
    """Blur width of round k (0-based), in grid cells: 4 * 2^-k."""
    return 4.0 * 2.0 ** (-k)


# The diffusion flow runs to t = infinity; it is cut where every
# non-constant mode has decayed by exp(-DIFFUSION_K) (the slowest decays as
# exp(-t / max(lx, ly)^2)).
DIFFUSION_K = 12.0


def diffusion_t_end(lx: int, ly: int, K: float = DIFFUSION_K) -> float:
    return K * float(max(lx, ly)) ** 2


@dataclass
class IterationResult:
    area_before: torch.Tensor
    rho: torch.Tensor
    rho_pad: torch.Tensor
    fields: torch.Tensor
    rho_bar: torch.Tensor
    stats: torch.Tensor
    h: torch.Tensor
    area_after: torch.Tensor
    err_after: torch.Tensor
    max_err_after: torch.Tensor


def iterate(ctx: Context, geom: Geometry, value, points, sigma: float,
            opts: IntegrateOpts | None = None, area_before=None) -> IterationResult:
    """One FFB iteration on the device: areas, density, flux, integration of
    ``points`` (whose first rows are the polygon vertices ``geom.xy``), areas
    and errors after.  Enqueue only; read results after ``ctx.sync()``."""
    if area_before is None:
        area_before, _, _ = ctx.area_error(geom, value)
    rho, pad = ctx.density(geom, value, area_before)
    fields, rho_bar = ctx.flux(rho, sigma)
    stats, h = ctx.integrate(fields, rho_bar, points, opts)
    area, err, mx = ctx.area_error(geom, value)
    return IterationResult(area_before, rho, pad, fields, rho_bar, stats, h, area, err, mx)


def iterate_diffusion(ctx: Context, geom: Geometry, value, points, sigma: float,
                      opts: IntegrateOpts | None = None, area_before=None,
                      t_end: float | None = None) -> IterationResult:
    """One round of the diffusion variant on the device: the same areas,
    density and blur as ``iterate``, then the diffusion flow to t_end.
    Waits for the integration (the number of steps is found on the device);
    ``fields`` and ``rho_bar`` of the result are None."""
    if area_before is None:
        area_before, _, _ = ctx.area_error(geom, value)
    rho, pad = ctx.density(geom, value, area_before)
    stats, h = ctx.diffusion(rho, sigma, points, t_end, opts)
    area, err, mx = ctx.area_error(geom, value)
    return IterationResult(area_before, rho, pad, None, None, stats, h, area, err, mx)


class FFBFunction(torch.autograd.Function):
    """K FFB rounds as a differentiable map value -> final region areas.

    forward(value, ctx, geom, points, sigmas, opts, max_steps, replay):
      on the device, recorded on the context's tape: one area call, then per
      sigma a round (density, flux, integration of ``points`` -- whose first
      rows are the vertices ``geom.xy``, advected in place -- and the areas
      after); returns the final areas [R] FP64.  ``replay`` (one FP64 device
      tensor of step sizes per round, or None) freezes the step schedules;
      otherwise the adaptive controller chooses them.
    backward: dL/dvalue by ffb_backward, with the forward's steps frozen.
    The context holds one record at a time: a later forward (or tape_begin)
    on the same context replaces it, and the backward of the earlier graph
    then raises FFBError(FFB_E_NO_TAPE) rather than differentiate the other
    forward."""

    @staticmethod
    def forward(fctx, value, ctx, geom, points, sigmas, opts=None, max_steps=512, replay=None):
        value = value.detach().contiguous()
        ctx.tape_begin(max_steps)
        fctx.generation = ctx.tape_generation()
        area, _, _ = ctx.area_error(geom, value)
        for k, sigma in enumerate(sigmas):
            rho, _ = ctx.density(geom, value, area)
            fields, rho_bar = ctx.flux(rho, sigma)
            ctx.integrate(fields, rho_bar, points, opts, h_cap=0,
                          replay_h=None if replay is None else replay[k])
            area, _, _ = ctx.area_error(geom, value)
        ctx.tape_end()
        fctx.ffb = ctx
        return area

    @staticmethod
    def backward(fctx, g_area):
        dval, _ = fctx.ffb.backward(g_area.detach().to(torch.float64).contiguous(),
                                    generation=fctx.generation)
        return dval, None, None, None, None, None, None, None


# ---------------------------------------------------------------- batches
@dataclass
class BatchOpts:
    stop_err: float = 0.01
    max_rounds: int = 30
    sigma0: float = 4.0
    integrate: IntegrateOpts | None = None
    use_graph: bool = True

    def struct(self) -> FFBBatchOpts:
        io = (self.integrate or IntegrateOpts()).struct()
        return FFBBatchOpts(self.stop_err, self.max_rounds, self.sigma0, io, int(self.use_graph))


class Batch:
    """Many maps iterated together on the device (ffb_batch_*).

    ``maps`` are objects with lx, ly, xy [V, 2], ring_offsets, ring_vidx,
    ring_region (per-map indices), n_regions and value; ``extra_points``
    optionally gives further points per map (e.g. its grid nodes), advected
    after its vertices.  The packed points live in ``self.points``."""

    def __init__(self, maps, extra_points=None, device="cuda", stream=None):
        import numpy as np
        M = len(maps)
        dev = torch.device(device)
        pts, voff, nvert, roff, goff = [], [0], [], [0], [0]
        offs, vidx, reg, vals = [0], [], [], []
        for k, m in enumerate(maps):
            p = np.asarray(m.xy, dtype=np.float32).reshape(-1, 2)
            extra = None if extra_points is None else extra_points[k]
            if extra is not None:
                p = np.concatenate([p, np.asarray(extra, dtype=np.float32).reshape(-1, 2)])
            base = voff[-1]
            pts.append(p)
            nvert.append(int(np.asarray(m.xy).reshape(-1, 2).shape[0]))
            o = np.asarray(m.ring_offsets, dtype=np.int64)
            offs.extend((o[1:] + offs[-1]).tolist())
            vidx.append(np.asarray(m.ring_vidx, dtype=np.int64) + base)
            reg.append(np.asarray(m.ring_region, dtype=np.int64) + roff[-1])
            vals.append(np.asarray(m.value, dtype=np.float64))
            voff.append(base + p.shape[0])
            roff.append(roff[-1] + int(m.n_regions))
            goff.append(goff[-1] + len(o) - 1)
        self.n_maps = M
        self.point_offsets = np.array(voff, dtype=np.int64)
        self.region_offsets = np.array(roff, dtype=np.int32)
        self.ring_offsets_map = np.array(goff, dtype=np.int32)
        self.n_vertices = np.array(nvert, dtype=np.int64)
        self.lx = np.array([m.lx for m in maps], dtype=np.int32)
        self.ly = np.array([m.ly for m in maps], dtype=np.int32)
        t32 = lambda a: torch.as_tensor(np.asarray(a, dtype=np.int32), device=dev).contiguous()
        self.points = torch.as_tensor(np.concatenate(pts), device=dev).contiguous()
        self.ring_offsets = t32(offs)
        self.ring_vidx = t32(np.concatenate(vidx))
        self.ring_region = t32(np.concatenate(reg))
        self.value = torch.as_tensor(np.concatenate(vals), device=dev).contiguous()
        self.n_regions = int(roff[-1])
        g = FFBGeometry(n_vertices=int(voff[-1]), xy=None, n_rings=int(goff[-1]),
                        ring_offsets=_ptr(self.ring_offsets, torch.int32),
                        ring_vidx=_ptr(self.ring_vidx, torch.int32),
                        ring_region=_ptr(self.ring_region, torch.int32),
                        n_regions=self.n_regions, n_entries=self.ring_vidx.numel())
        hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._host = (self.lx, self.ly, self.point_offsets, self.n_vertices,
                      self.ring_offsets_map, self.region_offsets)
        d = FFBBatchDesc(M, hp(self.lx), hp(self.ly), hp(self.point_offsets), hp(self.n_vertices),
                         hp(self.ring_offsets_map), hp(self.region_offsets), g,
                         _ptr(self.points, torch.float32), _ptr(self.value, torch.float64))
        h = ctypes.c_void_p()
        code = lib().ffb_batch_create(ctypes.byref(h), ctypes.byref(d), _stream_handle(stream))
        if code != FFB_OK:
            raise FFBError(code, "ffb_batch_create")
        self.handle = h
        _LIVE.add(self)

    def _check(self, code, what):
        if code != FFB_OK:
            raise FFBError(code, f"{what}: {lib().ffb_batch_last_error(self.handle).decode()}")

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib().ffb_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_shapes(self, fft_threads: int = 0, advect_threads: int = 0):
        self._check(lib().ffb_batch_set_shapes(self.handle, fft_threads, advect_threads),
                    "ffb_batch_set_shapes")

    def shapes(self):
        import numpy as np
        n = ctypes.c_int32()
        w = np.zeros(8, np.int32)
        f = np.zeros(8, np.int32)
        a = ctypes.c_int32()
        self._check(lib().ffb_batch_get_shapes(self.handle, ctypes.byref(n),
                                               w.ctypes.data_as(ctypes.c_void_p),
                                               f.ctypes.data_as(ctypes.c_void_p), ctypes.byref(a)),
                    "ffb_batch_get_shapes")
        return {"widths": w[:n.value].tolist(), "fft_threads": f[:n.value].tolist(),
                "advect_threads": a.value}

    def autotune(self, opts: BatchOpts | None = None):
        o = (opts or BatchOpts()).struct()
        self._check(lib().ffb_batch_autotune(self.handle, ctypes.byref(o)), "ffb_batch_autotune")
        return self.shapes()

    def reset(self):
        self._check(lib().ffb_batch_reset(self.handle), "ffb_batch_reset")

    def step(self, opts: BatchOpts | None = None, replay=None):
        """One round of every active map; ``replay`` = (offsets [M+1] int32,
        steps float64) device tensors of per-map accepted steps."""
        o = (opts or BatchOpts()).struct()
        ro, rh = (None, None) if replay is None else replay
        self._check(lib().ffb_batch_step(self.handle, ctypes.byref(o),
                                         _ptr(ro, torch.int32, name="replay_offsets"),
                                         _ptr(rh, torch.float64, name="replay_h")),
                    "ffb_batch_step")

    def run(self, opts: BatchOpts | None = None) -> int:
        o = (opts or BatchOpts()).struct()
        it = ctypes.c_int32()
        self._check(lib().ffb_batch_run(self.handle, ctypes.byref(o), ctypes.byref(it)),
                    "ffb_batch_run")
        return it.value

    def results(self):
        import numpy as np
        M = self.n_maps
        rounds = np.zeros(M, np.int32)
        mx = np.zeros(M, np.float64)
        stats = np.zeros((M, 4), np.int32)
        area = torch.empty(self.n_regions, dtype=torch.float64, device=self.points.device)
        self._check(lib().ffb_batch_results(self.handle, rounds.ctypes.data_as(ctypes.c_void_p),
                                            mx.ctypes.data_as(ctypes.c_void_p),
                                            stats.ctypes.data_as(ctypes.c_void_p),
                                            _ptr(area, torch.float64)), "ffb_batch_results")
        return rounds, mx, stats, area

    def map_points(self, m: int) -> torch.Tensor:
        return self.points[int(self.point_offsets[m]):int(self.point_offsets[m + 1])]
