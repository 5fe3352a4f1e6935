"""ffb_flux_noalloc (the flux for callers that cannot allocate) against
ffb_flux, through the C ABI: two calls in a row on the same device, the
second on a smaller grid, each compared with the context entry point on the
same density.  Both run the same FP64 transform kernels, so the fields
agree to the rounding of the twiddle tables (device- vs host-computed)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1802_07625_amd as ffb
import synth
from gpu_util import to_np

pytestmark = pytest.mark.gpu


def _density(lx, ly, seed):
    # positive cell densities with the range of the benchmark maps
    rng = np.random.default_rng(seed)
    return 1.0 + 300.0 * rng.random((ly, lx)) ** 8


def _noalloc(lx, ly, rho, sigma):
    lib = ffb.lib()
    fields = torch.empty(((ly + 2) * (lx + 2) * 4,), dtype=torch.float32, device="cuda")
    rb = torch.empty(1, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = lib.ffb_flux_noalloc(lx, ly, rho.data_ptr(), sigma, fields.data_ptr(),
                                rb.data_ptr(), status.data_ptr(), stream)
    return code, fields, rb, status


def _with_ctx(lx, ly, rho, sigma):
    ctx = ffb.Context(lx, ly)
    fields, rb = ctx.flux(rho, sigma)
    assert ctx.sync(check=False) == 0
    ctx.close()
    return fields, rb


@pytest.mark.parametrize("shape", [((512, 512), (128, 64))])
def test_noalloc_flux_matches_context_flux(shape):
    for k, (lx, ly) in enumerate(shape):
        rho = torch.as_tensor(_density(lx, ly, 7 + k), device="cuda")
        sigma = 4.0 / (k + 1)
        print(f"[noalloc] call {k}: {lx}x{ly} sigma={sigma}", flush=True)
        code, f1, rb1, st = _noalloc(lx, ly, rho, sigma)
        assert code == 0
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        f0, rb0 = _with_ctx(lx, ly, rho, sigma)
        a, b = to_np(f1).reshape(-1, 4), to_np(f0).reshape(-1, 4)
        scale = np.abs(b[:, :3]).max(axis=0)
        err = (np.abs(a[:, :3] - b[:, :3]) / scale).max()
        print(f"[noalloc] {lx}x{ly} max field diff / scale = {err:.3e} "
              f"rho_bar {float(rb1):.15g} {float(rb0):.15g}", flush=True)
        assert err <= 1e-6
        assert float(rb1) == float(rb0)


def test_noalloc_flux_rejects_sizes():
    rho = torch.ones((1024, 1024), dtype=torch.float64, device="cuda")
    code, _, _, _ = _noalloc(1024, 1024, rho, 1.0)
    assert code == ffb.FFB_E_TOO_LARGE          # beyond the fixed workspace
    code, _, _, _ = _noalloc(96, 64, rho, 1.0)
    assert code == ffb.FFB_E_INVALID
