"""CPU checks of the C ABI boundary: the library loads and exports every
function include/ffb.h declares, the ctypes structs match the C layout
(compiled here with gcc), host-side validation rejects bad arguments before
any GPU work, and the product path and the oracle stay independent."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ffb.h")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ffb_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1802_07625_amd as ffb
    if not os.path.exists(ffb.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return ffb.lib()


def test_every_declared_function_is_exported(lib):
    names = header_functions()
    assert {"ffb_create", "ffb_area_error", "ffb_density", "ffb_flux", "ffb_integrate"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_1802_07625_amd",
                                                                     "libffb.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ffb_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_struct_layout_matches_c(tmp_path):
    import paper_1802_07625_amd.api as api
    src = tmp_path / "layout.c"
    src.write_text(f'''#include <stddef.h>
#include <stdio.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu\\n", sizeof(ffb_geometry), offsetof(ffb_geometry, n_rings),
         offsetof(ffb_geometry, ring_region), offsetof(ffb_geometry, n_regions),
         offsetof(ffb_geometry, n_entries));
  printf("%zu %zu %zu %zu\\n", sizeof(ffb_integrate_opts), offsetof(ffb_integrate_opts, max_attempts),
         offsetof(ffb_integrate_opts, n_replay), offsetof(ffb_integrate_opts, replay_h));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(ffb_batch_desc), offsetof(ffb_batch_desc, lx),
         offsetof(ffb_batch_desc, geometry), offsetof(ffb_batch_desc, points),
         offsetof(ffb_batch_desc, value));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(ffb_batch_opts), offsetof(ffb_batch_opts, max_rounds),
         offsetof(ffb_batch_opts, sigma0), offsetof(ffb_batch_opts, integrate),
         offsetof(ffb_batch_opts, use_graph));
  return 0;
}}''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    g = [int(v) for v in lines[0].split()]
    o = [int(v) for v in lines[1].split()]
    G, O = api.FFBGeometry, api.FFBIntegrateOpts
    assert g == [ctypes.sizeof(G), G.n_rings.offset, G.ring_region.offset, G.n_regions.offset,
                 G.n_entries.offset]
    assert o == [ctypes.sizeof(O), O.max_attempts.offset, O.n_replay.offset, O.replay_h.offset]
    bd = [int(v) for v in lines[2].split()]
    bo = [int(v) for v in lines[3].split()]
    D, BO = api.FFBBatchDesc, api.FFBBatchOpts
    assert bd == [ctypes.sizeof(D), D.lx.offset, D.geometry.offset, D.points.offset, D.value.offset]
    assert bo == [ctypes.sizeof(BO), BO.max_rounds.offset, BO.sigma0.offset, BO.integrate.offset,
                  BO.use_graph.offset]


def test_status_codes_match_header():
    import paper_1802_07625_amd.api as api
    txt = open(HEADER).read()
    codes = {n: int(v) for n, v in re.findall(r"(FFB_\w+)\s*=\s*(\d+)", txt)}
    for code, name in api.STATUS.items():
        assert codes[name] == code


def test_option_ids_match_header():
    import paper_1802_07625_amd.api as api
    txt = open(HEADER).read()
    ids = {n: int(v) for n, v in re.findall(r"(FFB_OPT_\w+)\s*=\s*(\d+)", txt)}
    assert ids == {"FFB_OPT_ADVECT_STATE": api.OPT_ADVECT_STATE,
                   "FFB_OPT_ADVECT_BLOCKS": api.OPT_ADVECT_BLOCKS,
                   "FFB_OPT_DIFFUSION_GRAPH": api.OPT_DIFFUSION_GRAPH,
                   "FFB_OPT_POINT_ORDER": api.OPT_POINT_ORDER}
    # the point-order values the header documents
    for v, name in ((0, "POINT_ORDER_GIVEN"), (1, "POINT_ORDER_AUTO"),
                    (2, "POINT_ORDER_ALWAYS"), (3, "POINT_ORDER_KEEP")):
        assert getattr(api, name) == v
        assert f"{v} = " in txt.split("FFB_OPT_POINT_ORDER:")[1].split("Returns FFB_E_INVALID")[0]


def test_host_validation_without_gpu(lib):
    ctx = ctypes.c_void_p()
    # grid sizes must be powers of two in [8, 1024]
    for lx, ly in ((7, 16), (16, 2048), (0, 16), (48, 64)):
        assert lib.ffb_create(ctypes.byref(ctx), lx, ly, 0, None) == 1
    assert lib.ffb_create(None, 16, 16, 0, None) == 1
    assert lib.ffb_sync(None) == 1
    assert lib.ffb_area_error(None, None, None, None, None, None) == 1
    assert lib.ffb_density(None, None, None, None, None, None) == 1
    assert lib.ffb_flux(None, None, ctypes.c_float(1.0), None, None) == 1
    assert lib.ffb_integrate(None, None, None, None, 0, None, None, None, 0) == 1
    assert lib.ffb_diffusion(None, None, ctypes.c_float(1.0), 1.0, None, 0, None, None, None,
                             0) == 1
    assert lib.ffb_diffusion_fields(None, None, ctypes.c_float(1.0), 0.0, None) == 1
    assert lib.ffb_distortion(None, 4, 4, None, None, None, None) == 1
    assert lib.ffb_inverse(None, 4, 4, None, None, 0, None, None) == 1
    assert lib.ffb_destroy(None) == 1
    g = ctypes.c_int64()
    assert lib.ffb_tape_generation(None, ctypes.byref(g)) == 1
    assert lib.ffb_tape_check(None, 0) == 1
    assert lib.ffb_last_error(None) == b"null context"
    # batches: descriptions are checked before any device work
    import paper_1802_07625_amd.api as api
    b = ctypes.c_void_p()
    assert lib.ffb_batch_create(ctypes.byref(b), None, None) == 1
    assert lib.ffb_batch_create(ctypes.byref(b), ctypes.byref(api.FFBBatchDesc()), None) == 1
    assert lib.ffb_batch_destroy(None) == 1
    assert lib.ffb_batch_run(None, None, None) == 1
    assert lib.ffb_batch_last_error(None) == b"null batch"


def test_product_and_oracle_are_independent():
    pkg = os.path.join(ROOT, "paper_1802_07625_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b|ffbo_", txt), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "import paper_1802_07625_amd" not in txt and "ffb.h" not in txt, f
