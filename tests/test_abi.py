"""Host-side checks of the C ABI (no GPU needed): the built library loads and exports every
function include/diffhydro.h declares, the ctypes structures match the C layouts, and the
build entry point compiles the HIP sources for gfx950."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffhydro.h")
LIB = os.path.join(ROOT, "paper_2502_02294_amd", "libdiffhydro.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dh_[a-z_0-9]+)\s*\(", text)))


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2502_02294_amd import build_lib
        build_lib.build(verbose=False)


def test_library_exports_every_declared_function():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2502_02294_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()


def test_struct_layouts_match_c(tmp_path):
    from paper_2502_02294_amd import _lib
    src = tmp_path / "layout.c"
    src.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dh_config), sizeof(dh_params),
         offsetof(dh_config, subgrid), offsetof(dh_config, sf_seed),
         offsetof(dh_config, ckpt_every), offsetof(dh_params, w_t),
         offsetof(dh_config, closure), sizeof(dh_mlp_train_opts),
         offsetof(dh_mlp_train_opts, lr), sizeof(dh_mlp_sample_opts),
         offsetof(dh_mlp_sample_opts, dc_hi), offsetof(dh_config, cfl_forward),
         offsetof(dh_config, kdk), offsetof(dh_config, star_dm),
         offsetof(dh_config, sn_smooth), offsetof(dh_config, lpt),
         offsetof(dh_config, transfer), offsetof(dh_config, dual_energy));
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    C, P, T, S = _lib.Config, _lib.Params, _lib.MlpTrainOpts, _lib.MlpSampleOpts
    want = [ctypes.sizeof(C), ctypes.sizeof(P), C.subgrid.offset, C.sf_seed.offset,
            C.ckpt_every.offset, P.w_t.offset, C.closure.offset, ctypes.sizeof(T), T.lr.offset,
            ctypes.sizeof(S), S.dc_hi.offset, C.cfl_forward.offset, C.kdk.offset,
            C.star_dm.offset, C.sn_smooth.offset, C.lpt.offset, C.transfer.offset,
            C.dual_energy.offset]
    assert got == want


def test_defaults_and_error_strings_without_gpu():
    _ensure_built()
    from paper_2502_02294_amd import _lib
    lib = _lib.lib()
    c = _lib.Config()
    lib.dh_config_default(ctypes.byref(c))
    assert (c.n, c.box, c.cfl, c.dlna_max, c.tau, c.ckpt_every) == (32, 10.0, 0.4, 0.04, 0.1, 16)
    assert abs(c.cfl_forward - 0.6) < 1e-15
    p = _lib.Params()
    lib.dh_params_default(ctypes.byref(p))
    assert (p.A, p.beta, p.eps_sf, p.delta_c) == (0.3, 1.6, 0.02, 100.0)
    assert lib.dh_strerror(-4) == b"non-finite or non-positive state"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    bad = _lib.Config()
    lib.dh_config_default(ctypes.byref(bad))
    bad.n = 48
    assert lib.dh_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad.n = 32
    bad.omega_b = 0.5
    assert lib.dh_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    bad.omega_b = 0.05
    bad.cfl_forward = -1.0
    assert lib.dh_create(ctypes.byref(bad), ctypes.byref(h)) == -1
    assert lib.dh_step(None, None, None) == -1


@pytest.mark.slow
def test_build_entry_compiles_for_gfx950():
    import __graft_entry__
    __graft_entry__.build()
    assert os.path.exists(LIB)
