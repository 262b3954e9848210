"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/dg.h is exported by libdg.so, and the ctypes mirror has the same
struct layout as the C header (sizes and offsets compiled with gcc)."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_2605_26388_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libdg.so not built")
    lib = ctypes.CDLL(_abi.LIB_PATH)
    names = declared_functions()
    assert set(names) == set(_abi.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_without_device():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libdg.so not built")
    lib = _abi.load()
    assert lib.dg_strerror(0) == b"ok"
    assert lib.dg_strerror(_abi.DG_ERR_ARG) == b"invalid argument"
    # argument errors are reported synchronously, before touching a device
    assert lib.dg_create(None, None) == _abi.DG_ERR_ARG
    assert b"null" in lib.dg_last_error()


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "dg.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(dg_mechanism), sizeof(dg_desc), sizeof(dg_counters));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(dg_desc, mech), offsetof(dg_desc, gamma),
         offsetof(dg_desc, newton_tol), offsetof(dg_desc, device), offsetof(dg_desc, patch_hi),
         offsetof(dg_desc, volume));
  printf("%zu %zu %zu\n", offsetof(dg_desc, rho_floor), offsetof(dg_desc, p_floor), offsetof(dg_counters, floored));
  printf("%zu %zu %zu %zu\n", offsetof(dg_desc, vib), sizeof(dg_vibration), offsetof(dg_vibration, park_sigma),
         offsetof(dg_vibration, two_temp));
  printf("%zu %zu %zu\n", offsetof(dg_desc, warp), offsetof(dg_desc, bc), offsetof(dg_desc, bc_state));
  printf("%zu %zu %zu\n", offsetof(dg_mechanism, nu_f), offsetof(dg_mechanism, eff),
         offsetof(dg_mechanism, kappa_r));
  printf("%zu\n", offsetof(dg_counters, first_bad));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    M, D, C = _abi.Mechanism, _abi.Desc, _abi.Counters
    expect = [ctypes.sizeof(M), ctypes.sizeof(D), ctypes.sizeof(C),
              D.mech.offset, D.gamma.offset, D.newton_tol.offset, D.device.offset, D.patch_hi.offset,
              D.volume.offset, D.rho_floor.offset, D.p_floor.offset, C.floored.offset,
              D.vib.offset, ctypes.sizeof(_abi.Vibration), _abi.Vibration.park_sigma.offset,
              _abi.Vibration.two_temp.offset, D.warp.offset, D.bc.offset, D.bc_state.offset, M.nu_f.offset, M.eff.offset, M.kappa_r.offset, C.first_bad.offset]
    assert vals == expect


def test_product_path_does_not_import_oracle():
    """The binding and the build never import the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2605_26388_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
