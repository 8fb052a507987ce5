"""The C ABI: every function the header declares is exported by the built
library, and the binding's ctypes structures have the header's layout.  No
GPU needed (nothing here calls into the device)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trevr.h")
LIB = os.path.join(ROOT, "paper_1902_08083_amd", "libtrevr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trevr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("trevr_build_tree", "trevr_compute_flux", "trevr_compute_flux_adjoint"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    from paper_1902_08083_amd import trevr
    assert sorted(trevr.EXPORTED) == declared_functions()
    # status strings are host-only
    lib.trevr_status_string.restype = ctypes.c_char_p
    assert lib.trevr_status_string(0) == b"ok"
    assert lib.trevr_status_string(-2) == b"particle outside its box"


def test_struct_layouts_match_the_header(tmp_path):
    from paper_1902_08083_amd import trevr
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "trevr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(trevr_particles),
         offsetof(trevr_particles, prec), offsetof(trevr_particles, x),
         offsetof(trevr_particles, n_boxes), offsetof(trevr_particles, box_offsets),
         offsetof(trevr_particles, bucket_size), sizeof(trevr_launch));
  printf("%zu %zu %zu\n", sizeof(trevr_tree_info_t), offsetof(trevr_tree_info_t, prec),
         offsetof(trevr_tree_info_t, bucket_size));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    a = [int(v) for v in out[0].split()]
    b = [int(v) for v in out[1].split()]
    P = trevr._Particles
    assert a == [ctypes.sizeof(P), P.prec.offset, P.x.offset, P.n_boxes.offset,
                 P.box_offsets.offset, P.bucket_size.offset, ctypes.sizeof(trevr._Launch)]
    I = trevr._Info
    assert b == [ctypes.sizeof(I), I.prec.offset, I.bucket_size.offset]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1902_08083_amd import trevr
    monkeypatch.setattr(trevr, "_lib", None)
    monkeypatch.setattr(trevr, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(trevr.TrevrNotBuilt):
        trevr.Tree()
