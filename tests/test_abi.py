"""The C-ABI library loads (no GPU needed) and exports every function that
include/tls.h declares; the Python binding marshals exactly those."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tls.h")
LIB = os.path.join(ROOT, "paper_2401_03915_amd", "libtls.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tls_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2401_03915_amd import build
        build.build(verbose=False)
    from paper_2401_03915_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("tls_setup", "tls_apply", "tls_solve", "tls_info", "tls_destroy", "tls_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tls_[a-z_]+)\b", out))
    for name in _declared():
        assert name in exported, name
        assert hasattr(lib, name)


def test_binding_matches_header():
    from paper_2401_03915_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()


def test_struct_layouts_match_c():
    """Compile a tiny host program against tls.h and compare sizeof/offsets
    with the ctypes structures."""
    import ctypes
    from paper_2401_03915_amd import _lib
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "tls.h"
int main(void){
  printf("%zu %zu %zu %zu %zu\n", sizeof(tls_options), offsetof(tls_options, stream),
         offsetof(tls_options, seed), sizeof(tls_info_t), offsetof(tls_info_t, res_history));
  return 0; }
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    assert vals == [ctypes.sizeof(_lib.tls_options), _lib.tls_options.stream.offset, _lib.tls_options.seed.offset,
                    ctypes.sizeof(_lib.tls_info_t), _lib.tls_info_t.res_history.offset]


def test_setup_error_without_pointers(lib):
    """Argument validation happens before any device work."""
    import ctypes
    from paper_2401_03915_amd import _lib
    out = ctypes.c_void_p()
    st = lib.tls_setup(0, 0, None, None, None, None, 1, 1, 1, None, ctypes.byref(out))
    assert st == _lib.TLS_E_ARG and out.value is None
    assert "positive" in _lib.last_error(None)


def test_setup_rejects_nev1_for_general_matrices(lib):
    """eq. uppergevp vectors are defined for SPD A only: nev1 > 0 with
    matrix_kind = 1 is an argument error, raised before any device work
    (the host arrays below are never read)."""
    import ctypes

    import numpy as np
    from paper_2401_03915_amd import _lib
    opt = _lib.tls_options()
    lib.tls_default_options(ctypes.byref(opt))
    opt.matrix_kind = 1
    opt.nev1 = 2
    rp = np.array([0, 1, 2], dtype=np.int32)
    ci = np.array([0, 1], dtype=np.int32)
    val = np.ones(2)
    part = np.array([0, 1], dtype=np.int32)
    out = ctypes.c_void_p()
    st = lib.tls_setup(2, 2, rp.ctypes.data, ci.ctypes.data, val.ctypes.data, part.ctypes.data, 2, 1, 1,
                       ctypes.byref(opt), ctypes.byref(out))
    assert st == _lib.TLS_E_ARG and out.value is None
    assert "SPD" in _lib.last_error(None)
