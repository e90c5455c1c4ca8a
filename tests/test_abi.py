"""The C ABI library loads on the CPU host, exports every symbol declared in
include/*.h, and rejects bad arguments before touching a device."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(dgo_[a-z_0-9]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def dgo():
    from paper_2602_12105_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(dgo):
    names = _declared()
    assert "dgo_mesh_create" in names and "dgo_pcg" in names
    missing = [n for n in sorted(names) if not hasattr(dgo, n)]
    assert not missing, missing


def test_version_and_error(dgo):
    assert dgo.dgo_version().startswith(b"dgo")
    assert dgo.dgo_last_error() == b""


def test_rejects_bad_arguments_without_device(dgo):
    from paper_2602_12105_amd._lib import Sizes
    h = C.c_void_p()
    assert dgo.dgo_mesh_create(5, 10, 1, C.c_void_p(8), None, None, C.byref(h)) == 1
    assert b"dim" in dgo.dgo_last_error()
    assert dgo.dgo_mesh_create(2, 0, 1, C.c_void_p(8), None, None, C.byref(h)) == 1
    assert dgo.dgo_mesh_create(2, 10, 5, None, None, None, C.byref(h)) == 1
    assert dgo.dgo_mesh_create(2, 10, 5, C.c_void_p(8), None, None, None) == 1
    assert dgo.dgo_mesh_sizes(None, C.byref(Sizes())) == 1
    assert dgo.dgo_assemble(None, 1, 1, None, None, None, None, None, None) == 1
    assert dgo.dgo_spmv(None, 1, 1, 1.0, None, 1.0, None, 1, None, None, None) == 1
    assert dgo.dgo_pcg(None, 1, 1.0, None, 1.0, None, None, None, 1, None, None, None, None,
                       None) == 1
    assert dgo.dgo_linear_solve_vjp(None, 1, 1.0, 1.0, 1, None, None, None, None, None,
                                    None) == 1
    assert b"NULL" in dgo.dgo_last_error()
    assert dgo.dgo_assemble_vjp(None, 1, 1, None, None, None, None, None) == 1
    assert dgo.dgo_assemble_intrinsic(None, 1, 1, None, None, None, None, None, None) == 1
    assert dgo.dgo_face_gradient(None, 1, None, 1, None, None, None) == 1
    assert b"NULL" in dgo.dgo_last_error()
    assert dgo.dgo_face_divergence(None, 1, None, 1, None, None, None) == 1
    assert dgo.dgo_mesh_coo(None, None, None, None) == 1
    assert dgo.dgo_mesh_slots(None, None, None) == 1
    assert dgo.dgo_eigs_smallest(None, 1, None, None, 1, None, None, None, None, None) == 1
    assert dgo.dgo_conformal_laplacian(None, 1, None, None, None, None, None) == 1
    dgo.dgo_mesh_destroy(None)


def test_python_binding_fails_loudly_when_library_missing(monkeypatch, tmp_path):
    from paper_2602_12105_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.lib()
