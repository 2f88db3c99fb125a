"""The C-ABI library loads and exports what include/sdc.h declares (CPU only).

Only host-side calls are made here (collocation data); everything that
touches the device is in the gpu-marked tests.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.collocation import Collocation


def _lib_path(root):
    return os.path.join(root, "paper_2311_07206_amd", "libsdc.so")


def _declared(root):
    names = set()
    for fn in os.listdir(os.path.join(root, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(root, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sdc_[a-z_]+)\s*\(", src))
    return names


@pytest.fixture(scope="module")
def lib(root):
    path = _lib_path(root)
    if not os.path.exists(path):
        pytest.skip("libsdc.so not built (run python -m paper_2311_07206_amd.build)")
    return ctypes.CDLL(path)


def test_header_declares_the_entry_points(root):
    names = _declared(root)
    for n in ("sdc_setup_mesh", "sdc_set_active", "sdc_sweep", "sdc_step", "sdc_create",
              "sdc_destroy", "sdc_last_error", "sdc_solve", "sdc_select", "sdc_collocation"):
        assert n in names


def test_library_exports_every_declared_symbol(lib, root):
    for name in sorted(_declared(root)):
        assert hasattr(lib, name), name


def test_binding_declares_every_symbol(root):
    from paper_2311_07206_amd import _lib
    assert _declared(root) == set(_lib.SIGNATURES)


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6])
def test_library_collocation_matches_oracle(lib, M):
    tau, Q, QI, QE = (np.zeros(M), np.zeros((M, M)), np.zeros((M, M)), np.zeros((M, M)))
    f = lib.sdc_collocation
    f.restype = ctypes.c_int32
    rc = f(ctypes.c_int32(M), *[a.ctypes.data_as(ctypes.c_void_p) for a in (tau, Q, QI, QE)])
    assert rc == 0
    c = Collocation(M)
    # both sides are pinned by quadrature exactness; the oracle's power-basis
    # integration loses about 1e-14 at M = 5, 6
    assert np.allclose(tau, c.tau, rtol=0, atol=2e-15)
    assert np.allclose(Q, c.Q, rtol=0, atol=3e-14)
    assert np.allclose(QI, c.QI, rtol=0, atol=3e-14)
    assert np.array_equal(QE != 0, c.QE != 0) and np.allclose(QE, c.QE, atol=2e-15)
    for d in range(2 * M - 1):     # end point row exact to degree 2M-2
        assert abs((Q @ tau ** d)[-1] - 1 / (d + 1)) < 1e-15


def test_library_collocation_rejects_bad_M(lib):
    f = lib.sdc_collocation
    f.restype = ctypes.c_int32
    assert f(ctypes.c_int32(0), None, None, None, None) != 0
    assert f(ctypes.c_int32(7), None, None, None, None) != 0


# C structures of the header and their ctypes mirrors in the binding
_STRUCTS = {"sdc_params": "Params", "sdc_sweep_stats": "SweepStats", "sdc_step_stats": "StepStats",
            "sdc_emi": "Emi", "sdc_profile_stats": "ProfileStats", "sdc_info": "Info"}


def test_binding_structures_match_the_header_layout(root, tmp_path):
    """Size and every field offset of each structure, as the C compiler lays
    them out from include/sdc.h, equal the binding's ctypes layout."""
    import shutil
    import subprocess
    from paper_2311_07206_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sdc.h"', "int main(void) {"]
    for cname, pyname in _STRUCTS.items():
        lines.append(f'  printf("{pyname} . %zu\\n", sizeof({cname}));')
        for field, _ in getattr(_lib, pyname)._fields_:
            lines.append(f'  printf("{pyname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    n_checked = 0
    for line in filter(None, out):
        pyname, field, value = line.split()
        cls = getattr(_lib, pyname)
        got = ctypes.sizeof(cls) if field == "." else getattr(cls, field).offset
        assert got == int(value), (pyname, field, got, value)
        n_checked += 1
    assert n_checked == sum(len(getattr(_lib, p)._fields_) + 1 for p in _STRUCTS.values())


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built HIP library the binding raises."""
    from paper_2311_07206_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libsdc.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


def test_product_package_does_not_import_the_oracle(root):
    import ast
    pkg = os.path.join(root, "paper_2311_07206_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            tree = ast.parse(open(os.path.join(pkg, fn)).read())
            for node in ast.walk(tree):
                names = [a.name for a in node.names] if isinstance(node, ast.Import) else \
                    [node.module or ""] if isinstance(node, ast.ImportFrom) else []
                assert not any(n.split(".")[0] == "oracle" for n in names), fn
