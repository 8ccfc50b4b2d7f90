"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/feast.h
declares, and its host-only pieces (contour, argument validation) must
behave as documented.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import feast_oracle as O
from paper_0901_2665_amd import feast as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(feast_[a-z_0-9]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(F.LIB_PATH):
        pytest.fail("libfeast.so is not built; run __graft_entry__.build()")
    return F.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 10
    raw = ctypes.CDLL(F.LIB_PATH)
    for n in sorted(names):
        assert hasattr(raw, n), n
    assert names == set(F.EXPORTED)


def declared_arity():
    """Parameter count of every function prototype in include/*.h."""
    arity = {}
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            for name, params in re.findall(r"\b(feast_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
                params = params.strip()
                arity[name] = 0 if params in ("", "void") else params.count(",") + 1
    return arity


def test_binding_argtypes_match_header(lib):
    # every entry point the binding declares takes as many arguments as its
    # prototype (a parameter added to the header and not to the binding, or
    # the reverse, fails here rather than as a bad call on the GPU)
    arity = declared_arity()
    assert len(arity) >= 10
    checked = 0
    for name, n in sorted(arity.items()):
        argtypes = getattr(getattr(lib, name), "argtypes", None)
        if argtypes is None:
            continue
        assert len(argtypes) == n, (name, len(argtypes), n)
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("ne", [1, 4, 8, 16, 24])
def test_contour_matches_oracle(lib, ne):
    emin, emax = -3.2, -2.9
    x, w, Z, kappa = F.contour(ne, emin, emax)
    ct = O.contour(emin, emax, ne)
    assert np.max(np.abs(x - ct.x)) <= 1e-15
    assert np.max(np.abs(w - ct.w)) <= 2e-15
    assert np.max(np.abs(Z - ct.Z)) <= 1e-15 * max(abs(emin), abs(emax))
    assert np.max(np.abs(kappa - ct.kappa)) <= 1e-16 * 16


def test_contour_matches_printed_table(lib):
    tab = np.loadtxt(os.path.join(ROOT, "tests", "golden", "gauss_legendre_ne8.txt"))
    order = np.argsort(tab[:, 1])
    x, w, _, _ = F.contour(8, 0.0, 1.0)
    assert np.max(np.abs(x - tab[order, 1])) <= 1e-15
    assert np.max(np.abs(w - tab[order, 2])) <= 1e-15


def test_contour_argument_errors(lib):
    buf = [np.zeros(8) for _ in range(6)]
    ptrs = [b.ctypes.data for b in buf]
    assert lib.feast_contour(0, 0.0, 1.0, *ptrs) == -4
    assert lib.feast_contour(65, 0.0, 1.0, *ptrs) == -4
    assert lib.feast_contour(8, 1.0, 1.0, *ptrs) == -2
    assert lib.feast_contour(8, 0.0, float("inf"), *ptrs) == -2
    assert lib.feast_contour(8, 0.0, 1.0, None, *ptrs[1:]) == -5


def test_null_context_is_rejected(lib):
    ab = F.BTMatrix(2, 4, None, None, None, None)
    assert lib.feast_solve(None, ctypes.byref(ab), 0.0, 1.0, 4, 8, None, None, None,
                           None, None) == -5
    assert lib.feast_bt_multiply(None, ctypes.byref(ab), 0, 4, None, None) == -5
    assert lib.feast_destroy(None) == 0


def test_strerror_covers_codes(lib):
    for st in (0, -1, -2, -3, -4, -5, -6, -7, 1, 2, 3, 4, -101):
        assert lib.feast_strerror(st)


STRUCTS = [("feast_bt_matrix", F.BTMatrix), ("feast_opts", F.Opts), ("feast_info", F.Info),
           ("feast_problem", F.Problem), ("feast_zbt_matrix", F.ZBTMatrix)]
C_NAME = {"lam": "lambda"}  # C field names that are Python keywords


def test_struct_layouts_match_header(tmp_path):
    # the binding's ctypes structures against the C header, compiled by gcc:
    # same size and the same offset for every field
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "feast.h"',
             'int main(void) {']
    for cname, cls in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", '
                         f'offsetof({cname}, {C_NAME.get(fname, fname)}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True, timeout=60)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True,
                         timeout=30).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in STRUCTS:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    # the binding has no CPU path: without the built library it raises
    monkeypatch.setattr(F, "_lib", None)  # as in a fresh process
    with pytest.raises(RuntimeError, match="not built"):
        F.load_library(str(tmp_path / "libfeast.so"))
