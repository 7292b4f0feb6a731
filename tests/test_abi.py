"""The C-ABI library loads on the CPU and exports every symbol include/hisq.h declares."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2502_00152_amd import hisq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hisq_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(hisq.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(hisq.LIB_PATH):
        pytest.skip("libhisq.so not built")
    L = ctypes.CDLL(hisq.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_library_version_and_error_string_without_gpu():
    if not os.path.exists(hisq.LIB_PATH):
        pytest.skip("libhisq.so not built")
    L = hisq.lib()
    assert L.hisq_abi_version() == hisq.ABI_VERSION
    # argument checks run before any device call
    assert L.hisq_gauge_create(None, None, None, None, 1.0, 1.0, 0, None) == hisq.HISQ_ERR_INVALID_ARG
    assert b"null" in L.hisq_last_error()
    assert L.hisq_gauge_half_volume(None) == 0


def test_vector_bytes_matches_the_papers_storage_rule():
    """Section 3: V x N x 48 bytes in FP64 (more than 80 TB for 2048 vectors of
    144^3 x 288), halved by single parity (40 TB) and again by FP32 (20 TB)."""
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "eigvec_storage.txt"))
            if l.strip() and not l.startswith("#")]
    for lat, n, par, prec, tb, rel in rows:
        dims = [int(v) for v in lat.split("x")]
        p = {"fp64": hisq.HISQ_FP64, "fp32": hisq.HISQ_FP32}[prec]
        b = hisq.vector_bytes(dims, int(n), single_parity=(par == "single"), prec=p) / 1e12
        if rel == "more_than":
            assert float(tb) < b < 1.1 * float(tb)
        else:
            assert abs(b - float(tb)) / float(tb) < 0.1


STRUCTS = {
    "hisq_cg_params": hisq.CgParams,
    "hisq_cg_stats": hisq.CgStats,
    "hisq_eig_params": hisq.EigParams,
    "hisq_eig_stats": hisq.EigStats,
    "hisq_prop_params": hisq.PropParams,
    "hisq_prop_stats": hisq.PropStats,
    "hisq_tune_result": hisq.TuneResult,
    "hisq_system": hisq.System,
}


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets the
    C compiler gives the header's struct (a host C program prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "hisq.h"', "int main(void) {"]
    for cname, py in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    # the public header is plain C: it compiles without the HIP headers
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
