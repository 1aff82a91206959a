"""The C ABI library loads and exports what include/spmv.h declares (CPU only).

Only host-side entry points that touch no GPU are called here.
"""
import ctypes
import os
import re

import pytest

import paper_2302_05662_amd as S
from paper_2302_05662_amd import spmv as B


def test_every_declared_function_is_exported_and_bound():
    names = S.declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
        assert callable(getattr(B, n, None)), f"no Python wrapper named {n}"


def test_variant_catalogue():
    for fmt in range(6):
        for dt in (S.SPMV_F32, S.SPMV_F64):
            n = S.spmv_variant_count(fmt, dt)
            assert n >= 3
            kinds = {S.spmv_variant_describe(fmt, dt, i)["kernel"] for i in range(n)}
            want = {0: {"csr_scalar", "csr_vector", "csr_stream"},
                    1: {"coo", "coo_panel", "coo_sorted", "coo_split"}, 2: {"ell"}, 3: {"hyb"},
                    4: {"sell"}, 5: {"bell"}}[fmt]
            assert kinds == want
            with pytest.raises(S.SpmvError) as e:
                S.spmv_variant_describe(fmt, dt, n)
            assert e.value.status == "INVALID_ARG"
    assert S.spmv_variant_count(7, 0) == 0
    lanes = sorted({S.spmv_variant_describe(0, 0, i)["lanes"] for i in range(S.spmv_variant_count(0, 0))})
    assert lanes == [1, 2, 4, 8, 16, 32, 64]


def test_status_strings():
    assert S.spmv_status_string(0) == "ok"
    assert S.spmv_status_string(5) == "format not applicable"
    assert S.spmv_status_string(99) == "unknown status"


def test_header_defines_match_binding():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "spmv.h")).read()
    defines = dict(re.findall(r"#define\s+(SPMV_[A-Z0-9_]+)\s+(\d+)", text))
    assert defines, "no numeric defines found"
    for name, value in defines.items():
        assert getattr(S, name) == int(value), name
