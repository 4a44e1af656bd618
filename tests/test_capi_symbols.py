"""Host-side checks of the C ABI library: it loads without a GPU and exports every function
that include/ttcf.h declares (no compute calls are made here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ttcf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ttcf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    from paper_2312_02990_amd import build
    build.build(force=False)
    from paper_2312_02990_amd import ttcf
    return ttcf


def test_every_declared_symbol_is_exported(built):
    lib = built.lib()
    names = _declared()
    assert "ttcf_init_mother" in names and "ttcf_response" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(built.EXPORTED) == sorted(n for n in names)


def test_strerror_and_argument_checks_without_device(built):
    lib = built.lib()
    assert lib.ttcf_strerror(0) == b"ok"
    assert lib.ttcf_strerror(-4) == b"call out of order"
    # NULL context / bad arguments are rejected before any device work
    assert lib.ttcf_step(None, 1) == built.TTCF_EINVAL
    assert lib.ttcf_accumulate(None, None) == built.TTCF_EINVAL
    lib.ttcf_destroy(None)


def test_system_struct_layout_matches_header(built):
    import ctypes as C
    # int32 n, int32 potential, double box[3], temperature, dt, r_cut, c_attr, u_shift,
    # nh_tau, int32 precision, int32 block_threads
    assert C.sizeof(built.System) == 4 + 4 + 24 + 6 * 8 + 4 + 4
