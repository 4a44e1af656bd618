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


def test_static_scratch_refuses_an_input_beyond_its_size_before_device_work(built):
    """ttcf_pair_forces_static checks the size against its static scratch before any HIP call:
    here, with no GPU, an oversized input gets TTCF_ESCRATCH (a later check would report a
    device error instead)."""
    import ttcf_inputs as I
    s = I.System(10, density=0.7)  # 4000 atoms at 64 pairs per atom: 2^18 pair words
    sysd = built.make_system(s.n, s.box, s.temperature, s.dt, precision=1)
    lib = built.lib()
    assert lib.ttcf_pair_forces_static(sysd, 0.0, 0, 0.0, 64, None, None, None,
                                       None) == built.TTCF_EINVAL  # NULL buffers
    code = lib.ttcf_pair_forces_static(sysd, 0.0, 0, 0.0, 64, 1, 1, 1, None)
    assert code == built.TTCF_ESCRATCH
    assert b"static scratch" in lib.ttcf_strerror(code)


def _c_layout(struct: str, fields):
    """sizeof and offsetof of a struct of include/ttcf.h, from gcc."""
    import subprocess
    import tempfile
    lines = [f'printf("%zu\\n", sizeof({struct}));']
    lines += [f'printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"ttcf.h\"\nint main(void) {\n"
           + "\n".join(lines) + "\nreturn 0;\n}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("name,struct", [("System", "ttcf_system"), ("Shape", "ttcf_shape"),
                                         ("GraphDesc", "ttcf_graph_desc"),
                                         ("Channel", "ttcf_channel")])
def test_struct_layouts_match_header(built, name, struct):
    """Every ctypes mirror of a header struct has the C compiler's size and field offsets."""
    py = getattr(built, name)
    fields = [f[0] for f in py._fields_]
    size, offs = _c_layout(struct, fields)
    assert C_sizeof(py) == size
    assert [getattr(py, f).offset for f in fields] == offs


def C_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built library the binding raises (there is no CPU implementation to fall
    back on)."""
    from paper_2312_02990_amd import ttcf
    monkeypatch.setattr(ttcf, "_lib", None)
    monkeypatch.setattr(ttcf, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libttcf.so"))
    with pytest.raises(ImportError, match="no CPU implementation"):
        ttcf.lib()
