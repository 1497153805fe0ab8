"""The C-ABI library loads without a GPU, exports every entry point that
include/mbt.h declares, and rejects bad arguments on the host before any
device work."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from paper_2608_17844_amd import mbt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mbt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mbt.LIB_PATH):
        pytest.skip("libmbt.so not built")
    return mbt.lib()


def test_header_declares_the_binding_surface():
    assert set(_declared()) == set(mbt.exported_symbols())


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options_and_version(lib):
    o = mbt.mbt_default_opts()
    assert (o.prec, o.pc, o.restart, o.tol, o.max_cycles, o.refine_max) == (0, 1, 50, 1e-10, 400, 3)
    assert b"gfx950" in lib.mbt_version()


def test_null_and_invalid_arguments_rejected_on_host(lib):
    h = ctypes.c_void_p()
    d = mbt.mbt_dipole(0.5, 0.005, 15)
    l = mbt.mbt_lattice(5, 5, 0.5, 0.5)
    assert lib.mbt_array_create_dipole(None, ctypes.byref(d), ctypes.byref(l), ctypes.byref(h)) == mbt.MBT_EINVAL
    assert b"NULL" in lib.mbt_last_error()
    st = lib.mbt_port_admittance(None, None, 1.0, None, -1, None, None, None, None)
    assert st == mbt.MBT_EINVAL
    assert lib.mbt_footprint(None, 1, None) == 0
    assert lib.mbt_array_create_blocks(None, 2, 2, 3, None, ctypes.byref(h)) == mbt.MBT_EINVAL


def test_struct_layouts_match_header_sizes():
    assert ctypes.sizeof(mbt.mbt_dipole) == 24
    assert ctypes.sizeof(mbt.mbt_lattice) == 24
    assert ctypes.sizeof(mbt.mbt_solve_opts) == 56
    assert ctypes.sizeof(mbt.mbt_stats) == 72


STRUCTS = ["mbt_dipole", "mbt_lattice", "mbt_solve_opts", "mbt_stats", "mbt_predictors", "mbt_rwg_mesh",
           "mbt_request", "mbt_result"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_c99_and_binding_layouts_match_the_c_compiler(tmp_path):
    """The header compiles as strict C99, and every structure of the binding has
    the size and field offsets that the C compiler gives the header's."""
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "mbt.h"', 'int main(void) {']
    for name in STRUCTS:
        lines.append('    printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in getattr(mbt, name)._fields_:
            lines.append('    printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ['    return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name in STRUCTS:
        cls = getattr(mbt, name)
        assert int(got[name]) == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert int(got["%s.%s" % (name, field)]) == getattr(cls, field).offset, (name, field)


def test_binding_fails_loudly_without_the_library(monkeypatch):
    """No fallback: with the HIP library absent every entry point raises."""
    monkeypatch.setattr(mbt, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libmbt.so"))
    monkeypatch.setattr(mbt, "_lib", None)
    with pytest.raises(RuntimeError):
        mbt.lib()
    with pytest.raises(RuntimeError):
        mbt.mbt_ctx_create(0)
