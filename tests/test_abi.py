"""CPU-side checks of the C ABI: the library loads, exports every symbol declared in
include/ls.h, and validates arguments on the host (no GPU work is enqueued by these calls)."""
import ctypes as C
import os
import re

import pytest

from paper_1910_13844_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ls.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_A-Z]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert sorted(L.EXPORTS) == declared_symbols()


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libls.so not built")
    return L.load()


def test_all_symbols_exported(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def geom(**kw):
    g = dict(n=32, p=4, kbh=1.0469375, xg=32.0, prec=0)
    g.update(kw)
    return L.Geom(g["n"], g["p"], g["kbh"], g["xg"], g["prec"], 0)


def test_geometry_validation(lib):
    b = C.c_size_t()
    assert lib.ls_kernel_bytes(C.byref(geom()), C.byref(b)) == 0 and b.value > 0
    assert lib.ls_kernel_bytes(C.byref(geom(kbh=3.2)), C.byref(b)) == -1       # Nyquist: k h < pi
    assert lib.ls_kernel_bytes(C.byref(geom(p=3)), C.byref(b)) == -1           # p even
    assert lib.ls_kernel_bytes(C.byref(geom(n=31)), C.byref(b)) == -1          # n even
    assert lib.ls_kernel_bytes(C.byref(geom(xg=10.0)), C.byref(b)) == -1       # plane outside Omega
    assert lib.ls_kernel_bytes(C.byref(geom(n=48, xg=48.0)), C.byref(b)) == -3             # no kernels for n = 48
    assert lib.ls_kernel_bytes(C.byref(geom(n=512, prec=1, xg=512.0)), C.byref(b)) == -3   # nor for n = 512
    for n in (144, 192, 256):
        for prec in (0, 1):
            assert lib.ls_kernel_bytes(C.byref(geom(n=n, prec=prec, xg=float(n))), C.byref(b)) == 0
    assert lib.ls_kernel_bytes(None, C.byref(b)) == -1


def test_kernel_and_init_sizes(lib):
    b, w = C.c_size_t(), C.c_size_t()
    assert lib.ls_kernel_bytes(C.byref(geom(n=128, xg=128.0)), C.byref(b)) == 0
    M = 256
    assert b.value >= 129 * M * M * 8 + 129 * 128 * M * 8
    assert lib.ls_init_workspace_bytes(C.byref(geom(n=128, xg=128.0)), C.byref(w)) == 0
    assert w.value >= 2 * M ** 3 * 16


def test_null_context_rejected(lib):
    b = C.c_size_t()
    assert lib.ls_workspace_bytes(None, 4, 0, C.byref(b)) == -1
    assert lib.ls_forward(None, None, 1, None, None, None, None, None, 0, None) == -1
    assert lib.ls_forward_farfield(None, None, 1, None, None, None, None, None, None, 0, None) == -1
    assert lib.ls_forward_farfield_noalloc(None, None, 1, None, None, None, None, None, None) == -1
    assert lib.ls_residual(None, None, None, 1, 0, None, None, None, None) == -1
    assert lib.ls_strerror(-2).decode().startswith("workspace")


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes structures mirror include/ls.h: compile the header with the host C compiler and
    # compare sizes and field offsets
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "ls.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(ls_geom), offsetof(ls_geom, kbh), offsetof(ls_geom, xg), offsetof(ls_geom, prec));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(ls_solve_opts), offsetof(ls_solve_opts, maxit), offsetof(ls_solve_opts, max_restarts),
         offsetof(ls_solve_opts, x0_mode), offsetof(ls_solve_opts, breakdown));
  printf("%zu %zu %zu %zu\\n", sizeof(ls_solve_info), offsetof(ls_solve_info, relres_rec),
         offsetof(ls_solve_info, relres_true), offsetof(ls_solve_info, time_ms));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    g = [int(t) for t in lines[0].split()]
    o = [int(t) for t in lines[1].split()]
    i = [int(t) for t in lines[2].split()]
    assert g == [C.sizeof(L.Geom), L.Geom.kbh.offset, L.Geom.xg.offset, L.Geom.prec.offset]
    assert o == [C.sizeof(L.SolveOpts), L.SolveOpts.maxit.offset, L.SolveOpts.max_restarts.offset,
                 L.SolveOpts.x0_mode.offset, L.SolveOpts.breakdown.offset]
    assert i == [C.sizeof(L.SolveInfo), L.SolveInfo.relres_rec.offset, L.SolveInfo.relres_true.offset,
                 L.SolveInfo.time_ms.offset]
