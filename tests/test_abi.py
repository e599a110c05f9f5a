"""The C-ABI library loads and exports every declared symbol; host-side
validation paths that need no GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "irlsu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irlsu_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2401_09961_amd as pkg
    if not os.path.exists(pkg.library_path()):
        pytest.fail("libirlsu.so is not built; run __graft_entry__.build()")
    return pkg.load_library()


def test_header_and_binding_agree():
    import paper_2401_09961_amd as pkg
    assert declared_functions() == sorted(pkg.DECLARED_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    import paper_2401_09961_amd as pkg
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (irlsu_[a-z_]+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_status_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        s = lib.irlsu_status_string(code).decode()
        assert s.startswith("IRLSU_")
    assert b"unknown" in lib.irlsu_status_string(42)


def test_params_default(lib):
    import paper_2401_09961_amd as pkg
    p = pkg.Params()
    assert lib.irlsu_params_default(ctypes.byref(p), 0) == 0
    assert p.eps == 1e-3 and p.pcg_rtol == 1e-8 and p.irls_iters == 20 and p.pcg_max == 100
    assert lib.irlsu_params_default(ctypes.byref(p), 2) == 0
    assert p.pcg_rtol == 1e-6 and p.flexible == -1 and p.true_res_every == 32
    assert lib.irlsu_params_default(ctypes.byref(p), 9) == -8
    assert lib.irlsu_params_default(None, 0) == -1


def test_host_validation_without_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.irlsu_plan_create(None, 8, 8, 1, None) == -1
    assert lib.irlsu_plan_create(ctypes.byref(h), 1, 8, 1, None) == -2
    assert lib.irlsu_plan_create(ctypes.byref(h), 8, 0, 1, None) == -2
    assert lib.irlsu_plan_create(ctypes.byref(h), 8, 8, 7, None) == -8
    assert lib.irlsu_plan_create(ctypes.byref(h), 32769, 8, 1, None) == -2
    # form: 0 auto, 1 dense, 2 folded (even sides), 3 fast (powers of two
    # >= 128, or each side a multiple of 8 whose half is at most 8192 and has
    # no prime factor above 5)
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 8, 8, 1, 4, None) == -1
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 112, 128, 1, 3, None) == -2   # 56 = 8 x 7
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 100, 128, 1, 3, None) == -2   # 100 % 8
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 128, 20000, 1, 3, None) == -2  # 10000 > 8192
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 8, 8, 1, -1, None) == -1
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 9, 8, 1, 2, None) == -2
    assert lib.irlsu_plan_create_ex(ctypes.byref(h), 8, 7, 1, 2, None) == -2
    assert h.value is None
    assert lib.irlsu_workspace_bytes(None) == 0
    assert lib.irlsu_plan_destroy(None) == 0
    assert lib.irlsu_unwrap(None, None, 0, None, None, 0, None, 0, None, None, None, 0,
                            None, 0, None, None) == -1
    assert lib.irlsu_operator(None, None, None, None, None, None, None, 0, None) == -1
    assert lib.irlsu_precond(None, None, None, None, None, 0, None) == -1


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of the header's structs, compiled by gcc, equal the
    ctypes mirrors used by the binding."""
    import paper_2401_09961_amd as pkg
    src = tmp_path / "sz.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "irlsu.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(irlsu_params), sizeof(irlsu_iter_stats),
         sizeof(irlsu_stats), sizeof(irlsu_plan_desc));
  printf("%zu %zu %zu %zu\\n", offsetof(irlsu_params, irls_iters), offsetof(irlsu_stats, iter),
         offsetof(irlsu_plan_desc, workspace_bytes), offsetof(irlsu_plan_desc, folded));
  return 0;
}
""")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    offs = [int(x) for x in lines[1].split()]
    assert sizes == [ctypes.sizeof(pkg.Params), ctypes.sizeof(pkg.IterStats),
                     ctypes.sizeof(pkg.Stats), ctypes.sizeof(pkg.PlanDesc)]
    assert offs == [pkg.Params.irls_iters.offset, pkg.Stats.iter.offset,
                    pkg.PlanDesc.workspace_bytes.offset, pkg.PlanDesc.folded.offset]
