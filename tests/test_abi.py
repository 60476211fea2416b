"""CPU checks of the C ABI: the library loads and exports every function declared in the header.
No compute call is made (there is no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdirac.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_solver_calls():
    names = declared_functions()
    for n in ("wd_gauge_create", "wd_gauge_destroy", "wd_apply", "wd_apply_dag", "bicgstab_solve",
              "bicgstab_m_solve", "wd_multimass_solve", "wd_batch_solve", "wd_gauge_grad"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import ctypes

    import paper_1103_5103_amd as wd

    if not os.path.exists(wd.LIBPATH):
        pytest.skip("libwdirac.so not built")
    L = ctypes.CDLL(wd.LIBPATH)
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(wd.EXPORTED) <= set(declared_functions())


def test_binding_loads_and_defaults():
    import paper_1103_5103_amd as wd

    if not os.path.exists(wd.LIBPATH):
        pytest.skip("libwdirac.so not built")
    p = wd.params()
    assert p.tol == 1e-8 and p.recon == 12 and p.eo == 1 and p.mixed == 1 and p.mixed_mode == wd.WD_MIXED_RELIABLE
    assert wd.params(defect_correction=True).mixed_mode == wd.WD_MIXED_DEFECT
    assert p.guess_order == 0 and wd.params(guess_order=3).guess_order == 3
    assert p.temporal_gauge == 0 and wd.params(temporal_gauge=True).temporal_gauge == 1
    assert p.gamma_basis == 0 and wd.params(nonchiral=True).gamma_basis == 1
    assert wd._lib.status_name(4) == "WD_ERR_NOCONV"
    v = wd.op_variant()
    assert (v.red, v.stage, v.nontemporal, v.tile, v.copies, v.rhs_per_thread, v.dagger) == (0, -1, -1, -1, 1, -1, 0)


def test_struct_layout_matches_c_compiler(tmp_path):
    """ctypes mirrors of the header structs have the sizes and offsets gcc gives them."""
    import ctypes
    import subprocess

    import paper_1103_5103_amd as wd

    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "wdirac.h"\n'
        "int main(void){"
        'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(wd_solver_params), offsetof(wd_solver_params, delta_reliable),'
        " offsetof(wd_solver_params, dagger), offsetof(wd_solver_params, gamma_basis), sizeof(wd_solver_stats),"
        " offsetof(wd_solver_stats, true_rel_res),"
        " sizeof(wd_system), sizeof(wd_geom), sizeof(wd_op_variant), offsetof(wd_op_variant, dagger)); return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(wd.SolverParams), wd.SolverParams.delta_reliable.offset, wd.SolverParams.dagger.offset,
            wd.SolverParams.gamma_basis.offset, ctypes.sizeof(wd.SolverStats), wd.SolverStats.true_rel_res.offset, ctypes.sizeof(wd._lib.System),
            ctypes.sizeof(wd._lib.Geom), ctypes.sizeof(wd.OpVariant), wd.OpVariant.dagger.offset]
    assert got == want
