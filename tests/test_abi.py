"""The C-ABI library loads on the CPU and exports every entry point that
include/cpic.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cpic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(cpic_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_binding_surface():
    from paper_1311_2286_amd import cpic
    assert declared_functions() == sorted(cpic.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_1311_2286_amd import cpic
    if not os.path.exists(cpic.LIB_PATH):
        pytest.skip("libcpic.so not built")
    lib = ctypes.CDLL(cpic.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_argument_validation_without_gpu():
    from paper_1311_2286_amd import cpic
    if not os.path.exists(cpic.LIB_PATH):
        pytest.skip("libcpic.so not built")
    L = cpic.load()
    assert L.cpic_status_str(0) == b"ok"
    assert L.cpic_status_str(-2) == b"map not invertible on the domain"
    # descriptor validation happens before any HIP call
    h = ctypes.c_void_p()
    m = cpic.MapDesc(cpic.MAP_SINUSOIDAL, 2, (ctypes.c_double * 3)(1, 1, 1), 0.2, 1, 2)
    g = cpic.GridDesc()
    g.n[0] = g.n[1] = 16
    g.shape, g.precision, g.dt = cpic.SHAPE_B2, cpic.FP32, 0.1
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -2
    m.eps = 0.1
    g.dt = -1.0
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    g.dt = 0.1
    g.bc_lo[0] = cpic.BC_DIRICHLET  # mismatched periodicity
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    g.bc_hi[0] = cpic.BC_DIRICHLET  # walls on a non-orthogonal map
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -9
    m3 = cpic.MapDesc(cpic.MAP_SINUSOIDAL, 3, (ctypes.c_double * 3)(1, 1, 1), 0.14, 1, 2)
    g.bc_lo[0] = g.bc_hi[0] = 0
    g.n[2] = 8
    assert L.cpic_create(ctypes.byref(m3), ctypes.byref(g), None, None, ctypes.byref(h)) == -2
    # the spherical r-z map: 2D, 0 < r_in < r_out; Omega = x^1 needs a bounded
    # axis 0 and a map on which x^1 >= 0 (identity or spherical r-z)
    g.n[2] = 0
    sph = cpic.MapDesc(cpic.MAP_SPHERICAL_RZ, 2, (ctypes.c_double * 3)(1, 1, 1), 0.0, 2.0, 1.0, 1)
    assert L.cpic_create(ctypes.byref(sph), ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    sph.r_in, sph.r_out = 1.0, 10.0
    assert L.cpic_create(ctypes.byref(sph), ctypes.byref(g), None, None, ctypes.byref(h)) == -9  # periodic axis 0
    sph.omega = 2
    assert L.cpic_create(ctypes.byref(sph), ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    m.omega = 1
    g.bc_lo[0] = g.bc_hi[0] = cpic.BC_DIRICHLET
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -9  # sinusoidal
    # velocity step: unknown value; the cyclotronic step needs the Newton position update
    m.omega = 0
    g.bc_lo[0] = g.bc_hi[0] = cpic.BC_PERIODIC
    g.pusher = 7
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -1
    g.pusher = cpic.PUSH_CYCLOTRONIC
    g.mover = cpic.MOVER_PC
    assert L.cpic_create(ctypes.byref(m), ctypes.byref(g), None, None, ctypes.byref(h)) == -9
    # a tabulated map needs its vertex table
    g.pusher, g.mover = 0, 0
    tab = cpic.MapDesc(cpic.MAP_TABULATED, 2, (ctypes.c_double * 3)(1, 1, 1), 0.0, 1, 2, 0, None)
    assert L.cpic_create(ctypes.byref(tab), ctypes.byref(g), None, None, ctypes.byref(h)) == -1


def test_python_structures_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    that a C compiler gives the matching struct of include/cpic.h."""
    import shutil
    import subprocess
    from paper_1311_2286_amd import cpic
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("cpic_allocator", cpic.Allocator), ("cpic_map_desc", cpic.MapDesc),
             ("cpic_grid_desc", cpic.GridDesc), ("cpic_species_desc", cpic.SpeciesDesc),
             ("cpic_diag", cpic.Diag), ("cpic_case_desc", cpic.CaseDesc),
             ("cpic_case_result", cpic.CaseResult), ("cpic_server_stats", cpic.ServerStats)]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cpic.h"', "int main(void) {"]
    expect = []
    for cname, py in pairs:
        lines.append('  printf("%%zu\\n", sizeof(%s));' % cname)
        expect.append(ctypes.sizeof(py))
        for fname, _ in py._fields_:
            lines.append('  printf("%%zu\\n", offsetof(%s, %s));' % (cname, fname))
            expect.append(getattr(py, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect
