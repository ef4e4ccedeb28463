"""The C-ABI library loads and exports every function include/mgr355.h declares; the
Python structs have the C layout (checked against the header compiled by the host
compiler).  No compute calls (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mgr355.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[\w\s\*]+?)\b(\w+)\s*\(", text, flags=re.M)
    return sorted({n for n in names if n.startswith(("mgr_", "fgmres_"))})


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mgr_setup", "mgr_setup_numeric", "mgr_apply", "fgmres_solve", "mgr_destroy",
                 "mgr_footprint", "mgr_estimate_footprint", "mgr_set_allocator",
                 "mgr_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1904_05960_amd import mgr355
    if not os.path.exists(mgr355.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(mgr355.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_c(tmp_path):
    from paper_1904_05960_amd import mgr355 as m
    src = tmp_path / "sz.c"
    src.write_text('#include "%s"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu %%zu'
                   ' %%zu\\n", sizeof(mgr_opts),'
                   'sizeof(mgr_level_opts), sizeof(mgr_amg_opts), sizeof(fgmres_opts),'
                   'sizeof(fgmres_result), sizeof(mgr_csr), offsetof(mgr_opts, precision),'
                   'sizeof(mgr_server_config), sizeof(mgr_request), sizeof(mgr_result),'
                   'offsetof(mgr_result, batch));}\n'
                   % HEADER)
    exe = tmp_path / "sz"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    exp = [ctypes.sizeof(m.mgr_opts), ctypes.sizeof(m.mgr_level_opts),
           ctypes.sizeof(m.mgr_amg_opts), ctypes.sizeof(m.fgmres_opts),
           ctypes.sizeof(m.fgmres_result), ctypes.sizeof(m.mgr_csr), m.mgr_opts.precision.offset,
           ctypes.sizeof(m.mgr_server_config), ctypes.sizeof(m.mgr_request),
           ctypes.sizeof(m.mgr_result), m.mgr_result.batch.offset]
    assert got == exp


def test_poro_struct_layouts_match_c(tmp_path):
    from paper_1904_05960_amd import mgr355 as m
    src = tmp_path / "sz2.c"
    src.write_text('#include "%s"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%%zu %%zu %%zu %%zu %%zu %%zu\\n",'
                   'sizeof(mgr_poro_params), offsetof(mgr_poro_params, dt),'
                   'sizeof(mgr_newton_opts), sizeof(mgr_newton_stats),'
                   'offsetof(mgr_newton_stats, merit), offsetof(mgr_newton_stats, solve_ms));}\n'
                   % HEADER)
    exe = tmp_path / "sz2"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    exp = [ctypes.sizeof(m.mgr_poro_params), m.mgr_poro_params.dt.offset,
           ctypes.sizeof(m.mgr_newton_opts), ctypes.sizeof(m.mgr_newton_stats),
           m.mgr_newton_stats.merit.offset, m.mgr_newton_stats.solve_ms.offset]
    assert got == exp


def test_poro_defaults_without_gpu():
    from paper_1904_05960_amd import mgr355 as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("library not built")
    L = m.lib()
    p = m.mgr_poro_params()
    L.mgr_poro_default_params(ctypes.byref(p), 4, 3, 2)
    assert (p.nx, p.ny, p.nz, p.reserved) == (4, 3, 2, 0)
    assert p.rho0[0] == 1000.0 and p.visc[1] == 5.0e-3 and p.dt == 86400.0
    o = m.mgr_newton_opts()
    L.mgr_newton_default_opts(ctypes.byref(o))
    assert o.max_newton == 12 and o.tol_flow == 1e-6 and o.max_ds == 0.2
    h = ctypes.c_void_p()
    assert L.mgr_poro_create(ctypes.byref(p), None, None, None, None, None, None, None, None,
                             ctypes.byref(h)) == m.MGR_ERR_ARG
    assert L.mgr_poro_set_dt(None, 1.0) == m.MGR_ERR_ARG


def test_default_options_and_errors_without_gpu():
    """Host-side argument checks return documented statuses without touching the device."""
    from paper_1904_05960_amd import mgr355 as m
    if not os.path.exists(m.LIB_PATH):
        pytest.skip("library not built")
    L = m.lib()
    o = m.mgr_opts()
    L.mgr_default_opts(ctypes.byref(o))
    assert o.use_graph == 1 and o.precision == 0 and o.coarse == 0
    assert o.level[0].frelax_sweeps == 1 and o.level[0].nmax_drop == -1
    h = ctypes.c_void_p()
    assert L.mgr_setup(None, None, ctypes.byref(o), None, ctypes.byref(h)) == m.MGR_ERR_ARG
    assert L.mgr_apply(None, None, None, None) == m.MGR_ERR_ARG
    assert b"null" in L.mgr_last_error()
    b = ctypes.c_size_t()
    assert L.mgr_estimate_footprint(1000, 50000, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value > 50000 * 12
    assert L.fgmres_workspace_bytes(1000, 30) >= 61 * 1000 * 8
