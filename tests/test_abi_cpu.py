"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point the header declares, fills the paper's defaults, and
rejects invalid parameters before touching a device."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sphx.h")


@pytest.fixture(scope="module")
def sphx():
    from paper_2305_13380_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2305_13380_amd import sphx as mod
    return mod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(sphx_[a-z0-9_]+)\s*\(", text))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for must in ("sphx_ctx_create", "sphx_ctx_destroy", "sphx_workspace_bytes", "sphx_grid_build",
                 "sphx_tasks_build", "sphx_density", "sphx_ghost", "sphx_force", "sphx_step",
                 "sphx_grid_destroy", "sphx_tasks_destroy", "sphx_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(sphx):
    lib = C.CDLL(sphx.LIB_PATH)
    for name in sorted(declared_functions()):
        assert hasattr(lib, name), name
    assert declared_functions() <= set(sphx.SYMBOLS)


def test_default_params_are_the_papers(sphx):
    p = sphx.default_params()
    assert tuple(p.box) == (1.0, 1.0, 1.0) and p.periodic == 1
    assert p.h_tol == 1e-4 and p.beta_v == 3.0 and p.eps_balsara == 1e-4
    assert abs(p.gamma_gas - 5.0 / 3.0) < 1e-15
    assert abs(p.gamma_k - math.sqrt(15.0) / 2.0) < 1e-15
    assert p.eta == 1.2348 and p.leaf_max == 64 and p.max_iter == 30
    assert p.neighbour_lists == 0
    assert (p.density_tile, p.density_waves, p.force_tile, p.force_waves) == (0, 0, 0, 0)
    assert p.graph_passes == 0 and p.density_balance == 0


@pytest.mark.parametrize("field,value", [("eta", 0.0), ("h_tol", -1.0), ("max_iter", 0),
                                         ("leaf_max", 4), ("leaf_max", 65), ("gamma_k", 0.0),
                                         ("box", (1.0, 0.0, 1.0)), ("gamma_gas", 1.0),
                                         ("density_tile", 100), ("density_waves", 3),
                                         ("force_tile", 256), ("force_tile", 32), ("force_waves", -1),
                                         ("graph_passes", -1), ("graph_passes", 65),
                                         ("density_balance", 3)])
def test_ctx_create_rejects_invalid_params(sphx, field, value):
    p = sphx.default_params(**{field: value})
    h = C.c_void_p()
    st = sphx.lib.sphx_ctx_create(C.byref(p), 0, C.byref(h))
    assert st == sphx.E_INVALID
    assert sphx.last_error()
    assert not h.value


@pytest.mark.parametrize("extra", [{"density_balance": 1}, {"density_balance": 2},
                                   {"neighbour_lists": 1}, {"flavour": 6},
                                   {"flavour": "anarchy_pu", "density_balance": 2},
                                   {"flavour": "anarchy_pu", "neighbour_lists": 1}])
def test_ctx_create_rejects_loops_the_pressure_flavour_lacks(sphx, extra):
    kw = {"flavour": "pressure_energy"}
    kw.update(extra)
    p = sphx.default_params(**kw)
    h = C.c_void_p()
    assert sphx.lib.sphx_ctx_create(C.byref(p), 0, C.byref(h)) == sphx.E_INVALID
    assert sphx.last_error() and not h.value


def test_workspace_bytes_grows_with_n(sphx):
    p = sphx.default_params()
    a = sphx.lib.sphx_workspace_bytes(C.byref(p), 1000)
    b = sphx.lib.sphx_workspace_bytes(C.byref(p), 1_000_000)
    assert 0 < a < b
    assert b < 1_000_000 * 2000  # a few hundred bytes per particle
    assert sphx.lib.sphx_workspace_bytes(C.byref(p), -1) == 0


def test_null_arguments_are_errors(sphx):
    assert sphx.lib.sphx_ctx_create(None, 0, None) == sphx.E_INVALID
    assert sphx.lib.sphx_grid_build(None, None, None, None) == sphx.E_INVALID
    assert sphx.lib.sphx_step(None, None, None, None, None, None, None, None, None,
                              None) == sphx.E_INVALID


def test_one_hip_runtime_in_the_process(sphx):
    """Importing the binding alone leaves exactly one HIP runtime mapped (the
    one torch's streams and allocations belong to)."""
    import subprocess
    import sys
    code = ("from paper_2305_13380_amd import sphx\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(sorted(set(l.split()[-1] for l in maps if 'libamdhip64' in l)))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300, check=True).stdout.strip()
    import ast
    paths = ast.literal_eval(out)
    assert len(paths) == 1, paths


def test_kernel_setter_gives_each_kernels_gamma(sphx):
    import oracle
    assert sphx.default_params().kernel == 0
    for name, (kid, _) in oracle.KERNELS.items():
        p = sphx.default_params(kernel=name)
        assert p.kernel == kid == sphx.KERNELS[name]
        assert abs(p.gamma_k - oracle.kernel_gamma(name)) < 1e-15
    p = sphx.default_params()
    assert sphx.lib.sphx_params_set_kernel(C.byref(p), 6) == sphx.E_INVALID
    assert sphx.lib.sphx_params_set_kernel(C.byref(p), -1) == sphx.E_INVALID
    assert p.kernel == 0 and abs(p.gamma_k - math.sqrt(15.0) / 2.0) < 1e-15


@pytest.mark.parametrize("kernel", [-1, 6])
def test_ctx_create_rejects_unknown_kernel(sphx, kernel):
    p = sphx.default_params()
    p.kernel = kernel
    h = C.c_void_p()
    assert sphx.lib.sphx_ctx_create(C.byref(p), 0, C.byref(h)) == sphx.E_INVALID
    assert "kernel" in sphx.last_error() and not h.value


def test_grid_build_sets_rejects_null_arguments():
    """The set grid build refuses NULL handles and offsets before any device
    call (checked without a GPU)."""
    import ctypes as C
    from paper_2305_13380_amd import sphx
    h = C.c_void_p()
    pv = sphx.Particles()
    off = (C.c_int64 * 2)(0, 0)
    assert sphx.lib.sphx_grid_build_sets(None, C.byref(pv), off, 1, None, C.byref(h)) == \
        sphx.E_INVALID
    assert "NULL" in sphx.last_error()


def test_struct_layouts_match_the_header(sphx, tmp_path):
    """Every struct the binding passes through the C-ABI has the header's
    size and field offsets (a C program built from include/sphx.h prints
    them), so no call reads or writes past a Python-side struct."""
    import os
    import subprocess
    structs = {"sphx_params": sphx.Params, "sphx_particles": sphx.Particles,
               "sphx_density_out": sphx.DensityOut, "sphx_ghost_out": sphx.GhostOut,
               "sphx_force_out": sphx.ForceOut, "sphx_step_info": sphx.StepInfo}
    lines = ['#include <stdio.h>', '#include "sphx.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got["%s.%s" % (name, f[0])]) == getattr(cls, f[0]).offset, (name, f[0])
