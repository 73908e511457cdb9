"""CPU checks of the C-ABI library and its Python binding (no GPU calls).

The library must load, export every function include/mm.h declares, agree
with the binding on struct layouts, and reject bad parameters on the host.
The product package and the oracle must not import each other.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    import paper_1707_05333_amd as M
    lib = ctypes.CDLL(M.library_path())
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/mm.h but not exported"
    assert set(names) == set(M.SIGNATURES), "binding signatures differ from the header"


def test_struct_layouts_match_header(tmp_path):
    import paper_1707_05333_amd as M
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "mm.h"
int main(void) {
  printf("mm_params %zu %zu %zu %zu %zu %zu\n", sizeof(mm_params), offsetof(mm_params, gamma),
         offsetof(mm_params, precision), offsetof(mm_params, predictor_frame), offsetof(mm_params, half_step_mesh),
         offsetof(mm_params, mach_threshold));
  printf("mm_step_info %zu %zu %zu\n", sizeof(mm_step_info), offsetof(mm_step_info, floor_hits),
         offsetof(mm_step_info, flags));
  printf("mm_mesh_view %zu %zu\n", sizeof(mm_mesh_view), offsetof(mm_mesh_view, faces));
  printf("mm_sim_info %zu %zu %zu\n", sizeof(mm_sim_info), offsetof(mm_sim_info, floor_hits),
         offsetof(mm_sim_info, flags));
  printf("mm_request %zu %zu %zu %zu\n", sizeof(mm_request), offsetof(mm_request, params),
         offsetof(mm_request, steps), offsetof(mm_request, Q_out));
  printf("mm_request_result %zu %zu\n", sizeof(mm_request_result), offsetof(mm_request_result, t));
  printf("mm_serve_stats %zu %zu %zu\n", sizeof(mm_serve_stats), offsetof(mm_serve_stats, step_p99),
         offsetof(mm_serve_stats, max_resident));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = dict((l.split()[0], [int(x) for x in l.split()[1:]])
               for l in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    P, S, V = M.Params, M.StepInfo, M.MeshView
    assert out["mm_params"] == [ctypes.sizeof(P), P.gamma.offset, P.precision.offset, P.predictor_frame.offset,
                                P.half_step_mesh.offset, P.mach_threshold.offset]
    assert out["mm_step_info"] == [ctypes.sizeof(S), S.floor_hits.offset, S.flags.offset]
    assert out["mm_mesh_view"] == [ctypes.sizeof(V), V.faces.offset]
    I, R, RR, SS = M.SimInfo, M.Request, M.RequestResult, M.ServeStats
    assert out["mm_sim_info"] == [ctypes.sizeof(I), I.floor_hits.offset, I.flags.offset]
    assert out["mm_request"] == [ctypes.sizeof(R), R.params.offset, R.steps.offset, R.Q_out.offset]
    assert out["mm_request_result"] == [ctypes.sizeof(RR), RR.t.offset]
    assert out["mm_serve_stats"] == [ctypes.sizeof(SS), SS.step_p99.offset, SS.max_resident.offset]


def test_defaults_and_version():
    import paper_1707_05333_amd as M
    p = M.default_params()
    assert list(p.box) == [1.0, 1.0, 1.0]
    assert abs(p.gamma - 5 / 3) < 1e-15 and p.cfl == 0.3 and p.eta == 1.0 and p.chi == 1.0
    assert p.zeta == 0.25 and p.theta == 0.49 and p.limit_mask == 3 and p.predictor_frame == 0
    assert M.version().startswith("mm-mi355x")


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("cfl", 0.0), ("zeta", -1.0), ("rho_floor", 0.0),
                                         ("precision", 7), ("limit_mask", 4), ("predictor_frame", 2)])
def test_create_rejects_bad_parameters_on_host(field, value):
    import paper_1707_05333_amd as M
    lib = M.load_library()
    p = M.default_params()
    setattr(p, field, value)
    ctx = ctypes.c_void_p()
    rc = lib.mm_create(ctypes.byref(ctx), ctypes.byref(p), 100, 0, None)
    assert rc == -1 and not ctx.value
    assert lib.mm_last_error(None)


def test_create_rejects_bad_capacity_and_box():
    import paper_1707_05333_amd as M
    lib = M.load_library()
    ctx = ctypes.c_void_p()
    p = M.default_params()
    assert lib.mm_create(ctypes.byref(ctx), ctypes.byref(p), 0, 0, None) == -1
    assert lib.mm_create(ctypes.byref(ctx), ctypes.byref(p), 10, -1, None) == -1
    p.box[1] = float("nan")
    assert lib.mm_create(ctypes.byref(ctx), ctypes.byref(p), 10, 0, None) == -1


def test_calls_on_null_context_fail_cleanly():
    import paper_1707_05333_amd as M
    lib = M.load_library()
    assert lib.mm_tessellate(None, 10, None, None) == -1
    assert lib.mm_step(None, 10, None, None, None, 1.0, None) == -1
    assert lib.mm_destroy(None) == -1
    assert lib.mm_last_error(None) is not None


def test_batch_footprint_and_host_validation():
    import paper_1707_05333_amd as M
    lib = M.load_library()
    f64, mix = M.batch_footprint(1000, "fp64"), M.batch_footprint(1000, "mixed")
    assert f64 > mix > 0
    assert M.batch_footprint(2000, "mixed") - mix == mix - M.batch_footprint(0, "mixed")
    b = ctypes.c_void_p()
    assert lib.mm_batch_create(ctypes.byref(b), 7, 1 << 30, 8, None) == -1 and not b.value
    assert lib.mm_batch_create(ctypes.byref(b), M.MM_MIXED, 1 << 30, 0, None) == -1
    assert lib.mm_batch_create(ctypes.byref(b), M.MM_MIXED, 100, 8, None) == -1
    assert lib.mm_batch_last_error(None)
    for fn, args in [("mm_batch_step", (None, None, 0, None)), ("mm_batch_evict", (None, 0)),
                     ("mm_batch_read", (None, 0, None, None, None)), ("mm_batch_destroy", (None,)),
                     ("mm_serve", (None, None, 0, None, None))]:
        assert getattr(lib, fn)(*args) == -1


def test_make_params_validates_names():
    import paper_1707_05333_amd as M
    with pytest.raises(TypeError):
        M.make_params(box=(1, 1, 1), nonsense=1.0)
    p = M.make_params(box=(4, 1, 1), gamma=1.4, precision="mixed", theta=0.0, limit_mask=1)
    assert p.precision == M.MM_MIXED and p.theta == 0.0 and p.limit_mask == 1 and list(p.box) == [4, 1, 1]


def _imports(path):
    out = set()
    for dirpath, _, files in os.walk(path):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                out |= set(re.findall(r"^\s*(?:from|import)\s+([\w.]+)", text, flags=re.M))
                out |= set(re.findall(r'#include\s+"([^"]+)"', text))
    return out


def test_product_and_oracle_are_independent():
    prod = _imports(os.path.join(ROOT, "paper_1707_05333_amd"))
    orc = _imports(os.path.join(ROOT, "oracle"))
    assert not any(m.split(".")[0] == "oracle" for m in prod)
    assert not any("oracle" in m for m in prod if m.endswith(".h"))
    assert not any(m.split(".")[0] == "paper_1707_05333_amd" for m in orc)
    assert not any("mm_internal" in m or "mm.h" in m for m in orc)


def test_workloads_are_seeded_and_inside_the_box():
    import numpy as np
    import workloads as W
    a, b = W.c2_sod(shape=(16, 4, 4)), W.c2_sod(shape=(16, 4, 4))
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.prim, b.prim)
    for wl in (a, W.c1_uniform_random_velocity(n_side=5), W.c3_point_blast(n_side=8), W.c4_kelvin_helmholtz(3)):
        L = np.asarray(wl.box)
        assert np.all(wl.pos >= 0) and np.all(wl.pos < L)
        assert np.all(wl.prim[:, 0] > 0) and np.all(wl.prim[:, 4] > 0)
    hot = W.c3_point_blast(n_side=16)
    assert len(hot.energy_cells) == 32 and abs(hot.energy_amount * 32 - 1.0) < 1e-15


def test_static_step_validates_on_host():
    # The allocation-free step refuses bad arguments before touching a device.
    import ctypes
    import paper_1707_05333_amd as M
    L = M.load_library()
    info = M.StepInfo()
    assert L.mm_step_static(None, 10, None, None, None, 1.0, ctypes.byref(info), None) == -1
    p = M.make_params()
    assert L.mm_step_static(ctypes.byref(p), 0, None, None, None, 1.0, ctypes.byref(info), None) == -1
    assert b"MM_STATIC_MAX_POINTS" in L.mm_last_error(None)
    assert L.mm_step_static(ctypes.byref(p), M.STATIC_MAX_POINTS + 1, None, None, None, 1.0,
                            ctypes.byref(info), None) == -1
