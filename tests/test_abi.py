"""The C-ABI library: exports and host-side error paths (CPU, no kernel runs)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2508_04076_amd import cem, meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cem.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(cem_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(cem.LIB_PATH):
        from paper_2508_04076_amd import build
        build.build()
    return cem.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(cem.EXPORTS) == names


def _opts(**kw):
    o = dict(device=0, stream=None, precision=0, split_mode=0, gsig=0, max_splits=16, graph_steps=0)
    o.update(kw)
    return cem.cem_options(o["device"], o["stream"], o["precision"], o["split_mode"], o["gsig"],
                           o["max_splits"], o["graph_steps"])


def _create(lib, **kw):
    ctx = C.c_void_p()
    r = lib.cem_create(C.byref(_opts(**kw)), C.byref(ctx))
    return r, ctx


def test_create_validates_options(lib):
    for bad in [dict(precision=5), dict(split_mode=2), dict(gsig=7), dict(max_splits=-1),
                dict(graph_steps=-3), dict(device=-1)]:
        r, ctx = _create(lib, **bad)
        assert r == cem.CEM_EINVAL and not ctx.value
    r, ctx = _create(lib)
    assert r == cem.CEM_OK and ctx.value
    lib.cem_destroy(ctx)


def test_calls_out_of_order(lib):
    r, ctx = _create(lib)
    assert r == 0
    assert lib.cem_step(ctx, 1) == cem.CEM_ESTATE
    assert b"no mesh" in lib.cem_last_error(ctx)
    d = C.c_double()
    assert lib.cem_critical_dt(ctx, C.byref(d)) == cem.CEM_ESTATE
    assert lib.cem_set_dt(ctx, 1e-6) == cem.CEM_ESTATE
    e = cem.cem_energy()
    assert lib.cem_read_energy(ctx, C.byref(e)) == cem.CEM_ESTATE
    n = C.c_int32()
    assert lib.cem_read_splits(ctx, 0, None, C.byref(n)) == cem.CEM_ESTATE
    assert lib.cem_set_launch(ctx, 1024, 8, 0) == cem.CEM_ESTATE
    g, l, lay, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
    assert lib.cem_autotune(ctx, 5, C.byref(g), C.byref(l), C.byref(lay), C.byref(ms)) == cem.CEM_ESTATE
    assert lib.cem_set_precision(ctx, 1) == cem.CEM_ESTATE
    # graph size and the last-run record are host settings
    assert lib.cem_set_graph_steps(ctx, -1) == cem.CEM_EINVAL
    assert lib.cem_set_graph_steps(ctx, 25) == cem.CEM_OK
    run = np.ones(4, dtype=np.int64)
    assert lib.cem_last_run(ctx, run.ctypes.data_as(C.c_void_p)) == cem.CEM_OK
    assert run.tolist() == [0, 0, 0, 0]
    # the topology mode is a host setting: checked without a mesh or a device
    for bad in (-1, 3):
        assert lib.cem_set_topology_mode(ctx, bad) == cem.CEM_EINVAL
    for ok in (0, 1, 2):
        assert lib.cem_set_topology_mode(ctx, ok) == cem.CEM_OK
    lib.cem_destroy(ctx)


def _upload(lib, X, tets, mat=None):
    r, ctx = _create(lib)
    X = np.ascontiguousarray(X, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    m = cem.cem_material(**(mat or dict(E=32e9, nu=0.2, rho=2450.0, Gc=3.0)))
    r = lib.cem_upload_mesh(ctx, len(X), X.ctypes.data_as(C.c_void_p), len(tets),
                            tets.ctypes.data_as(C.c_void_p), C.byref(m))
    msg = lib.cem_last_error(ctx)
    lib.cem_destroy(ctx)
    return r, msg


def test_mesh_errors_found_on_the_host(lib):
    m = mg.kuhn_box(2, 2, 2)
    # degenerate tet: collapse one node onto another
    t = m.tets.copy()
    t[5, 1] = t[5, 0]
    assert _upload(lib, m.X, t)[0] == cem.CEM_EMESH
    # flat tet
    X = m.X.copy()
    t2 = np.vstack([m.tets, [[0, 1, 2, 2]]])
    assert _upload(lib, X, t2)[0] == cem.CEM_EMESH
    # duplicated tet
    t3 = np.vstack([m.tets, m.tets[:1]])
    r, msg = _upload(lib, m.X, t3)
    assert r == cem.CEM_EMESH
    # face shared by three tets: reflect a tet through one face twice
    X4 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0.3, 0.3, -1], [0.2, 0.2, -2]], float)
    t4 = np.array([[0, 1, 2, 3], [0, 2, 1, 4], [0, 2, 1, 5]])
    r, msg = _upload(lib, X4, t4)
    assert r == cem.CEM_EMESH and b"face" in msg
    # ids out of range
    t5 = m.tets.copy()
    t5[0, 0] = 10 ** 6
    assert _upload(lib, m.X, t5)[0] == cem.CEM_EMESH
    # empty inputs and a non-finite coordinate
    none = np.zeros((0, 4), np.int32)
    assert _upload(lib, m.X, none)[0] == cem.CEM_EINVAL
    assert _upload(lib, m.X[:3], m.tets[:0])[0] == cem.CEM_EINVAL
    X6 = m.X.copy()
    X6[3, 1] = np.nan
    r, msg = _upload(lib, X6, m.tets)
    assert r == cem.CEM_EINVAL and b"finite" in msg
    # bad material
    assert _upload(lib, m.X, m.tets, dict(E=-1.0, nu=0.2, rho=1.0, Gc=1.0))[0] == cem.CEM_EINVAL
    assert _upload(lib, m.X, m.tets, dict(E=1.0, nu=0.5, rho=1.0, Gc=1.0))[0] == cem.CEM_EINVAL


def test_hex_mesh_errors_found_on_the_host(lib):
    m = mg.hex_box(2, 2, 2)

    def up(X, h):
        r, ctx = _create(lib, max_splits=0)
        X = np.ascontiguousarray(X, dtype=np.float64)
        h = np.ascontiguousarray(h, dtype=np.int32)
        mat = cem.cem_material(E=32e9, nu=0.2, rho=2450.0, Gc=3.0)
        r = lib.cem_upload_hex_mesh(ctx, len(X), X.ctypes.data_as(C.c_void_p), len(h),
                                    h.ctypes.data_as(C.c_void_p), C.byref(mat))
        msg = lib.cem_last_error(ctx)
        lib.cem_destroy(ctx)
        return r, msg

    assert up(m.X, m.hexes[:0])[0] == cem.CEM_EINVAL
    h = m.hexes.copy()
    h[0, 0] = len(m.X)
    assert up(m.X, h)[0] == cem.CEM_EMESH
    # a degenerate hexahedron (two corners merged); a wholly inverted one is
    # mirrored, not refused
    h = m.hexes.copy()
    h[0, 6] = h[0, 0]
    r, msg = up(m.X, h)
    assert r == cem.CEM_EMESH and b"hexahedron" in msg


def test_valid_mesh_needs_a_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = mg.kuhn_box(2, 2, 2)
    r, msg = _upload(lib, m.X, m.tets)
    assert r == cem.CEM_EHIP


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(RuntimeError, match="missing"):
        cem._lib, saved = None, cem._lib
        try:
            cem.load_library(str(tmp_path / "nope.so"))
        finally:
            cem._lib = saved


def test_plain_c_caller_compiles_and_links(tmp_path):
    """include/cem.h is a C header: a C99 program (tests/c_abi/cube_force.c)
    compiles against it with -pedantic -Werror and links to libcem.so alone."""
    import importlib.util
    import subprocess
    here = os.path.join(ROOT, "tests", "c_abi", "build.py")
    spec = importlib.util.spec_from_file_location("c_abi_build", here)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = str(tmp_path / "cube_force")
    r = subprocess.run(mod.command(out), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    dyn = subprocess.run(["readelf", "-d", out], capture_output=True, text=True).stdout
    assert "[libcem.so]" in dyn and "libstdc++" not in dyn and "torch" not in dyn
