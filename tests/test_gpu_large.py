"""GPU checks at the large notched-block sizes, through the C-ABI.

The oracle cannot build meshes of this size in a test's time, so these are
properties that hold at any size: symmetry of the smoothed stiffness
(<K u, v> = <u, K v>), zero force under rigid-body motion, the linear patch
test (constant strain reproduced, no force away from boundaries and crack
faces), the fixed-point tiled force pass at its full tile size against the
term layout (1e-12 normwise), and mixed precision against FP64 within the
1e-5 relative L2 bound on u with the FP64 split schedule replayed.
"""
import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _sim(mesh, **kw):
    from paper_2508_04076_amd.cem import Simulation
    kw.setdefault("max_splits", len(mesh.presplit_tets) + mesh.n_tets // 16)
    return Simulation.from_mesh(mesh, MAT, ramp_t0=1e-6, **kw)


@pytest.fixture(scope="module")
def block8m():
    return mg.block_notched(220, 110, 55)


def test_block8m_symmetry_rigid_and_patch(block8m):
    _case("block 7,986,000 tets: symmetry, rigid modes, patch test")
    mesh = block8m
    sim = _sim(mesh, graph_steps=50)
    n = sim.n_nodes
    rng = np.random.default_rng(1)
    u = rng.standard_normal((n, 3)) * 1e-7
    v = rng.standard_normal((n, 3)) * 1e-7
    Ku, Kv = sim.internal_force(u), sim.internal_force(v)
    a, b = (Ku * v).sum(), (u * Kv).sum()
    assert abs(a - b) <= 1e-12 * np.sqrt((Ku * Ku).sum() * (v * v).sum())
    assert (u * Ku).sum() > 0
    # extra nodes of the pre-split copies sit on their twins: build the
    # coordinates of every node from the original node coordinates
    n0 = mesh.n_nodes
    X = np.zeros((n, 3))
    X[:n0] = mesh.X
    tets = mesh.tets[np.sort(mesh.presplit_tets)]
    X[n0:] = mesh.X[tets.reshape(-1)]  # extra node n0 + 4 s + l copies local node l of split s
    W = np.array([[0, -0.3, 0.2], [0.3, 0, -0.1], [-0.2, 0.1, 0]]) * 1e-6
    f = sim.internal_force(X @ W.T + 1e-6)
    assert np.abs(f).max() < 1e-9 * MAT["E"] * 1e-6 * 1e-6  # |f| ~ E strain area
    A = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.2, 0.0, 0.7]]) * 1e-5
    f = sim.internal_force(X @ A.T)
    lo, hi = mesh.X.min(0), mesh.X.max(0)
    free = np.ones(n, bool)
    free[n0:] = False
    free[np.unique(tets)] = False
    inner = np.all((mesh.X > lo + 1e-9) & (mesh.X < hi - 1e-9), axis=1)
    free[:n0] &= inner
    scale = np.abs(f).max()
    assert scale > 0 and np.abs(f[free]).max() < 1e-9 * scale
    sim.close()


def test_block8m_mixed_against_fp64(block8m):
    _case("block 7,986,000 tets: mixed vs FP64, 300 steps, schedule replayed")
    mesh = block8m
    s64 = _sim(mesh, graph_steps=50)
    dt = 0.5 * s64.critical_dt()
    s64.set_dt(dt)
    s64.step(300)
    u64 = s64.get_state()[0]
    ev = s64.splits()[0]
    s64.close()
    mx = _sim(mesh, graph_steps=50, precision="mixed")
    mx.set_dt(dt)
    dyn = ev[ev[:, 3] > 0][:, :3]
    if len(dyn):
        mx.replay_splits(dyn)
    mx.step(300)
    um = mx.get_state()[0]
    assert mx.counts()["splits"] == len(ev)
    err = np.linalg.norm(um - u64) / np.linalg.norm(u64)
    assert err < 1e-5, err
    mx.close()


def test_block48m_symmetry_and_mixed():
    # the 400 x 200 x 100-cell block (48,000,000 tets, 960,000 pre-split)
    _case("block 48,000,000 tets: symmetry; fixed-point tiles vs terms; mixed with fixed-point "
          "tiles vs FP64, 100 steps, schedule replayed")
    mesh = mg.block_notched()
    s64 = _sim(mesh, graph_steps=50)
    n = s64.n_nodes
    rng = np.random.default_rng(2)
    u = rng.standard_normal((n, 3)) * 1e-7
    v = rng.standard_normal((n, 3)) * 1e-7
    Ku, Kv = s64.internal_force(u), s64.internal_force(v)
    assert abs((Ku * v).sum() - (u * Kv).sum()) <= 1e-12 * np.sqrt((Ku * Ku).sum() * (v * v).sum())
    # the fixed-point tiles at their full size (8.1M nodes: 1,536-node tiles),
    # the bench's force pass, against the term layout
    s64.set_launch(8192, 4, "tiles_fx")
    Ku_fx = s64.internal_force(u)
    assert np.linalg.norm(Ku_fx - Ku) <= 1e-12 * np.linalg.norm(Ku)
    s64.set_launch(2048, 8, "terms")
    dt = 0.5 * s64.critical_dt()
    s64.set_dt(dt)
    s64.step(100)
    u64 = s64.get_state()[0]
    ev = s64.splits()[0]
    s64.close()
    mx = _sim(mesh, graph_steps=50, precision="mixed")
    mx.set_launch(8192, 4, "tiles_fx")
    mx.set_dt(dt)
    dyn = ev[ev[:, 3] > 0][:, :3]
    if len(dyn):
        mx.replay_splits(dyn)
    mx.step(100)
    err = np.linalg.norm(mx.get_state()[0] - u64) / np.linalg.norm(u64)
    assert err < 1e-5, err
    mx.close()
