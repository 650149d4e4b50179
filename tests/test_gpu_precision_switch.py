"""Precision switch and graph size of an uploaded context, through the C-ABI.

- A context created in FP64 and switched to mixed before its first step runs
  bit for bit like one created mixed (same splits, same u).
- Switching mid-run keeps mesh, topology and state: the mixed continuation
  stays within the mixed tolerance (1e-5 relative L2 on u) of the FP64 one,
  and switching back and reloading the FP64 checkpoint reproduces the FP64
  run bit for bit.  A checkpoint loads only at the precision it was taken at.
- cem_set_graph_steps / cem_last_run: graph launches and plain remainders as
  requested, with the same bits as plain launches.
"""
import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _sim(mesh, **kw):
    from paper_2508_04076_amd.cem import Simulation
    return Simulation.from_mesh(mesh, MAT, ramp_t0=2e-5, max_splits=mesh.n_tets, **kw)


def test_switch_before_stepping_equals_created_mixed():
    print("\n[case] fp64 context switched to mixed vs created mixed, cube 6", flush=True)
    m = mg.cube_notched(6)
    a = _sim(m, precision="mixed")
    b = _sim(m, precision="fp64")
    dt = 0.5 * a.critical_dt()
    for s in (a, b):
        s.set_dt(dt)
    b.set_precision("mixed")
    a.step(300)
    b.step(300)
    ea, eb = a.splits()[0], b.splits()[0]
    assert len(ea) > len(m.presplit_tets)
    assert np.array_equal(ea, eb)
    assert np.array_equal(a.get_state()[0], b.get_state()[0])


def test_switch_mid_run_and_back():
    from paper_2508_04076_amd.cem import CemError
    print("\n[case] fp64 -> mixed -> fp64 mid-run, cube 6", flush=True)
    m = mg.cube_notched(6)
    s = _sim(m)
    dt = 0.5 * s.critical_dt()
    s.set_dt(dt)
    s.step(16)  # splits run from step 13 to 24
    ck = s.save_state()
    s.step(100)
    u64 = s.get_state()[0]
    ev64 = s.splits()[0]
    s.load_state(ck)
    s.set_precision("mixed")
    ckm = s.save_state()
    # the FP64 run's splits of these 100 steps, replayed
    late = ev64[(ev64[:, 0] > 16) & (ev64[:, 3] > 0)][:, :3]
    assert len(late) > 0
    s.replay_splits(late)
    s.step(100)
    um = s.get_state()[0]
    assert um.shape == u64.shape
    assert np.linalg.norm(um - u64) / np.linalg.norm(u64) < 1e-5
    with pytest.raises(CemError):
        s.load_state(ck)  # an FP64 checkpoint does not load at mixed precision
    s.load_state(ckm)
    s.set_precision("fp64")
    with pytest.raises(CemError):
        s.load_state(ckm)
    s.load_state(ck)
    s.step(100)
    assert np.array_equal(s.get_state()[0], u64)
    assert np.array_equal(s.splits()[0], ev64)


def test_graph_steps_and_last_run():
    print("\n[case] graph size and last-run record, cube 6", flush=True)
    m = mg.cube_notched(6)
    g = _sim(m)
    p = _sim(m)
    dt = 0.5 * g.critical_dt()
    for s in (g, p):
        s.set_dt(dt)
    g.set_graph_steps(50)
    g.step(120)
    assert g.last_run() == dict(steps=120, graph_launches=2, graph_steps=50, plain_steps=20)
    g.set_graph_steps(0)
    g.step(30)
    assert g.last_run() == dict(steps=30, graph_launches=0, graph_steps=0, plain_steps=30)
    g.set_graph_steps(25)
    g.step(10)  # fewer steps than a graph: plain launches
    assert g.last_run() == dict(steps=10, graph_launches=0, graph_steps=0, plain_steps=10)
    p.step(160)
    assert np.array_equal(g.get_state()[0], p.get_state()[0])
    assert np.array_equal(g.splits()[0], p.splits()[0])
