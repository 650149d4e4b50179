"""The oracle's optional threads partition elements, edges and nodes and keep
every sum in the serial order: a threaded run equals the one-thread run
bit for bit (states, split events, energies)."""
import numpy as np

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def _run(mesh, threads, steps, **kw):
    o = Oracle.from_mesh(mesh, MAT, **kw)
    o.set_threads(threads)
    o.set_dt(0.5 * o.critical_dt())
    o.step(steps)
    u, v, a = o.get_state()
    return u, v, a, o.splits(), o.energy()


def test_threads_bitwise_equal_through_splits():
    m = mg.cube_notched(6)
    ref = _run(m, 1, 150)
    assert len(ref[3][0]) > len(m.presplit_tets)  # dynamic splits happened
    for nt in (3, 8):
        got = _run(m, nt, 150)
        for x, y in zip(got[:3], ref[:3]):
            assert np.array_equal(x, y)
        assert np.array_equal(got[3][0], ref[3][0]) and np.array_equal(got[3][1], ref[3][1])
        assert got[4] == ref[4]


def test_threads_bitwise_equal_erosion_and_force():
    m = mg.plate_notched(20, 8, 2, 0.01, 0.004, 0.001, 0.005)
    ref = _run(m, 1, 60, split_mode="erode")
    got = _run(m, 5, 60, split_mode="erode")
    for x, y in zip(got[:3], ref[:3]):
        assert np.array_equal(x, y)
    o1, o4 = Oracle.from_mesh(m, MAT), Oracle.from_mesh(m, MAT)
    o4.set_threads(4)
    u = mg.random_displacement(o1.n_nodes, 1e-6, seed=4)
    assert np.array_equal(o1.internal_force(u), o4.internal_force(u))
