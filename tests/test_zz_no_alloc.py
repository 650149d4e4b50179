"""The allocation-free crack-front read (static device staging) against the
allocating one, through the C-ABI: the same records bit for bit on two calls
in a row on one GPU, the second with a smaller input (fewer fronts), then a
third on the first context again; more candidates than the staging holds
give CEM_ECAPACITY while the allocating read still works."""
import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _loaded(n, steps, **kw):
    from paper_2508_04076_amd.cem import Simulation
    m = mg.cube_notched(n)
    s = Simulation.from_mesh(m, MAT, max_splits=m.n_tets, **kw)
    s.set_dt(0.5 * s.critical_dt())
    s.step(steps)
    return s


def _same(s):
    t0, g0 = s.front_G()
    t1, g1 = s.front_G_static()
    assert len(t0) > 0
    assert np.array_equal(t0, t1)
    assert np.array_equal(g0, g1)
    return len(t0)


def test_static_front_read_matches_the_allocating_read():
    print("\n[case] static front read: cube 8 after 12 steps, then cube 4, then cube 8", flush=True)
    a = _loaded(8, 12)
    na = _same(a)
    b = _loaded(4, 6, precision="mixed")
    nb = _same(b)
    assert nb < na
    assert _same(a) == na
    # cap below the count: refused, nothing written
    from paper_2508_04076_amd.cem import CemError
    import ctypes as C
    from paper_2508_04076_amd.cem import cem_front_g
    n = C.c_int32()
    arr = (cem_front_g * 1)()
    r = a.lib.cem_read_front_G_static(a.ctx, 1, C.cast(arr, C.c_void_p), C.byref(n))
    assert r == -1 and n.value == na
    del CemError


def test_static_front_read_capacity():
    from paper_2508_04076_amd.cem import CemError, Simulation
    print("\n[case] static front read beyond its staging: 30^3-cell box, every 4th tet pre-split",
          flush=True)
    m = mg.kuhn_box(30, 30, 30)
    s = Simulation(m.X, m.tets, MAT, max_splits=m.n_tets)
    idx = np.arange(0, m.n_tets, 4, dtype=np.int32)
    s.presplit(idx, np.full(len(idx), 1, dtype=np.uint8))
    s.set_dt(0.5 * s.critical_dt())
    tfl, _ = s.front_G()
    assert len(np.unique(tfl[:, 0])) > 16384
    with pytest.raises(CemError) as ei:
        s.front_G_static()
    assert "CEM_ECAPACITY" in str(ei.value)
