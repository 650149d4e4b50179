"""Topology modes through the C-ABI: one workgroup, whole chip and automatic
application of split batches give bitwise the same run, and the same run as
the oracle (forced schedule with batches of up to 400 splits in one step, so
the whole-chip path is taken).

Tolerances: bitwise between modes; FP64 state 1e-10 relative L2 and identical
split records against the oracle.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _schedule(mesh, seed=9):
    rng = np.random.default_rng(seed)
    free = np.setdiff1d(np.arange(mesh.n_tets), mesh.presplit_tets)
    sizes = [400, 300, 150, 100]
    tets = rng.choice(free, sum(sizes), replace=False)
    masks = rng.choice([1, 2, 4, 8, 3, 5, 6, 9, 10, 12], sum(sizes))
    steps = np.repeat([3, 6, 9, 12], sizes)
    return np.stack([steps, tets, masks], axis=1).astype(np.int32)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_topology_modes_agree_bitwise_and_with_the_oracle(precision):
    _case(f"topology modes, forced batches up to 400 splits, {precision}")
    from paper_2508_04076_amd.cem import CemError, Simulation
    mesh = mg.cube_notched(10)
    sched = _schedule(mesh)
    out = {}
    for mode in ("single", "chip", "auto"):
        sim = Simulation.from_mesh(mesh, MAT, precision=precision, max_splits=mesh.n_tets,
                                   graph_steps=5)
        sim.set_topology_mode(mode)
        dt = 0.5 * sim.critical_dt()
        sim.set_dt(dt)
        sim.replay_splits(sched)
        sim.step(20)
        u, v, a = sim.get_state()
        out[mode] = (u, v, sim.splits()[0], sim.energy())
        if mode == "auto":
            with pytest.raises(CemError):
                sim.set_topology_mode(3)
        sim.close()
    u0, v0, e0, en0 = out["single"]
    per_step = np.unique(e0[e0[:, 0] > 0][:, 0], return_counts=True)[1]
    assert per_step.max() == 400  # the whole-chip path was taken
    for mode in ("chip", "auto"):
        u, v, e, en = out[mode]
        assert np.array_equal(u, u0) and np.array_equal(v, v0) and np.array_equal(e, e0), mode
        for k in ("KE", "SE", "Wext", "Ud"):
            assert en[k] == en0[k], (mode, k)
    if precision == "fp64":
        orc = Oracle.from_mesh(mesh, MAT)
        orc.set_dt(dt)
        orc.replay(sched)
        orc.step(20)
        eo = orc.splits()[0]
        assert np.array_equal(e0[:, :3], eo[:, :3])
        assert _rel(u0, orc.get_state()[0]) < 1e-10


@pytest.mark.parametrize("mode", ["single", "chip"])
def test_split_batches_beyond_the_on_chip_sort(mode):
    """Batches of 3,000 and 2,100 splits in one step (above the 2,048 the
    one-workgroup rank sort holds on chip, so the topology pass sorts them in
    global memory) against the oracle."""
    _case(f"forced batches of 3000 and 2100 splits, topology mode {mode}")
    from paper_2508_04076_amd.cem import Simulation
    mesh = mg.cube_notched(12)
    rng = np.random.default_rng(12)
    free = np.setdiff1d(np.arange(mesh.n_tets), mesh.presplit_tets)
    sizes = [3000, 2100]
    tets = rng.choice(free, sum(sizes), replace=False)
    masks = rng.choice([1, 2, 4, 8, 3, 5, 6, 9, 10, 12], sum(sizes))
    sched = np.stack([np.repeat([2, 5], sizes), tets, masks], axis=1).astype(np.int32)
    sim = Simulation.from_mesh(mesh, MAT, max_splits=mesh.n_tets)
    sim.set_topology_mode(mode)
    dt = 0.5 * sim.critical_dt()
    sim.set_dt(dt)
    sim.replay_splits(sched)
    sim.step(8)
    eg = sim.splits()[0]
    per_step = np.unique(eg[eg[:, 0] > 0][:, 0], return_counts=True)[1]
    assert per_step.tolist() == sizes
    orc = Oracle.from_mesh(mesh, MAT)
    orc.set_dt(dt)
    orc.replay(sched)
    orc.step(8)
    eo = orc.splits()[0]
    assert np.array_equal(eg[:, :3], eo[:, :3])
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-10 and _rel(vg, vo) < 1e-10
    sim.close()
