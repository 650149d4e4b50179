"""The full 768k-tet plate in the launch shapes the benchmark times (the
stress-sum force layout at grids 4096 and 8192 with 8 lanes per node, and
whatever the library's autotuner picks), as captured HIP graphs, against the
CPU oracle over the first steps of the ramped load.

Tolerances as the other parity tests: FP64 1e-10 relative L2 on u and v and
identical split records; mixed precision 1e-5 relative L2 on u.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)
STEPS = 12


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def plate():
    mesh = mg.plate_notched()
    orc = Oracle.from_mesh(mesh, MAT, ramp_t0=1e-6)
    dt = 0.5 * orc.critical_dt()
    orc.set_dt(dt)
    orc.step(STEPS)
    u, v, _ = orc.get_state()
    return mesh, dt, u, v, orc.splits()[0]


@pytest.mark.parametrize("precision,launch", [
    ("fp64", (4096, 8, "stress_sums")),
    ("fp64", (8192, 8, "stress_sums")),
    ("fp64", "autotuned"),
    ("mixed", "autotuned"),
])
def test_plate_in_the_benchmark_launch(plate, precision, launch):
    _case(f"plate 768k, {precision}, launch {launch}, graphs of 6 steps")
    from paper_2508_04076_amd.cem import Simulation
    mesh, dt, uo, vo, eo = plate
    sim = Simulation.from_mesh(mesh, MAT, ramp_t0=1e-6, precision=precision,
                               max_splits=40000, graph_steps=6)
    sim.set_dt(dt)
    if launch == "autotuned":
        picked = sim.autotune(trial_steps=3)  # trials leave the state as it was
        print(f"[case] autotuned {picked}", flush=True)
        assert sim.energy()["step"] == 0
    else:
        sim.set_launch(*launch)
    sim.step(STEPS)
    ug, vg, _ = sim.get_state()
    eg = sim.splits()[0]
    if precision == "fp64":
        assert _rel(ug, uo) < 1e-10 and _rel(vg, vo) < 1e-10
        assert np.array_equal(eg[:, :3], eo[:, :3])
    else:
        assert _rel(ug, uo) < 1e-5
        assert np.array_equal(eg[:, :3], eo[:, :3])
    sim.close()
