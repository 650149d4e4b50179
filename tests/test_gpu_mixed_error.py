"""Mixed precision (FP32 force arithmetic, FP64 state) against FP64 after a
whole run of the 768,000-tet notched plate: 20,000 steps (680 us), HIP
graphs.  With the FP64 run's split schedule replayed the displacement field
stays within 1e-5 relative L2 of the FP64 one; the free-running mixed run's
split events are compared with the FP64 ones and the difference is printed
(a different split changes the field, so L2 is not compared there).

The FP64 run itself follows the oracle's split events through 2,400 steps
(tests/test_gpu_plate_fracture.py)."""
import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)
STEPS = 20000


def _run(mesh, precision, dt, sched=None):
    from paper_2508_04076_amd.cem import Simulation
    s = Simulation.from_mesh(mesh, MAT, ramp_t0=1e-6, precision=precision,
                             max_splits=mesh.n_tets, graph_steps=50)
    s.set_dt(dt)
    if sched is not None:
        s.replay_splits(sched)
    for k in range(0, STEPS, 5000):
        s.step(5000)
        e = s.energy()
        print(f"  {precision}{' replay' if sched is not None else ''}: step {k + 5000}, "
              f"splits {e['n_split']}", flush=True)
    u = s.get_state()[0]
    ev = s.splits()[0]
    s.close()
    return u, ev


def test_plate_mixed_error_after_the_run():
    from paper_2508_04076_amd.cem import Simulation
    print(f"\n[case] plate 768k, {STEPS} steps FP64, then mixed with the FP64 split schedule "
          "replayed and free-running", flush=True)
    mesh = mg.plate_notched()
    probe = Simulation.from_mesh(mesh, MAT, max_splits=10000)
    dt = 0.5 * probe.critical_dt()
    probe.close()
    u64, ev64 = _run(mesh, "fp64", dt)
    dyn = ev64[ev64[:, 3] > 0]
    assert len(dyn) > 1000
    um, evm = _run(mesh, "mixed", dt, sched=dyn[:, :3])
    assert np.array_equal(evm[:, :3], ev64[:, :3])
    err = np.linalg.norm(um - u64) / np.linalg.norm(u64)
    print(f"  rel L2 of u after {STEPS} steps, schedule replayed: {err:.3e}", flush=True)
    assert err <= 1e-5
    uf, evf = _run(mesh, "mixed", dt)
    a = {tuple(r) for r in ev64[:, :3].tolist()}
    b = {tuple(r) for r in evf[:, :3].tolist()}
    first = min([r[0] for r in (a ^ b)], default=None)
    print(f"  free-running mixed: {len(b)} split events against {len(a)} in FP64, "
          f"{len(a - b)} only in FP64, {len(b - a)} only in mixed, first difference at step "
          f"{first}", flush=True)
