"""The C-ABI from a plain C program (tests/c_abi/cube_force.c, built by
__graft_entry__.build()): no PyTorch and no Python binding in the process.
Its internal force, critical step and 40-step trajectory under a face traction
are checked against the oracle on a jittered 4 x 4 x 4 Kuhn cube.

Tolerances as the other parity tests: forces 1e-12 normwise, dt_crit 1e-12,
trajectory 1e-10 relative L2.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_abi", "cube_force")
MAT = dict(mg.BRANCHING_MATERIAL)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_plain_c_caller_matches_the_oracle(tmp_path):
    print("\n[case] plain C caller, jittered 4^3 cube, force + 40 steps", flush=True)
    if not os.path.exists(BIN):
        pytest.skip("tests/c_abi/cube_force is not built: run __graft_entry__.build()")
    m = mg.jitter(mg.kuhn_box(4, 4, 4), 0.2, seed=6)
    m.presplit_tets = None
    mg.add_tension(m, 2, 1e6)
    u = mg.random_displacement(len(m.X), 1e-6, seed=2)
    arrays = {"X.bin": (m.X, np.float64), "tets.bin": (m.tets, np.int32), "u.bin": (u, np.float64),
              "tri.bin": (m.load_tris, np.int32), "trac.bin": (m.load_trac, np.float64)}
    for name, (a, dt) in arrays.items():
        np.ascontiguousarray(a, dtype=dt).tofile(str(tmp_path / name))
    steps = 40
    args = [BIN, str(tmp_path), str(len(m.X)), str(len(m.tets)), str(len(m.load_tris)), str(steps),
            repr(MAT["E"]), repr(MAT["nu"]), repr(MAT["rho"])]
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    f = np.fromfile(str(tmp_path / "f.bin"), dtype=np.float64).reshape(-1, 3)
    us = np.fromfile(str(tmp_path / "us.bin"), dtype=np.float64).reshape(-1, 3)
    dtc = float(r.stdout.split()[1])

    orc = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    assert _rel(f, orc.internal_force(u)) < 1e-12
    assert abs(dtc / orc.critical_dt() - 1) < 1e-12
    orc.set_traction(m.load_tris, m.load_trac, 0.0)
    orc.set_dt(0.5 * dtc)
    orc.step(steps)
    assert _rel(us, orc.get_state()[0]) < 1e-10
