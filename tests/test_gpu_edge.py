"""GPU edge cases against the oracle and closed forms, through the C-ABI.

The single-tet mesh (every edge patch is the one tet), a node that no element
holds (zero mass: zero acceleration, it keeps its velocity), momentum equal to
the load's trapezoidal impulse, zero steps, and zero displacement.
Tolerances: FP64 trajectories 1e-10 relative L2 against the oracle, momentum
1e-11 (FP64) and 1e-5 (mixed) of the impulse.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)
TRAC = np.array([2e5, -1e5, 1e6])


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _mesh(name):
    if name == "single_tet":
        X = np.array([[0, 0, 0], [1e-3, 0, 0], [0.2e-3, 1.1e-3, 0], [0.3e-3, 0.2e-3, 0.9e-3]])
        tri = np.array([[0, 1, 2]])
        area = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
        return X, np.array([[0, 1, 2, 3]]), tri, area
    m = mg.jitter(mg.kuhn_box(3, 3, 3, 1e-2, 1e-2, 1e-2), 0.2, seed=4)
    return m.X, m.tets, mg.face_triangles(m, 2, 1), 1e-4


def _ramp(t, t0):
    return 1.0 if t0 == 0 else min(t / t0, 1.0)


@pytest.mark.parametrize("name", ["single_tet", "jittered_box"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trajectory_and_momentum(name, precision):
    _case(f"{name} {precision}: trajectory and momentum")
    from paper_2508_04076_amd.cem import Simulation
    X, tets, tri, area = _mesh(name)
    sim = Simulation(X, tets, MAT, precision=precision, graph_steps=8)
    orc = Oracle(X, tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * orc.critical_dt()
    assert abs(sim.critical_dt() / orc.critical_dt() - 1) < 1e-12
    t0 = 20 * dt
    for o in (sim, orc):
        o.set_traction(tri, np.tile(TRAC, (len(tri), 1)), t0)
        o.set_dt(dt)
    n = 60
    sim.step(n)
    orc.step(n)
    us, vs, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert _rel(us, uo) < tol and _rel(vs, vo) < tol
    p = (orc.masses()[:, None] * vs).sum(0)
    impulse = dt * sum(0.5 * (_ramp(k * dt, t0) + _ramp((k + 1) * dt, t0)) for k in range(n))
    want = impulse * area * TRAC
    assert np.linalg.norm(p - want) < (1e-11 if precision == "fp64" else 1e-5) * np.linalg.norm(want)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_node_without_element(precision):
    _case(f"node without element {precision}")
    from paper_2508_04076_amd.cem import Simulation
    X, tets, tri, _ = _mesh("jittered_box")
    X2 = np.vstack([X, [[0.05, 0.05, 0.05]]])
    rng = np.random.default_rng(7)
    u0 = np.vstack([rng.standard_normal(X.shape) * 1e-7, np.zeros(3)])
    vx = np.array([1.0, -2.0, 0.5])
    v0 = np.vstack([rng.standard_normal(X.shape) * 1e-3, vx])
    sim = Simulation(X2, tets, MAT, precision=precision, graph_steps=8)
    orc = Oracle(X2, tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * orc.critical_dt()
    for o in (sim, orc):
        o.set_traction(tri, np.tile(TRAC, (len(tri), 1)), 10 * dt)
        o.set_dt(dt)
        o.set_state(u0, v0)
    n = 40
    sim.step(n)
    orc.step(n)
    us, vs, as_ = sim.get_state()
    uo, vo, _ = orc.get_state()
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert _rel(us, uo) < tol and _rel(vs, vo) < tol
    assert (vs[-1] == vx).all() and (as_[-1] == 0).all()
    assert np.allclose(us[-1], n * dt * vx, rtol=1e-13, atol=0)
    sim.close()


def test_zero_steps_and_zero_displacement():
    _case("zero steps, zero displacement")
    from paper_2508_04076_amd.cem import Simulation
    mesh = mg.cube_notched(4)
    sim = Simulation.from_mesh(mesh, MAT, max_splits=256)
    n = sim.n_nodes
    assert (sim.internal_force(np.zeros((n, 3))) == 0).all()
    sim.set_dt(0.5 * sim.critical_dt())
    sim.step(5)
    u1, v1, a1 = sim.get_state()
    e1 = sim.energy()
    sim.step(0)
    u2, v2, a2 = sim.get_state()
    assert (u1 == u2).all() and (v1 == v2).all() and (a1 == a2).all()
    assert sim.energy()["step"] == e1["step"] == 5
    sim.close()
