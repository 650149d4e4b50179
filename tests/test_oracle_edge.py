"""Oracle pins on edge cases of the explicit step (Eqs. newmark_u to newmark_v,
lumped mass, face loads).

Pinned against: momentum balance under a one-sided face load (the element
forces sum to zero at every step, so the total momentum is the load's
trapezoidal impulse: it catches a load assembled twice or with a wrong area,
a mass missing from a node, or an internal force that does not balance); a
node that no element holds (it has no mass and no force: zero acceleration,
so it keeps its velocity, and nothing else changes); the single-tet mesh.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)
TRAC = np.array([2e5, -1e5, 1e6])


def _case(name):
    """(X, tets, loaded triangles, loaded area, volume) of a small test mesh."""
    if name == "single_tet":
        X = np.array([[0, 0, 0], [1e-3, 0, 0], [0.2e-3, 1.1e-3, 0], [0.3e-3, 0.2e-3, 0.9e-3]])
        tri = np.array([[0, 1, 2]])
        area = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0]))
        vol = abs(np.linalg.det(X[1:] - X[0])) / 6
        return X, np.array([[0, 1, 2, 3]]), tri, area, vol
    m = mg.jitter(mg.kuhn_box(3, 3, 3, 1e-2, 1e-2, 1e-2), 0.2, seed=4)
    return m.X, m.tets, mg.face_triangles(m, 2, 1), 1e-4, 1e-6  # jitter keeps the boundary


def _ramp(t, t0):
    return 1.0 if t0 == 0 else min(t / t0, 1.0)


@pytest.mark.parametrize("name", ["single_tet", "jittered_box"])
@pytest.mark.parametrize("ramp_steps", [0, 20])
def test_momentum_is_the_load_impulse(name, ramp_steps):
    X, tets, tri, area, vol = _case(name)
    o = Oracle(X, tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * o.critical_dt()
    t0 = ramp_steps * dt
    o.set_traction(tri, np.tile(TRAC, (len(tri), 1)), t0)
    o.set_dt(dt)
    n = 60
    o.step(n)
    _, v, _ = o.get_state()
    p = (o.masses()[:, None] * v).sum(0)
    impulse = dt * sum(0.5 * (_ramp(k * dt, t0) + _ramp((k + 1) * dt, t0)) for k in range(n))
    want = impulse * area * TRAC
    assert np.linalg.norm(p - want) < 1e-11 * np.linalg.norm(want)
    assert abs(o.masses().sum() / (MAT["rho"] * vol) - 1) < 1e-12


def test_node_without_element_keeps_its_velocity():
    X, tets, tri, _, _ = _case("jittered_box")
    X2 = np.vstack([X, [[0.05, 0.05, 0.05]]])
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal(X.shape) * 1e-7
    v0 = rng.standard_normal(X.shape) * 1e-3
    vx = np.array([1.0, -2.0, 0.5])
    oa = Oracle(X, tets, MAT["E"], MAT["nu"], MAT["rho"])
    ob = Oracle(X2, tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * oa.critical_dt()
    assert ob.critical_dt() == oa.critical_dt()
    for o in (oa, ob):
        o.set_traction(tri, np.tile(TRAC, (len(tri), 1)), 10 * dt)
        o.set_dt(dt)
    oa.set_state(u0, v0)
    ob.set_state(np.vstack([u0, np.zeros(3)]), np.vstack([v0, vx]))
    n = 40
    oa.step(n)
    ob.step(n)
    ua, va, _ = oa.get_state()
    ub, vb, ab = ob.get_state()
    assert ob.masses()[-1] == 0
    assert np.array_equal(ub[:-1], ua) and np.array_equal(vb[:-1], va)
    assert (vb[-1] == vx).all() and (ab[-1] == 0).all()
    assert np.allclose(ub[-1], n * dt * vx, rtol=1e-13, atol=0)
    ea, eb = oa.energy(), ob.energy()
    for k in ("KE", "SE", "Wext"):
        assert eb[k] == ea[k], k
