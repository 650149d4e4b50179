"""Pins of the oracle's prescribed-velocity (Dirichlet) boundaries and reactions.

The velocity history v0 * t/t0 up to t0, then v0, is the loading of the
paper's Dirichlet examples (Sections 4.1, 4.2, 4.3 and 4.5).  Pinned against
closed forms: a rigid translation (reaction = total mass x acceleration), the
impedance of a bar driven at one end (rho c A v0) and its doubling at a fixed
end, the static stiffness E A / L of a slowly stretched bar, and the energy
balance KE + SE = work of the reactions.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle, OracleError
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def _end_nodes(mesh, axis, side):
    x = mesh.X[:, axis]
    v = x.min() if side == 0 else x.max()
    return np.nonzero(np.abs(x - v) < 1e-12)[0].astype(np.int32)


def _x_only(nodes, v0x):
    vel = np.zeros((len(nodes), 3))
    vel[:, 0] = v0x
    return np.ones(len(nodes), np.int32), vel


def test_rigid_translation_reaction_is_total_mass_times_acceleration():
    m = mg.jitter(mg.kuhn_box(3, 3, 2), 0.2, seed=2)
    o = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    n = len(m.X)
    v0 = np.array([1.5, -0.5, 0.25])
    t0 = 50 * dt
    assert o.add_velocity_bc(np.arange(n), np.full(n, 7), np.tile(v0, (n, 1)), t0) == 0
    o.step(60)
    rows, work = o.reactions(0)
    M = o.masses().sum()
    assert rows.shape == (60, 6) and (rows[:, 0] == np.arange(1, 61)).all()
    for r in rows:
        t = r[1]
        ramp = t <= t0 * (1 + 1e-12)
        acc = 1.0 / t0 if ramp else 0.0
        S = t * t / (2 * t0) if ramp else t - t0 / 2
        assert np.allclose(r[2:5], M * v0 * acc, rtol=1e-9, atol=1e-9 * M / t0)
        assert abs(r[5] - S) <= 1e-15 * S
    u, v, _ = o.get_state()
    t = 60 * dt
    assert np.allclose(u, v0 * (t - t0 / 2), rtol=1e-12, atol=0)
    assert np.allclose(v, v0, rtol=1e-14, atol=0)
    # the work of the reactions is the kinetic energy gained, up to the
    # trapezoid's error at the kink of the velocity history: the acceleration
    # is taken on the ramp at t = t0, one extra half step
    KE = 0.5 * M * v0 @ v0
    assert abs(work / KE - 1 - dt / t0) < 1e-9
    assert abs(o.energy()["KE"] / KE - 1) < 1e-12


def _bar(n=100, lx=1.0, w=0.01):
    m = mg.bar(n, lx, w)
    o = Oracle(m.X, m.tets, MAT["E"], 0.0, MAT["rho"])  # nu = 0: 1D bar speed exact
    return m, o


def test_driven_bar_impedance_and_fixed_end_doubling():
    m, o = _bar()
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    left, right = _end_nodes(m, 0, 0), _end_nodes(m, 0, 1)
    v0 = 0.1
    gl = o.add_velocity_bc(left, *_x_only(left, v0), t0=20 * dt)
    gr = o.add_velocity_bc(right, *_x_only(right, 0.0), t0=0.0)
    c = np.sqrt(MAT["E"] / MAT["rho"])
    A = 0.01 * 0.01
    o.step(int(1.9 / c / dt))  # before the reflection returns to the driven end
    rl, _ = o.reactions(gl)
    rr, _ = o.reactions(gr)
    t = rl[:, 1]
    imp = MAT["rho"] * c * A * v0
    # the driven end pushes with rho c A v0; the fixed end holds nothing until
    # the wave arrives at L / c, then -2 rho c A v0 (reflection at a wall)
    assert abs(rl[(t > 0.2 / c) & (t < 1.8 / c), 2].mean() / imp - 1) < 0.02
    assert np.abs(rr[t < 0.8 / c, 2]).max() < 1e-6 * imp
    assert abs(rr[(t > 1.2 / c) & (t < 1.85 / c), 2].mean() / imp + 2) < 0.04


def test_slow_stretch_gives_static_stiffness():
    m, o = _bar(10, 0.1, 0.01)
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    left, right = _end_nodes(m, 0, 0), _end_nodes(m, 0, 1)
    c = np.sqrt(MAT["E"] / MAT["rho"])
    L, A = 0.1, 1e-4
    t0 = 40 * L / c
    v0 = 1e-3
    gl = o.add_velocity_bc(left, np.full(len(left), 7), np.zeros((len(left), 3)), t0)
    gr = o.add_velocity_bc(right, *_x_only(right, v0), t0=t0)
    o.step(int(1.5 * t0 / dt))
    rl, _ = o.reactions(gl)
    rr, wr = o.reactions(gr)
    late = rr[:, 1] > t0
    k = MAT["E"] * A / L
    u_end = v0 * rr[late, 5]
    # the constant-stress state of a uniaxial bar is exact in ES-FEM (patch
    # test), so the quasi-static reaction is E A / L times the stretch; the
    # slow ramp leaves an inertial ripple of a few per cent
    assert np.abs(rr[late, 2] / (k * u_end) - 1).max() < 0.05
    assert np.abs(rl[late, 2] / (k * u_end) + 1).max() < 0.05
    # the driven end's work is the stored energy plus the small kinetic energy
    e = o.energy()
    assert abs(e["SE"] + e["KE"] - wr) < 0.01 * wr


def test_reaction_work_balances_energy():
    m, o = _bar(40, 0.4, 0.01)
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    left = _end_nodes(m, 0, 0)
    o.add_velocity_bc(left, *_x_only(left, 0.2), t0=30 * dt)
    o.step(300)
    _, work = o.reactions(0)
    e = o.energy()
    # explicit central differences conserve energy to O(dt^2): within 1%
    assert abs(e["KE"] + e["SE"] - work) < 1e-2 * work
    assert e["Wext"] == 0.0


def test_bc_argument_checks():
    m = mg.kuhn_box(2, 2, 2)
    o = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o.set_dt(1e-6)
    with pytest.raises(OracleError):
        o.add_velocity_bc([0, 0], [1, 1], np.zeros((2, 3)))
    with pytest.raises(OracleError):
        o.add_velocity_bc([1], [8], np.zeros((1, 3)))
    o.add_velocity_bc([1], [1], np.zeros((1, 3)))
    with pytest.raises(OracleError):
        o.add_velocity_bc([1], [2], np.zeros((1, 3)))
    o.step(1)
    with pytest.raises(OracleError):
        o.add_velocity_bc([2], [1], np.zeros((1, 3)))
    with pytest.raises(OracleError):
        o.window_gradient(2)


def test_prescribed_velocity_is_the_rate_of_the_prescribed_displacement():
    # on the ramp the prescribed displacement is quadratic in t, so its central
    # difference over two steps is its derivative exactly: it must equal the
    # prescribed velocity at the middle step
    m = mg.jitter(mg.kuhn_box(3, 3, 2), 0.2, seed=4)
    o = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    n = len(m.X)
    v0 = np.array([0.8, -0.3, 0.5])
    o.add_velocity_bc(np.arange(n), np.full(n, 7), np.tile(v0, (n, 1)), 40 * dt)
    us, vs = [], []
    for _ in range(30):
        o.step(1)
        u, v, _ = o.get_state()
        us.append(u)
        vs.append(v)
    for k in range(1, 29):
        rate = (us[k + 1] - us[k - 1]) / (2 * dt)
        assert np.allclose(vs[k], rate, rtol=1e-9, atol=1e-12), k
    # and it ramps: at step k + 1 (time (k + 1) dt) the velocity is v0 (k + 1) / 40
    assert np.allclose(vs[9], v0 * 10 / 40, rtol=1e-12, atol=0)
