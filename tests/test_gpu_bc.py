"""GPU prescribed velocities (Dirichlet groups) and reaction histories against
the oracle, through the C-ABI.

Tolerances: FP64 states 1e-10 and reaction histories 1e-10 relative L2
(rounding order differs, nothing else); identical split events; mixed
precision 1e-5 on the reactions with the FP64 split schedule replayed.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _face(mesh, axis, side):
    x = mesh.X[:, axis]
    v = x.min() if side == 0 else x.max()
    return np.nonzero(np.abs(x - v) < 1e-12)[0].astype(np.int32)


def _pair(mesh, nu=None, **kw):
    from paper_2508_04076_amd.cem import Simulation
    mat = dict(MAT)
    if nu is not None:
        mat["nu"] = nu
    kw.setdefault("max_splits", max(mesh.n_tets // 4, 64))
    sim = Simulation.from_mesh(mesh, mat, traction=False, **kw)
    orc = Oracle.from_mesh(mesh, mat, traction=False)
    return sim, orc


def _both(sim, orc, fn, *a):
    ga = getattr(sim, fn)(*a)
    gb = getattr(orc, fn)(*a)
    return ga, gb


def test_rigid_translation():
    _case("prescribed rigid translation")
    mesh = mg.kuhn_box(4, 3, 2)
    mesh.X = mg.jitter(mesh, 0.2, seed=2).X
    mesh.presplit_tets = None
    sim, orc = _pair(mesh)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    n = len(mesh.X)
    v0 = np.tile([1.5, -0.5, 0.25], (n, 1))
    g = _both(sim, orc, "add_velocity_bc", np.arange(n), np.full(n, 7), v0, 30 * dt)
    assert g == (0, 0)
    sim.step(45)
    orc.step(45)
    (rs, ws), (ro, wo) = sim.reactions(0), orc.reactions(0)
    assert rs.shape == ro.shape == (45, 6)
    assert (rs[:, 0] == ro[:, 0]).all()
    assert _rel(rs, ro) < 1e-12 and abs(ws / wo - 1) < 1e-12
    assert _rel(sim.get_state()[0], orc.get_state()[0]) < 1e-12
    sim.close()


def test_driven_bar_two_groups():
    _case("bar driven at one end, fixed at the other")
    mesh = mg.bar(60, 0.6, 0.01)
    sim, orc = _pair(mesh, nu=0.0)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    left, right = _face(mesh, 0, 0), _face(mesh, 0, 1)
    vl = np.zeros((len(left), 3))
    vl[:, 0] = 0.1
    for o in (sim, orc):
        assert o.add_velocity_bc(left, np.ones(len(left)), vl, 20 * dt) == 0
        assert o.add_velocity_bc(right, np.full(len(right), 7), np.zeros((len(right), 3)), 0) == 1
    sim.step(400)
    orc.step(400)
    for g in (0, 1):
        (rs, ws), (ro, wo) = sim.reactions(g), orc.reactions(g)
        assert _rel(rs, ro) < 1e-10, (g, _rel(rs, ro))
        assert abs(ws - wo) <= 1e-10 * abs(wo) + 1e-30
    us, vs, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(us, uo) < 1e-10 and _rel(vs, vo) < 1e-10
    # impedance of the driven end (closed form rho c A v0, 1D bar speed)
    c = np.sqrt(MAT["E"] / MAT["rho"])
    rs = sim.reactions(0)[0]
    t = rs[:, 1]
    sel = (t > 0.1 / c) & (t < 1.0 / c)
    assert abs(rs[sel, 2].mean() / (MAT["rho"] * c * 1e-4 * 0.1) - 1) < 0.03
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_dirichlet_fracture_parity(precision):
    # notched cube pulled apart by a velocity on its top face with the bottom
    # face held in z: cracks grow from the notch under Dirichlet loading
    _case(f"dirichlet fracture {precision}")
    mesh = mg.cube_notched(6)
    sim, orc = _pair(mesh, precision=precision)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    top, bot = _face(mesh, 2, 1), _face(mesh, 2, 0)
    vt = np.zeros((len(top), 3))
    vt[:, 2] = 1.0
    for o in (sim, orc):
        o.add_velocity_bc(top, np.full(len(top), 4), vt, 20 * dt)
        o.add_velocity_bc(bot, np.full(len(bot), 4), np.zeros((len(bot), 3)), 0.0)
    steps = 250
    if precision == "fp64":
        sim.step(steps)
        orc.step(steps)
        ev_s, ev_o = sim.splits()[0], orc.splits()[0]
        assert len(ev_o) > len(mesh.presplit_tets), "the case must split"
        assert (ev_s[:, :3] == ev_o[:, :3]).all()
        assert _rel(sim.get_state()[0], orc.get_state()[0]) < 1e-10
        for g in (0, 1):
            assert _rel(sim.reactions(g)[0], orc.reactions(g)[0]) < 1e-10
    else:
        orc.step(steps)
        ev_o = orc.splits()[0]
        dyn = ev_o[len(mesh.presplit_tets):]
        sim.replay_splits(dyn[:, :3])
        sim.step(steps)
        for g in (0, 1):
            assert _rel(sim.reactions(g)[0], orc.reactions(g)[0]) < 1e-5
    sim.close()


def test_bc_refusals_and_checkpoint():
    _case("prescribed velocity refusals and checkpoint")
    from paper_2508_04076_amd.cem import CemError
    mesh = mg.cube_notched(5)
    sim, _ = _pair(mesh)
    sim.set_dt(5e-6)
    top = _face(mesh, 2, 1)
    vt = np.zeros((len(top), 3))
    vt[:, 2] = 0.5
    with pytest.raises(CemError):
        sim.add_velocity_bc(top, np.full(len(top), 8), vt)
    with pytest.raises(CemError):
        sim.add_velocity_bc(np.concatenate([top, top[:1]]), np.full(len(top) + 1, 4),
                            np.vstack([vt, vt[:1]]))
    sim.add_velocity_bc(top, np.full(len(top), 4), vt, 1e-5)
    with pytest.raises(CemError):
        sim.add_velocity_bc(top[:1], [1], vt[:1])
    with pytest.raises(CemError):
        sim.window_forward(4, 2)
    sim.step(10)
    buf = sim.save_state()
    sim.step(15)
    r1, w1 = sim.reactions(0)
    u1 = sim.get_state()[0]
    sim.load_state(buf)
    sim.step(15)
    r2, w2 = sim.reactions(0)
    assert (r1 == r2).all() and w1 == w2 and (sim.get_state()[0] == u1).all()
    with pytest.raises(CemError):
        sim.add_velocity_bc(top[:1], [1], vt[:1])
    sim.close()


def test_dirichlet_plate_mid_size():
    _case("dirichlet plate 40x16x2")
    mesh = mg.plate_notched(40, 16, 2, 0.01, 0.004, 0.0005, 0.005)
    sim, orc = _pair(mesh, graph_steps=10)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    top, bot = _face(mesh, 1, 1), _face(mesh, 1, 0)
    vt = np.zeros((len(top), 3))
    vt[:, 1] = 3.318
    for o in (sim, orc):
        o.add_velocity_bc(top, np.full(len(top), 2), vt, 40 * dt)
        o.add_velocity_bc(bot, np.full(len(bot), 7), np.zeros((len(bot), 3)), 0.0)
    sim.step(120)
    orc.step(120)
    assert (sim.splits()[0][:, :3] == orc.splits()[0][:, :3]).all()
    for g in (0, 1):
        assert _rel(sim.reactions(g)[0], orc.reactions(g)[0]) < 1e-10
    assert _rel(sim.get_state()[0], orc.get_state()[0]) < 1e-10
    sim.close()
