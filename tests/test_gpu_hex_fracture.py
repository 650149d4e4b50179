"""Hexahedral crack patterns III-VI (Section 3) on the GPU against the oracle,
through the C-ABI.

- Front rates: every candidate row (hex, face, plane, pattern) equal, G within
  1e-12 relative (FP64) on a distorted block with random precracks and a
  random state.
- Through fracture: a 320-hex distorted block with 30 random precracks under
  a ramped 10 MPa pull runs 400 steps; the crack events (step, hex, plane,
  pattern) are identical, with patterns III, IV, V and VI all among them, G
  within 1e-9, u, v within 1e-9 (relative L2), U_d and Gmax within 1e-9.  Mixed
  precision: the same events over the first 200 steps, u within 1e-5.
- A checkpoint taken between cracks restores the same continuation bitwise.
- A jittered notched plate pulled apart by prescribed velocities: identical
  crack events, u within 1e-9, reactions and their work within 1e-9.
- Refusals: a plane index past 22, a forced schedule, the static readback.
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


def _block(traction=1e7, n_pre=30, seed=5):
    m = mg.jitter(mg.hex_box(10, 8, 4, 10e-3, 8e-3, 4e-3), 0.15, seed=2)
    mg.add_tension(m, 1, traction)
    rng = np.random.default_rng(seed)
    m.precrack_hexes = rng.choice(m.n_hex, size=n_pre, replace=False).astype(np.int32)
    m.precrack_planes = rng.integers(0, 23, size=n_pre).astype(np.uint8)
    return m


def _sim(m, **kw):
    from paper_2508_04076_amd.cem import Simulation
    return Simulation.from_hex_mesh(m, MAT, ramp_t0=1e-6, **kw)


def test_front_rates_match_the_oracle():
    _case("hex front G rows, distorted 4x4x3 block, 10 random precracks, random state")
    m = mg.jitter(mg.hex_box(4, 4, 3, 4e-3, 4e-3, 3e-3), 0.2, seed=7)
    rng = np.random.default_rng(8)
    m.precrack_hexes = rng.choice(m.n_hex, size=10, replace=False).astype(np.int32)
    m.precrack_planes = rng.integers(0, 23, size=10).astype(np.uint8)
    u = mg.random_displacement(m.n_nodes, 2e-6, seed=9) + 1e-4 * np.outer(m.X[:, 1], [0.3, 1.0, -0.2])
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.set_state(u)
    ro, go = o.front_G()
    for precision, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        sim = _sim(m, traction=False, precision=precision)
        sim.set_state(u)
        rg, gg = sim.front_G()
        assert rg.tolist() == ro.tolist() and gg[:, 1].tolist() == go[:, 1].tolist()
        assert len(ro) > 20 and set(go[:, 1]) == {3, 4, 5, 6}
        scale = np.abs(go[:, 0]).max()
        assert np.abs(gg[:, 0] - go[:, 0]).max() <= tol * scale, precision
        assert sim.counts()["fronts"] == o.counts()["fronts"]
        sim.close()


def test_fracture_run_matches_the_oracle():
    _case("hex block 10x8x4 distorted, 30 random precracks, 10 MPa ramped, 400 steps FP64")
    m = _block()
    o = Oracle.hex_mesh(m, MAT, ramp_t0=1e-6)
    sim = _sim(m, graph_steps=50)
    dt = 0.5 * o.critical_dt()
    assert sim.critical_dt() == pytest.approx(2 * dt, rel=1e-12)
    o.set_dt(dt)
    sim.set_dt(dt)
    for _ in range(4):
        o.step(100)
        sim.step(100)
        eo, Go = o.splits()
        eg, Gg = sim.splits()
        assert np.array_equal(eg, eo)
        dyn = eo[:, 3] > 0
        assert np.allclose(Gg[dyn], Go[dyn], rtol=1e-9, atol=0)
        ug, vg, _ = sim.get_state()
        uo, vo, _ = o.get_state()
        assert _rel(ug, uo) < 1e-9 and _rel(vg, vo) < 1e-9
    pats = set(eo[eo[:, 3] > 0, 3].tolist())
    assert pats == {3, 4, 5, 6}, pats
    Eg, Eo = sim.energy(), o.energy()
    for k in ("Ud", "Gmax", "KE", "SE", "Wext"):
        assert Eg[k] == pytest.approx(Eo[k], rel=1e-9), k
    assert Eg["n_split"] == Eo["n_split"] and Eg["n_front"] == Eo["n_front"]
    sim.close()


def test_mixed_precision_fracture_run():
    _case("hex block mixed precision, 200 steps against the FP64 oracle")
    m = _block()
    o = Oracle.hex_mesh(m, MAT, ramp_t0=1e-6)
    sim = _sim(m, precision="mixed")
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    sim.set_dt(dt)
    o.step(200)
    sim.step(200)
    eo, _ = o.splits()
    eg, _ = sim.splits()
    assert (eo[:, 3] > 0).sum() > 50
    assert np.array_equal(eg, eo)
    assert _rel(sim.get_state()[0], o.get_state()[0]) < 1e-5
    sim.close()


def test_checkpoint_between_cracks():
    _case("hex block: checkpoint after the first cracks, restore, rerun bitwise")
    m = _block()
    sim = _sim(m, graph_steps=20)
    sim.set_dt(0.5 * sim.critical_dt())
    sim.step(60)
    n0 = sim.counts()["splits"]
    buf = sim.save_state()
    sim.step(140)
    u1, e1 = sim.get_state()[0], sim.splits()[0]
    assert len(e1) > n0
    sim.load_state(buf)
    sim.step(140)
    assert np.array_equal(sim.get_state()[0], u1) and np.array_equal(sim.splits()[0], e1)
    fresh = _sim(m, graph_steps=20)
    fresh.load_state(buf)
    fresh.step(140)
    assert np.array_equal(fresh.get_state()[0], u1) and np.array_equal(fresh.splits()[0], e1)
    fresh.close()
    sim.close()


def test_refusals():
    _case("hex refusals: plane index 23, forced schedule, static readback")
    from paper_2508_04076_amd.cem import CemError
    m = _block(n_pre=2)
    sim = _sim(m, presplit=False)
    with pytest.raises(CemError):
        sim.presplit([0], [23])
    with pytest.raises(CemError):
        sim.replay_splits(np.array([[1, 0, 1]], dtype=np.int32))
    with pytest.raises(CemError):
        sim.front_G_static()
    sim.presplit(m.precrack_hexes, m.precrack_planes)
    ev, G = sim.splits()
    o = Oracle.hex_mesh(m, MAT)
    assert np.array_equal(ev, o.splits()[0])
    sim.close()


def test_fracture_under_prescribed_velocities():
    _case("hex notched plate pulled apart by prescribed velocities, 300 steps FP64")
    m = mg.hex_notched(16, 10, 2)
    m.X = mg.jitter(m, 0.1, seed=11).X
    m.load_tris, m.load_trac = None, None
    top = np.nonzero(np.abs(m.X[:, 1] - m.X[:, 1].max()) < 1e-12)[0]
    bot = np.nonzero(np.abs(m.X[:, 1]) < 1e-12)[0]
    vt = np.zeros((len(top), 3))
    vt[:, 1] = 2.0
    o = Oracle.hex_mesh(m, MAT)
    sim = _sim(m)
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    sim.set_dt(dt)
    for x in (o, sim):
        x.add_velocity_bc(top, np.full(len(top), 2), vt, 50 * dt)
        x.add_velocity_bc(bot, np.full(len(bot), 2), np.zeros((len(bot), 3)), 0.0)
    o.step(300)
    sim.step(300)
    eo, Go = o.splits()
    eg, Gg = sim.splits()
    assert (eo[:, 3] > 0).sum() > 10 and np.array_equal(eg, eo)
    assert np.allclose(Gg, Go, rtol=1e-9, atol=0)
    assert _rel(sim.get_state()[0], o.get_state()[0]) < 1e-9
    for g in (0, 1):
        ro, wo = o.reactions(g)
        rg, wg = sim.reactions(g)
        assert _rel(rg[:, 2:5], ro[:, 2:5]) < 1e-9 and wg == pytest.approx(wo, rel=1e-9)
    sim.close()
