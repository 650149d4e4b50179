"""GPU (HIP, through the C-ABI) against the CPU oracle.

Tolerances: FP64 forces 1e-12 normwise relative; FP64 trajectories 1e-10
relative L2 (rounding order differs, no other difference); identical split
events (step, tet, side mask); mixed precision 1e-5 relative L2 on u with the
FP64 split schedule replayed.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

MAT = dict(mg.BRANCHING_MATERIAL)


def _sim(mesh, **kw):
    from paper_2508_04076_amd.cem import Simulation
    kw.setdefault("max_splits", max(mesh.n_tets // 4, 64))
    return Simulation.from_mesh(mesh, MAT, **kw)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


@pytest.mark.parametrize("name", ["cube6", "cube10_notched", "jitter5", "plate_small"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_parity(name, precision):
    _case(f"force parity {name} {precision}")
    if name == "cube6":
        mesh = mg.cube_notched(6)
        mesh.presplit_tets = None
    elif name == "cube10_notched":
        mesh = mg.cube_notched(10)
    elif name == "jitter5":
        mesh = mg.cube_notched(5)
        base = mg.kuhn_box(5, 5, 5)
        mesh.X = mg.jitter(base, 0.2, seed=0).X
    else:
        mesh = mg.plate_notched(20, 8, 2, 0.01, 0.004, 0.001, 0.005)
    sim = _sim(mesh, precision=precision)
    orc = Oracle.from_mesh(mesh, MAT)
    assert sim.n_nodes == orc.n_nodes
    for seed in range(2):
        u = mg.random_displacement(sim.n_nodes, 1e-6, seed=seed)
        fg, fo = sim.internal_force(u), orc.internal_force(u)
        err = _rel(fg, fo)
        assert err < (1e-12 if precision == "fp64" else 1e-5), err
    # a smooth field: the mixed path differences u in float64 first
    u = 1e-4 * np.sin(3 * mesh.X) if sim.n_nodes == mesh.n_nodes else None
    if u is not None:
        err = _rel(sim.internal_force(u), orc.internal_force(u))
        assert err < (1e-12 if precision == "fp64" else 1e-5), err
    sim.close()


def test_force_parity_full_plate():
    _case("force parity full 768k-tet plate")
    mesh = mg.plate_notched()
    sim = _sim(mesh, max_splits=20000)
    orc = Oracle.from_mesh(mesh, MAT, ramp_t0=1e-6)
    assert sim.n_nodes == orc.n_nodes
    u = mg.random_displacement(sim.n_nodes, 1e-7, seed=5)
    assert _rel(sim.internal_force(u), orc.internal_force(u)) < 1e-12
    assert abs(sim.critical_dt() / orc.critical_dt() - 1) < 1e-12
    c = sim.counts()
    assert c["edges0"] == 951008 and c["splits"] == 4800
    sim.close()


def test_critical_dt_jittered():
    _case("critical dt jittered")
    base = mg.kuhn_box(5, 4, 3, 0.5, 0.4, 0.3)
    mesh = mg.jitter(base, 0.25, seed=3)
    sim = _sim(mesh)
    orc = Oracle.from_mesh(mesh, MAT)
    assert abs(sim.critical_dt() / orc.critical_dt() - 1) < 1e-12
    sim.close()


def _run_pair(mesh, steps, chunks=1, sim_kw=None, orc_kw=None, ramp_t0=0.0, Gc=None):
    sim = _sim(mesh, ramp_t0=ramp_t0, Gc=Gc, **(sim_kw or {}))
    orc = Oracle.from_mesh(mesh, MAT, ramp_t0=ramp_t0, Gc=Gc, **(orc_kw or {}))
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    for _ in range(chunks):
        sim.step(steps // chunks)
        orc.step(steps // chunks)
    return sim, orc


def test_trajectory_without_fracture():
    _case("trajectory Gc=inf cube 6, 300 steps")
    mesh = mg.cube_notched(6)
    sim, orc = _run_pair(mesh, 300, chunks=3, Gc=np.inf)
    ug, vg, ag = sim.get_state()
    uo, vo, ao = orc.get_state()
    assert _rel(ug, uo) < 1e-10 and _rel(vg, vo) < 1e-10 and _rel(ag, ao) < 1e-9
    eg, eo = sim.energy(), orc.energy()
    for k in ("KE", "SE", "Wext"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * abs(eo[k]), (k, eg[k], eo[k])
    assert eg["step"] == 300 and eg["n_split"] == len(mesh.presplit_tets)
    assert eg["n_front"] == eo["n_front"]
    sim.close()


def _events_equal(sim, orc):
    eg, Gg = sim.splits()
    eo, Go = orc.splits()
    assert eg.shape == eo.shape, (eg.shape, eo.shape)
    assert np.array_equal(eg, eo)
    dyn = eo[:, 3] > 0
    if dyn.any():
        assert np.allclose(Gg[dyn], Go[dyn], rtol=1e-9, atol=0)
    return eo


@pytest.mark.parametrize("mode", ["phantom", "erode"])
def test_split_events_small_cube(mode):
    _case(f"split events cube 6 {mode}")
    mesh = mg.cube_notched(6)
    sim, orc = _run_pair(mesh, 240, chunks=4, sim_kw=dict(split_mode=mode),
                         orc_kw=dict(split_mode=mode))
    ev = _events_equal(sim, orc)
    assert (ev[:, 3] > 0).sum() > 0
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-9 and _rel(vg, vo) < 1e-9
    eg, eo = sim.energy(), orc.energy()
    assert abs(eg["Ud"] - eo["Ud"]) <= 1e-12 * eo["Ud"]
    sim.close()


def test_front_G_readback():
    _case("front G readback cube 10")
    mesh = mg.cube_notched(10)
    sim, orc = _run_pair(mesh, 20)
    tg, gg = sim.front_G()
    to, go = orc.front_G()
    assert np.array_equal(tg, to)
    scale = np.abs(go).max()
    assert scale > 0
    assert np.abs(gg - go).max() <= 1e-10 * scale
    eg, eo = sim.energy(), orc.energy()
    assert abs(eg["Gmax"] - eo["Gmax"]) <= 1e-10 * abs(eo["Gmax"])
    sim.close()


@pytest.mark.parametrize("mode", ["phantom", "erode"])
def test_split_events_cube10_full_run(mode):
    # 10^3-cell cube, 6,000 tets, notch z = 0.5 over x < 0.3, 2,000 steps
    _case(f"split events 10^3-cell cube, 2000 steps, graphs of 100 steps, {mode}")
    mesh = mg.cube_notched(10)
    sim, orc = _run_pair(mesh, 2000, chunks=4, sim_kw=dict(graph_steps=100, split_mode=mode),
                         orc_kw=dict(split_mode=mode))
    ev = _events_equal(sim, orc)
    assert (ev[:, 3] > 0).sum() > 100
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-8 and _rel(vg, vo) < 1e-8
    eg, eo = sim.energy(), orc.energy()
    for k in ("KE", "SE", "Wext", "Ud"):
        assert abs(eg[k] - eo[k]) <= 1e-8 * abs(eo[k]), (k, eg[k], eo[k])
    sim.close()


def test_plate_prefix_parity():
    # full-size 768k-tet plate, ramped load: the first steps
    _case("plate 768k prefix 12 steps")
    mesh = mg.plate_notched()
    sim, orc = _run_pair(mesh, 12, sim_kw=dict(max_splits=40000), ramp_t0=1e-6)
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-10 and _rel(vg, vo) < 1e-10
    _events_equal(sim, orc)
    sim.close()


def test_deterministic_and_graph_equals_plain():
    _case("determinism cube 10, 300 steps, plain vs graph")
    mesh = mg.cube_notched(10)
    out = []
    for gs in (0, 50, 50):
        sim = _sim(mesh, graph_steps=gs)
        sim.set_dt(6.797514528978e-06)
        sim.step(300)
        u, v, a = sim.get_state()
        ev, G = sim.splits()
        out.append((u, v, a, ev, G))
        sim.close()
    for o in out[1:]:
        for x, y in zip(out[0], o):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_checkpoint_resume_bitwise(precision):
    # the checkpoint holds split copies made by dynamic splits of the first
    # context only: the second must take their geometry (in mixed precision
    # the corner-normal rows of the copies) from the restored topology
    _case(f"checkpoint cube 8 {precision}")
    mesh = mg.cube_notched(8)
    a = _sim(mesh, precision=precision)
    dt = 0.5 * a.critical_dt()
    a.set_dt(dt)
    a.step(80)
    ev0, _ = a.splits()
    assert (ev0[:, 0] > 0).sum() > 0
    buf = a.save_state()
    a.step(80)
    ua, va, _ = a.get_state()
    eva, _ = a.splits()
    b = _sim(mesh, precision=precision)
    b.set_dt(dt)
    b.load_state(buf)
    b.step(80)
    ub, vb, _ = b.get_state()
    evb, _ = b.splits()
    assert np.array_equal(ua, ub) and np.array_equal(va, vb) and np.array_equal(eva, evb)
    a.close()
    b.close()


def test_capacity_error_leaves_state_at_failing_step():
    _case("capacity error cube 6")
    from paper_2508_04076_amd.cem import CemError, CEM_ECAPACITY
    mesh = mg.cube_notched(6)
    orc = Oracle.from_mesh(mesh, MAT)
    dt = 0.5 * orc.critical_dt()
    orc.set_dt(dt)
    orc.step(240)
    ev, _ = orc.splits()
    npre = len(mesh.presplit_tets)
    cap = npre + int((ev[:, 3] > 0).sum() // 2)
    sim = _sim(mesh, max_splits=cap)
    sim.set_dt(dt)
    with pytest.raises(CemError) as ei:
        sim.step(240)
    assert ei.value.code == CEM_ECAPACITY
    e = sim.energy()
    step = int(e["step"])
    assert e["n_split"] <= cap
    o2 = Oracle.from_mesh(mesh, MAT)
    o2.set_dt(dt)
    o2.step(step)
    ug, _, _ = sim.get_state()
    uo, _, _ = o2.get_state()
    assert ug.shape == uo.shape and _rel(ug, uo) < 1e-9
    sim.close()


def test_unstable_time_step_is_reported():
    _case("unstable dt cube 4")
    from paper_2508_04076_amd.cem import CemError, CEM_EUNSTABLE
    mesh = mg.cube_notched(4)
    sim = _sim(mesh)
    sim.set_dt(4.0 * sim.critical_dt())
    with pytest.raises(CemError) as ei:
        sim.step(400)
    assert ei.value.code == CEM_EUNSTABLE
    sim.close()


def test_replay_fp64_matches_free_run_and_mixed_error():
    _case("replay + mixed precision cube 8")
    mesh = mg.cube_notched(8)
    ref = _sim(mesh)
    dt = 0.5 * ref.critical_dt()
    ref.set_dt(dt)
    ref.step(200)
    ev, _ = ref.splits()
    u64, _, _ = ref.get_state()
    sched = ev[ev[:, 3] > 0][:, :3]
    assert len(sched) > 0
    rep = _sim(mesh)
    rep.set_dt(dt)
    rep.replay_splits(sched)
    rep.step(200)
    ur, _, _ = rep.get_state()
    evr, _ = rep.splits()
    assert np.array_equal(evr[:, :3], ev[:, :3])
    assert _rel(ur, u64) < 1e-12
    mix = _sim(mesh, precision="mixed")
    mix.set_dt(dt)
    mix.replay_splits(sched)
    mix.step(200)
    um, _, _ = mix.get_state()
    err = _rel(um, u64)
    print(f"mixed vs fp64 relative L2 of u after 200 steps: {err:.3e}", flush=True)
    assert err < 1e-5
    for s in (ref, rep, mix):
        s.close()


def test_permuted_input_numbering():
    # random relabelling of nodes and tets: the library renumbers internally
    # and answers in the caller's numbering; split order follows caller ids
    _case("permuted input cube 6, 240 steps")
    mesh = mg.permute(mg.cube_notched(6), seed=1)
    sim, orc = _run_pair(mesh, 240, chunks=2)
    _events_equal(sim, orc)
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-9 and _rel(vg, vo) < 1e-9
    tg, gg = sim.front_G()
    to, go = orc.front_G()
    assert np.array_equal(tg, to)
    u = mg.random_displacement(sim.n_nodes, 1e-6, seed=9)
    assert _rel(sim.internal_force(u), orc.internal_force(u)) < 1e-12
    sim.close()


def test_replay_with_a_repeated_tet_splits_it_once():
    _case("replay schedule naming one tet twice, jittered 4^3 cube")
    m = mg.jitter(mg.kuhn_box(4, 4, 4), 0.2, seed=8)
    m.presplit_tets = None
    sched = np.array([[2, 17, 3], [2, 101, 1], [4, 17, 6], [5, 230, 9]], dtype=np.int32)
    sim = _sim(m, Gc=3.0)
    orc = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"], Gc=3.0)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    rng = np.random.default_rng(3)
    v0 = rng.standard_normal((len(m.X), 3)) * 1e-3
    sim.set_state(None, v0)
    orc.set_state(None, v0)
    sim.replay_splits(sched)
    orc.replay(sched)
    sim.step(8)
    orc.step(8)
    eg, eo = sim.splits()[0], orc.splits()[0]
    assert eg[:, 1].tolist() == [17, 101, 230] and np.array_equal(eg[:, :3], eo[:, :3])
    ug, vg, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(ug, uo) < 1e-10 and _rel(vg, vo) < 1e-10
    sim.close()


def test_front_G_under_a_quarter_turn():
    # two tets sharing a face, the first pre-split with node 1 alone: the
    # second is a front.  A quarter turn about z with a 1% stretch lengthens
    # every edge although each displacement points against its edge, so the
    # stretch test must keep delta = du (the quadratic term decides)
    _case("front G, two tets, quarter turn + 1% stretch")
    from paper_2508_04076_amd.cem import Simulation
    X = np.array([[0.2, -1.0, 0.1], [0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [1.0, 0.0, 0.0],
                  [0.0, 1.0, 1.0]])
    t = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
    mat = dict(MAT, Gc=1e30)
    sim = Simulation(X, t, mat, max_splits=8)
    orc = Oracle(X, t, mat["E"], mat["nu"], mat["rho"], Gc=1e30)
    sim.presplit([0], [2])
    orc.presplit([0], [2])
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    ur = X @ (1.01 * Rz - np.eye(3)).T
    uq = np.zeros((sim.n_nodes, 3))
    uq[:5] = ur
    uq[5:9] = ur[[0, 1, 2, 3]]
    sim.set_state(uq, None)
    orc.set_state(uq, None)
    tg, gg = sim.front_G()
    to, go = orc.front_G()
    assert np.array_equal(tg, to) and go[0, 0] != 0
    assert np.abs(gg - go).max() <= 1e-10 * np.abs(go).max()
    sim.close()
