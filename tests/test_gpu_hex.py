"""GPU trilinear hexahedra (ES-H-FEM) against the oracle, through the C-ABI.

Tolerances: FP64 forces 1e-12 normwise relative, FP64 trajectories and
reactions 1e-10 relative L2, critical time step 1e-12; mixed precision 1e-5
on forces.
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


def _pair(mesh, mat=MAT, ramp_t0=0.0, **kw):
    from paper_2508_04076_amd.cem import Simulation
    sim = Simulation.from_hex_mesh(mesh, mat, ramp_t0=ramp_t0, **kw)
    orc = Oracle.hex_mesh(mesh, mat, ramp_t0=ramp_t0)
    return sim, orc


@pytest.mark.parametrize("name", ["jitter3", "plate_small"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hex_force_and_dt_parity(name, precision):
    _case(f"hex force parity {name} {precision}")
    if name == "jitter3":
        mesh = mg.jitter(mg.hex_box(3, 3, 2), 0.2, seed=1)
    else:
        mesh = mg.hex_box(40, 16, 2, 0.01, 0.004, 0.0005)
    sim, orc = _pair(mesh, precision=precision)
    assert sim.n_nodes == orc.n_nodes == mesh.n_nodes
    tol = 1e-12 if precision == "fp64" else 1e-5
    for seed in range(2):
        u = mg.random_displacement(mesh.n_nodes, 1e-6, seed=seed)
        assert _rel(sim.internal_force(u), orc.internal_force(u)) < tol
    assert abs(sim.critical_dt() / orc.critical_dt() - 1) < 1e-12
    c = sim.counts()
    assert c["edges0"] == orc.counts()["edges"]
    sim.close()


def test_hex_trajectory_with_traction_and_energy():
    _case("hex trajectory, traction")
    mesh = mg.add_tension(mg.jitter(mg.hex_box(6, 6, 6), 0.15, seed=2), 2, 1e6)
    sim, orc = _pair(mesh, ramp_t0=1e-5, graph_steps=16)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    sim.step(200)
    orc.step(200)
    us, vs, _ = sim.get_state()
    uo, vo, _ = orc.get_state()
    assert _rel(us, uo) < 1e-10 and _rel(vs, vo) < 1e-10
    es, eo = sim.energy(), orc.energy()
    for k in ("KE", "SE", "Wext"):
        assert abs(es[k] / eo[k] - 1) < 1e-9, k
    assert es["n_split"] == 0 and es["n_front"] == 0
    sim.close()


def test_hex_bar_velocity_groups():
    _case("hex bar, prescribed velocities")
    mesh = mg.hex_bar(60, 0.6, 0.01)
    mat = dict(MAT, nu=0.0)
    sim, orc = _pair(mesh, mat=mat)
    dt = 0.5 * orc.critical_dt()
    sim.set_dt(dt)
    orc.set_dt(dt)
    x = mesh.X[:, 0]
    left, right = np.nonzero(x < 1e-12)[0], np.nonzero(x > 0.6 - 1e-12)[0]
    vl = np.zeros((len(left), 3))
    vl[:, 0] = 0.1
    for o in (sim, orc):
        o.add_velocity_bc(left, np.ones(len(left)), vl, 20 * dt)
        o.add_velocity_bc(right, np.full(len(right), 7), np.zeros((len(right), 3)), 0.0)
    sim.step(300)
    orc.step(300)
    for g in (0, 1):
        (rs, ws), (ro, wo) = sim.reactions(g), orc.reactions(g)
        assert _rel(rs, ro) < 1e-10 and abs(ws - wo) <= 1e-10 * abs(wo) + 1e-30
    assert _rel(sim.get_state()[0], orc.get_state()[0]) < 1e-10
    sim.close()


def test_hex_refusals_numbering_and_checkpoint():
    _case("hex refusals, relabelled input, checkpoint")
    from paper_2508_04076_amd.cem import CemError, Simulation
    mesh = mg.add_tension(mg.jitter(mg.hex_box(4, 3, 3), 0.2, seed=5), 1, 3e7)
    mesh.precrack_hexes = np.array([5, 20], dtype=np.int32)
    mesh.precrack_planes = np.array([1, 7], dtype=np.uint8)
    sim = Simulation.from_hex_mesh(mesh, MAT, presplit=False)
    with pytest.raises(CemError):
        sim.presplit([0], [23])  # crack plane indices run 0-22
    with pytest.raises(CemError):
        sim.set_modulus(np.full(mesh.n_hex, MAT["E"]))
    sim.presplit(mesh.precrack_hexes, mesh.precrack_planes)
    dt = 0.5 * sim.critical_dt()
    sim.set_dt(dt)
    with pytest.raises(CemError):
        sim.window_forward(2, 1)
    assert len(sim.front_G()[0]) > 0
    # relabelled nodes and hexes give the same answer in the caller's numbering
    rng = np.random.default_rng(3)
    pn, ph = rng.permutation(mesh.n_nodes), rng.permutation(mesh.n_hex)
    inv = np.empty_like(pn)
    inv[pn] = np.arange(len(pn))
    hinv = np.argsort(ph)  # hex ph[i] of the mesh is hex i of the relabelled one
    m2 = mg.HexMesh(X=mesh.X[pn], hexes=inv[mesh.hexes[ph]].astype(np.int32),
                    load_tris=inv[mesh.load_tris].astype(np.int32), load_trac=mesh.load_trac,
                    precrack_hexes=hinv[mesh.precrack_hexes].astype(np.int32),
                    precrack_planes=mesh.precrack_planes)
    sim2 = Simulation.from_hex_mesh(m2, MAT)
    sim2.set_dt(dt)
    sim.step(40)
    sim2.step(40)
    u1 = sim.get_state()[0]
    u2 = sim2.get_state()[0]
    assert _rel(u2, u1[pn]) < 1e-12
    e1, e2 = sim.splits()[0], sim2.splits()[0]
    assert len(e1) > 2 and len(e1) == len(e2)
    back = e2.copy()
    back[:, 1] = ph[e2[:, 1]]
    key = lambda e: sorted(map(tuple, e.tolist()))
    assert key(back) == key(e1)
    buf = sim.save_state()
    sim.step(10)
    ua = sim.get_state()[0]
    sim.load_state(buf)
    sim.step(10)
    assert (sim.get_state()[0] == ua).all()
    sim.close()
    sim2.close()


def test_hex_plate_full_size_force():
    # the plate at 200 x 80 x 8 hexahedral cells (128,000 hexes)
    _case("hex plate 128k force parity")
    mesh = mg.hex_box(200, 80, 8, 0.1, 0.04, 0.004)
    sim, orc = _pair(mesh)
    u = mg.random_displacement(mesh.n_nodes, 1e-7, seed=4)
    assert _rel(sim.internal_force(u), orc.internal_force(u)) < 1e-12
    # (the time step is compared on the smaller meshes: the oracle's 24 x 24
    # eigenproblem per hex takes minutes at this size)
    sim.close()
