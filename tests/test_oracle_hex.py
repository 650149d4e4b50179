"""Pins of the oracle's trilinear hexahedra (ES-H-FEM, Eqs. hex_strain_discretization
and hex_fint_discretization, factor 1/12).  Each hex enters the smoothing
domain of edge k with its shape-function gradients at G_k, the edge midpoint
(Eq. strain_discretization writes dN/dx at G_i).

Pinned against: a dense stiffness assembled by independent numpy code
straight from that formula (gradients by solving J^T g = dN/dxi at each edge
midpoint, volumes from surface integrals); exactly six zero-energy modes
(rigid motions) on free meshes and rank 18 on one hex (no hourglass modes);
the patch test; rigid-body modes; the element-bound time step against the
dense spectrum; the 1D bar wave speed.
"""
import numpy as np

from oracle import bruteforce as bf
from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def _jittered(g=(2, 2, 2), amount=0.2, seed=0):
    m = mg.hex_box(*g)
    return mg.jitter(m, amount, seed=seed)


def test_hex_force_equals_dense_edge_point_K():
    for g, seed in (((2, 2, 2), 0), ((3, 2, 2), 1)):
        m = _jittered(g, 0.2, seed)
        o = Oracle.hex_mesh(m, MAT)
        K, V = bf.assemble_hex(m.X, m.hexes, MAT["E"], MAT["nu"])
        assert abs(V.sum() - 1.0) < 1e-12  # interior jitter keeps the unit box
        # lumped masses rho V / 8 carry the surface-integral volumes
        assert abs(o.masses().sum() - MAT["rho"] * V.sum()) < 1e-12 * MAT["rho"]
        u = np.random.default_rng(3).standard_normal(m.X.shape) * 1e-6
        f = o.internal_force(u)
        ref = K @ u.ravel()
        assert np.linalg.norm(f.ravel() - ref) < 1e-12 * np.linalg.norm(ref)
        # symmetric positive semi-definite with the six rigid modes only
        assert np.allclose(K, K.T, atol=1e-12 * abs(K).max())
        w = np.linalg.eigvalsh(K)
        assert w.min() > -1e-9 * w.max()
        assert (w < 1e-10 * w.max()).sum() == 6


def test_single_hex_has_no_hourglass_modes():
    # one hex: every edge patch is the hex, K = (V / 12) sum_q B_q^T C B_q,
    # of rank 24 - 6
    X = np.array([[0, 0, 0], [1.0, 0.1, 0], [1.1, 0.9, 0.05], [0.1, 1.0, 0],
                  [0.05, 0, 1.0], [1.0, 0.05, 1.1], [1.0, 1.0, 1.0], [0, 1.1, 0.9]])
    h = np.arange(8)[None]
    o = Oracle(X, h, MAT["E"], MAT["nu"], MAT["rho"], hexes=True)
    K, V = bf.assemble_hex(X, h, MAT["E"], MAT["nu"])
    w = np.linalg.eigvalsh(K)
    assert (w > 1e-10 * w.max()).sum() == 18
    u = np.random.default_rng(0).standard_normal((8, 3)) * 1e-6
    assert np.linalg.norm(o.internal_force(u).ravel() - K @ u.ravel()) < 1e-12 * np.linalg.norm(K @ u.ravel())


def test_edge_point_gradients_of_a_unit_cube():
    # unit cube, local node order of the reference cube: at the midpoint of
    # the edge from node 0 to node 1 (y = z = 0), N_i = prod (1/2 +- x_d) with
    # the signs of node i, so dN_0/dx = -1/2, dN_1/dx = 1/2, dN_0/dy = -1/2,
    # dN_3/dy = 1/2, dN_1/dy = -1/2, dN_2/dy = 1/2 ... (closed form below)
    s = bf._HEX_SIGN
    X = (s + 1) / 2.0
    g = bf.hex_gradients_at(X, [0.0, -1.0, -1.0])
    p = np.array([0.5, 0.0, 0.0])  # the edge midpoint in physical coordinates
    f = np.where(s > 0, p, 1 - p)  # 1D factors of each node
    want = np.stack([s[:, 0] * f[:, 1] * f[:, 2], f[:, 0] * s[:, 1] * f[:, 2],
                     f[:, 0] * f[:, 1] * s[:, 2]], axis=1)
    assert np.abs(g - want).max() < 1e-15
    # the oracle's strain of a field that is linear along x only at that edge
    o = Oracle(X, np.arange(8)[None], MAT["E"], MAT["nu"], MAT["rho"], hexes=True)
    u = np.zeros((8, 3))
    u[:, 0] = X[:, 0] * X[:, 1]  # u_x = x y: du_x/dy = x = 1/2 at (1/2, 0, 0)
    nodes, eps, _ = o.edges(u)
    k = [i for i, (a, b) in enumerate(nodes.tolist()) if {a, b} == {0, 1}][0]
    assert abs(eps[k][0] - 0.0) < 1e-15 and abs(eps[k][3] - 0.5) < 1e-15


def test_hex_patch_test_and_rigid_modes():
    A = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.2, 0.0, 0.7]]) * 1e-4
    S = 0.5 * (A + A.T)
    want = np.array([S[0, 0], S[1, 1], S[2, 2], 2 * S[0, 1], 2 * S[1, 2], 2 * S[0, 2]])
    # a linear field has its exact strain at every edge point of any hex
    # (trilinear shape functions reproduce it), distorted ones included
    m = _jittered((3, 3, 2), 0.2, 2)
    o = Oracle.hex_mesh(m, MAT)
    u = m.X @ A.T + np.array([1e-5, -2e-5, 3e-5])
    _, eps, _ = o.edges(u)
    assert np.abs(eps - want).max() < 1e-12 * np.abs(want).max()
    # rigid rotation + translation: no force
    W = np.array([[0, -0.3, 0.2], [0.3, 0, -0.1], [-0.2, 0.1, 0]]) * 1e-6
    f = o.internal_force(m.X @ W.T + 1e-6)
    assert np.abs(f).max() < 1e-12 * MAT["E"] * 1e-6
    # parallelepipeds (an affine image of the box): the twelve edge points
    # with weight V / 12 integrate grad N_i exactly, so a constant stress
    # leaves no force on interior nodes
    m = mg.hex_box(3, 3, 3)
    Q = np.array([[1.0, 0.25, -0.1], [0.05, 0.9, 0.2], [-0.15, 0.1, 1.1]])
    m.X = m.X @ Q.T
    o = Oracle.hex_mesh(m, MAT)
    u = m.X @ A.T
    _, eps, _ = o.edges(u)
    assert np.abs(eps - want).max() < 1e-12 * np.abs(want).max()
    f = o.internal_force(u)
    n = np.rint(np.linalg.solve(Q, m.X.T).T * 3).astype(int)  # grid indices
    interior = np.all((n > 0) & (n < 3), axis=1)
    assert interior.sum() == 8
    assert np.abs(f[interior]).max() < 1e-12 * np.abs(f).max()


def test_hex_critical_dt_bounds_dense_spectrum():
    m = _jittered((2, 2, 2), 0.15, 4)
    o = Oracle.hex_mesh(m, MAT)
    K, _ = bf.assemble_hex(m.X, m.hexes, MAT["E"], MAT["nu"])
    mass = np.repeat(o.masses(), 3)
    assert abs(o.masses().sum() - MAT["rho"]) < 1e-12 * MAT["rho"]
    w2 = np.linalg.eigvalsh(K / np.sqrt(np.outer(mass, mass)))
    dt = o.critical_dt()
    assert dt <= 2.0 / np.sqrt(w2.max()) * (1 + 1e-12)
    # a regular cube grid: the bound scales with h
    o2 = Oracle.hex_mesh(mg.hex_box(4, 4, 4, 0.5, 0.5, 0.5), MAT)
    o4 = Oracle.hex_mesh(mg.hex_box(4, 4, 4), MAT)
    assert abs(o4.critical_dt() / o2.critical_dt() - 2) < 1e-12


def test_hex_bar_wave_speed():
    m = mg.hex_bar(100, 1.0, 0.01)
    o = Oracle(m.X, m.hexes, MAT["E"], 0.0, MAT["rho"], hexes=True)
    dt = 0.5 * o.critical_dt()
    o.set_dt(dt)
    left = np.nonzero(m.X[:, 0] < 1e-12)[0]
    vel = np.zeros((len(left), 3))
    vel[:, 0] = 0.1
    o.add_velocity_bc(left, np.ones(len(left), np.int32), vel, 0.0)
    c = np.sqrt(MAT["E"] / MAT["rho"])
    n = int(0.6 / c / dt)
    o.step(n)
    _, v, _ = o.get_state()
    x = m.X[:, 0]
    # the front (half of the driven velocity) sits at c t
    xs = np.sort(np.unique(np.round(x, 9)))
    vm = np.array([v[np.abs(x - xv) < 1e-9, 0].mean() for xv in xs])
    k = np.nonzero(vm < 0.05)[0][0]
    x_front = xs[k - 1] + (vm[k - 1] - 0.05) / (vm[k - 1] - vm[k]) * (xs[k] - xs[k - 1])
    assert abs(x_front / (c * n * dt) - 1) < 0.02
