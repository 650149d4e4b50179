"""Pins of the oracle's trilinear hexahedra (ES-H-FEM, Eqs. hex_strain_discretization
and hex_fint_discretization, factor 1/12).

Pinned against: a dense stiffness assembled by independent numpy code whose
element gradients come from surface integrals (divergence theorem) instead of
the oracle's volume Gauss points; the patch test; rigid-body modes; the
element-bound time step against the dense spectrum; the 1D bar wave speed.
"""
import numpy as np

from oracle import bruteforce as bf
from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def _jittered(g=(2, 2, 2), amount=0.2, seed=0):
    m = mg.hex_box(*g)
    return mg.jitter(m, amount, seed=seed)


def test_hex_force_equals_dense_surface_integral_K():
    m = _jittered((3, 2, 2), 0.2, 1)
    o = Oracle.hex_mesh(m, MAT)
    K, V = bf.assemble_hex(m.X, m.hexes, MAT["E"], MAT["nu"])
    assert abs(V.sum() - 1.0) < 1e-12  # interior jitter keeps the unit box
    u = np.random.default_rng(3).standard_normal(m.X.shape) * 1e-6
    f = o.internal_force(u)
    ref = K @ u.ravel()
    assert np.linalg.norm(f.ravel() - ref) < 1e-12 * np.linalg.norm(ref)
    # symmetric positive semi-definite; rigid modes plus the hourglass modes
    # that element-average gradients leave without stiffness
    assert np.allclose(K, K.T, atol=1e-12 * abs(K).max())
    w = np.linalg.eigvalsh(K)
    assert w.min() > -1e-9 * w.max()
    assert (w < 1e-10 * w.max()).sum() >= 6


def test_single_hex_has_rank_six():
    # one hex: every edge patch is the hex, K = V Bbar^T C Bbar of rank 6
    X = np.array([[0, 0, 0], [1.0, 0.1, 0], [1.1, 0.9, 0.05], [0.1, 1.0, 0],
                  [0.05, 0, 1.0], [1.0, 0.05, 1.1], [1.0, 1.0, 1.0], [0, 1.1, 0.9]])
    h = np.arange(8)[None]
    o = Oracle(X, h, MAT["E"], MAT["nu"], MAT["rho"], hexes=True)
    K, V = bf.assemble_hex(X, h, MAT["E"], MAT["nu"])
    w = np.linalg.eigvalsh(K)
    assert (w > 1e-10 * w.max()).sum() == 6
    u = np.random.default_rng(0).standard_normal((8, 3)) * 1e-6
    assert np.linalg.norm(o.internal_force(u).ravel() - K @ u.ravel()) < 1e-12 * np.linalg.norm(K @ u.ravel())


def test_hex_patch_test_and_rigid_modes():
    m = _jittered((3, 3, 2), 0.2, 2)
    o = Oracle.hex_mesh(m, MAT)
    A = np.array([[1.0, 0.3, -0.2], [0.1, -0.5, 0.4], [0.2, 0.0, 0.7]]) * 1e-4
    u = m.X @ A.T + np.array([1e-5, -2e-5, 3e-5])
    _, eps, _ = o.edges(u)
    S = 0.5 * (A + A.T)
    want = np.array([S[0, 0], S[1, 1], S[2, 2], 2 * S[0, 1], 2 * S[1, 2], 2 * S[0, 2]])
    assert np.abs(eps - want).max() < 1e-12 * np.abs(want).max()
    f = o.internal_force(u)
    lo, hi = m.X.min(0), m.X.max(0)
    interior = np.all((m.X > lo + 1e-9) & (m.X < hi - 1e-9), axis=1)
    assert np.abs(f[interior]).max() < 1e-9 * np.abs(f).max()
    # rigid rotation + translation: no force
    W = np.array([[0, -0.3, 0.2], [0.3, 0, -0.1], [-0.2, 0.1, 0]]) * 1e-6
    f = o.internal_force(m.X @ W.T + 1e-6)
    assert np.abs(f).max() < 1e-12 * MAT["E"] * 1e-6


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
