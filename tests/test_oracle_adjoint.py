"""Pins of the oracle's per-tet modulus and its fixed-topology window gradient.

The gradient is the reverse of the Newmark update (beta = 0, gamma = 1/2, end
of Section 2.2) with the smoothed stiffness of Eq. CSTet_fint_discretization;
a per-tet modulus enters each edge's smoothing domain as the volume-averaged
elasticity C_k = sum_j w_jk C_j.  Pinned against things other than the
oracle's own arithmetic: dense stiffness matrices assembled by independent
numpy code, a dense forward-mode (tangent) integration, and central finite
differences of the oracle's forward steps.
"""
import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def _split_setup(n=3, jit=0.1, seed=4, len_cells=2):
    m = mg.jitter(mg.kuhn_box(n, n, n), jit, seed=seed)
    pt, pm = mg.notch_presplit(mg.kuhn_box(n, n, n), axis_normal=2, plane_index=n // 2 + 1,
                               axis_len=0, len_cells=len_cells)
    return m, pt, pm


def _dense_model(o, m, E_tet):
    """Dense K(E), dK/dE_j per original tet, masses and loads of the oracle's
    current element list, from independent numpy assembly."""
    c = o.counts()
    el = o.elements()
    parent = el["parent"]
    X = np.vstack([m.X, m.X[np.zeros(c["nodes"] - len(m.X), int)]])
    geo = m.tets[parent]
    K, _ = bf.assemble(X, el["nodes"], E_tet[parent], MAT["nu"], Veff=el["Veff"], grads_from=geo)
    parts_el = bf.modulus_parts(X, el["nodes"], MAT["nu"], Veff=el["Veff"], grads_from=geo)
    parts = [np.zeros_like(K) for _ in range(len(m.tets))]
    for j, P in enumerate(parts_el):
        parts[parent[j]] += P
    mass = np.repeat(bf.lumped_mass(c["nodes"], el["nodes"], el["Veff"], MAT["rho"]), 3)
    return K, parts, mass


def test_per_tet_modulus_force_equals_dense_K():
    m, pt, pm = _split_setup()
    E = mg.modulus_field(len(m.tets), MAT["E"], 0.3, seed=7)
    o = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o.set_modulus(E)
    o.presplit(pt, pm)
    K, parts, _ = _dense_model(o, m, E)
    # K(E) is linear in the moduli: sum_j E_j dK/dE_j
    Ks = sum(e * P for e, P in zip(E, parts))
    assert np.abs(Ks - K).max() <= 1e-12 * np.abs(K).max()
    u = np.random.default_rng(1).standard_normal((o.n_nodes, 3)) * 1e-6
    f = o.internal_force(u)
    ref = K @ u.ravel()
    assert np.linalg.norm(f.ravel() - ref) < 1e-12 * np.linalg.norm(ref)
    w = np.linalg.eigvalsh(K)
    assert np.allclose(K, K.T, atol=1e-12 * abs(K).max()) and w.min() > -1e-9 * w.max()


def test_uniform_modulus_scales_force_and_time_step():
    m = mg.jitter(mg.kuhn_box(3, 2, 2), 0.2, seed=3)
    o1 = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o2 = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o2.set_modulus(np.full(len(m.tets), 4.0 * MAT["E"]))
    u = np.random.default_rng(2).standard_normal(m.X.shape) * 1e-6
    f1, f2 = o1.internal_force(u), o2.internal_force(u)
    assert np.linalg.norm(f2 - 4 * f1) <= 1e-14 * np.linalg.norm(f2)
    # omega scales with sqrt(E): dt_crit halves
    assert abs(o2.critical_dt() / o1.critical_dt() - 0.5) < 1e-14
    # the modulus equal to the scalar E everywhere is the scalar material
    o3 = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o3.set_modulus(np.full(len(m.tets), MAT["E"]))
    assert (o3.internal_force(u) == f1).all()


def _window_case(m, pt, pm, E, ramp_steps=6, seed=11, dt=None):
    o = Oracle(m.X, m.tets, MAT["E"], MAT["nu"], MAT["rho"])
    o.set_modulus(E)
    o.presplit(pt, pm)
    if dt is None:
        dt = 0.5 * o.critical_dt()
    tri = mg.face_triangles(m, 1, 1)
    trac = np.tile([0.0, 1e6, 0.0], (len(tri), 1))
    o.set_traction(tri, trac, ramp_t0=ramp_steps * dt)
    o.set_dt(dt)
    rng = np.random.default_rng(seed)
    n = o.n_nodes
    u0 = rng.standard_normal((n, 3)) * 1e-7
    v0 = rng.standard_normal((n, 3)) * 1e-3
    o.set_state(u0, v0)
    return o, dt, u0, v0


def test_window_gradient_matches_dense_tangent():
    m, pt, pm = _split_setup(n=2, jit=0.15, seed=5, len_cells=1)
    E = mg.modulus_field(len(m.tets), MAT["E"], 0.2, seed=8)
    o, dt, u0, v0 = _window_case(m, pt, pm, E)
    nsteps = 25
    K, parts, mass = _dense_model(o, m, E)
    F = o.loads().ravel()
    ramp_t0 = 6 * dt
    r = lambda k: min(k * dt / ramp_t0, 1.0)
    rng = np.random.default_rng(12)
    gu = rng.standard_normal(u0.shape)
    gv = rng.standard_normal(u0.shape) * 1e-4
    gu0, gv0, gE = o.window_gradient(nsteps, gu, gv)
    uN, vN, _ = o.get_state()

    # dense forward with tangents: columns of dU are d u / d E_j, then the
    # linear maps of u0 and v0
    ndof, ne = len(F), len(E)
    u, v = u0.ravel().copy(), v0.ravel().copy()
    a = (r(0) * F - K @ u) / mass
    dU, dV = np.zeros((ndof, ne)), np.zeros((ndof, ne))
    PU = lambda x: np.stack([P @ x for P in parts], 1)
    dA = -(PU(u) + K @ dU) / mass[:, None]
    Mu, Mv = np.eye(ndof), np.zeros((ndof, ndof))  # d(u, v)/du0
    Nu, Nv = np.zeros((ndof, ndof)), np.eye(ndof)  # d(u, v)/dv0
    Ma, Na = -(K @ Mu) / mass[:, None], -(K @ Nu) / mass[:, None]
    for k in range(nsteps):
        u1 = u + dt * v + 0.5 * dt * dt * a
        a1 = (r(k + 1) * F - K @ u1) / mass
        v = v + 0.5 * dt * (a + a1)
        dU1 = dU + dt * dV + 0.5 * dt * dt * dA
        dA1 = -(PU(u1) + K @ dU1) / mass[:, None]
        dV = dV + 0.5 * dt * (dA + dA1)
        Mu1 = Mu + dt * Mv + 0.5 * dt * dt * Ma
        Ma1 = -(K @ Mu1) / mass[:, None]
        Mv = Mv + 0.5 * dt * (Ma + Ma1)
        Nu1 = Nu + dt * Nv + 0.5 * dt * dt * Na
        Na1 = -(K @ Nu1) / mass[:, None]
        Nv = Nv + 0.5 * dt * (Na + Na1)
        u, a, dU, dA, Mu, Ma, Nu, Na = u1, a1, dU1, dA1, Mu1, Ma1, Nu1, Na1
    assert np.linalg.norm(uN.ravel() - u) < 1e-11 * np.linalg.norm(u)
    assert np.linalg.norm(vN.ravel() - v) < 1e-11 * np.linalg.norm(v)
    g = gu.ravel(), gv.ravel()
    ref_E = g[0] @ dU + g[1] @ dV
    ref_u0 = g[0] @ Mu + g[1] @ Mv
    ref_v0 = g[0] @ Nu + g[1] @ Nv
    assert np.linalg.norm(gE - ref_E) < 1e-10 * np.linalg.norm(ref_E)
    assert np.linalg.norm(gu0.ravel() - ref_u0) < 1e-10 * np.linalg.norm(ref_u0)
    assert np.linalg.norm(gv0.ravel() - ref_v0) < 1e-10 * np.linalg.norm(ref_v0)


def _J(m, pt, pm, E, u0, v0, n, gu, gv, dt):
    # the time step is an input of the window, held fixed as E varies
    o, _, _, _ = _window_case(m, pt, pm, E, dt=dt)
    o.set_state(u0, v0)
    o.set_frozen(True)
    o.step(n)
    u, v, _ = o.get_state()
    return float((gu * u).sum() + (gv * v).sum())


def test_window_gradient_matches_central_differences():
    m, pt, pm = _split_setup(n=4, jit=0.1, seed=6, len_cells=2)
    E = mg.modulus_field(len(m.tets), MAT["E"], 0.1, seed=3)
    o, dt, u0, v0 = _window_case(m, pt, pm, E)
    n = 40
    rng = np.random.default_rng(21)
    gu = rng.standard_normal(u0.shape)
    gv = rng.standard_normal(u0.shape) * 1e-4
    gu0, gv0, gE = o.window_gradient(n, gu, gv)
    J = lambda E_, u_, v_: _J(m, pt, pm, E_, u_, v_, n, gu, gv, dt)
    # direction in the moduli, relative step 1e-6
    dE = rng.choice([-1.0, 1.0], len(E)) * E
    h = 1e-6
    fd = (J(E + h * dE, u0, v0) - J(E - h * dE, u0, v0)) / (2 * h)
    assert abs(fd - gE @ dE) < 1e-6 * abs(fd)
    # single tets: one in the notch (split copies add to their parent) and one away
    for t in (int(pt[0]), int(np.argmax(np.abs(gE)))):
        e = np.zeros(len(E))
        e[t] = E[t]
        fd = (J(E + h * e, u0, v0) - J(E - h * e, u0, v0)) / (2 * h)
        assert abs(fd - gE[t] * E[t]) < 1e-5 * abs(fd) + 1e-9 * abs(gE @ dE)
    # J is affine in the initial state: differences are exact up to rounding
    du = rng.standard_normal(u0.shape) * 1e-7
    dv = rng.standard_normal(u0.shape) * 1e-3
    fd_u = (J(E, u0 + du, v0) - J(E, u0 - du, v0)) / 2
    fd_v = (J(E, u0, v0 + dv) - J(E, u0, v0 - dv)) / 2
    assert abs(fd_u - (gu0 * du).sum()) < 1e-7 * abs(fd_u)
    assert abs(fd_v - (gv0 * dv).sum()) < 1e-7 * abs(fd_v)


def test_window_leaves_end_state_and_frozen_topology():
    m, pt, pm = _split_setup(n=3)
    E = mg.modulus_field(len(m.tets), MAT["E"], 0.1, seed=3)
    o, _, u0, v0 = _window_case(m, pt, pm, E)
    c0 = o.counts()
    o.window_gradient(10, np.ones(u0.shape))
    u, v, _ = o.get_state()
    o2, _, _, _ = _window_case(m, pt, pm, E)
    o2.set_frozen(True)
    o2.step(10)
    u2, v2, _ = o2.get_state()
    assert (u == u2).all() and (v == v2).all()
    assert o.counts() == c0 and o.energy()["step"] == 10


def test_strain_energy_modulus_gradient():
    # explicit dSE/dE_j at fixed u against central differences of the
    # oracle's strain energy, and Euler's identity sum_j E_j dSE/dE_j = SE
    # (SE is linear in the moduli at fixed u)
    m, pt, pm = _split_setup(n=3)
    E = mg.modulus_field(len(m.tets), MAT["E"], 0.2, seed=4)
    o, _, u0, _ = _window_case(m, pt, pm, E)
    u = np.random.default_rng(5).standard_normal(u0.shape) * 1e-6
    g = o.strain_energy_grad(u)

    def se(E_):
        oo, _, _, _ = _window_case(m, pt, pm, E_)
        oo.set_state(u, np.zeros_like(u))
        return oo.energy()["SE"]

    assert abs(g @ E - se(E)) < 1e-12 * se(E)
    # the internal force is dSE/du
    f = o.internal_force(u)
    assert abs(0.5 * (f * u).sum() - se(E)) < 1e-12 * se(E)
    for t in (int(pt[0]), 5, int(np.argmax(g))):
        e = np.zeros(len(E))
        e[t] = 1e-4 * E[t]
        fd = (se(E + e) - se(E - e)) / 2e-4
        assert abs(fd - g[t] * E[t]) < 1e-8 * abs(se(E))
