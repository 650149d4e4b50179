"""Dense brute-force checker for tiny meshes -- TEST INFRASTRUCTURE ONLY.

Independent numpy code (it calls nothing in the oracle library) that assembles
the full ES-T-FEM stiffness matrix K = sum_k V_k Bt_k^T C Bt_k, where
Bt_k = sum_{j in patch k} w_jk B_j is the smoothed strain-displacement matrix
of edge k (Eqs. strain_discretization and CSTet_fint_discretization, with
V_k = (1/6) sum_j V_j), and the standard FEM stiffness K_FEM = sum_j V_j B_j^T
C B_j for comparison.  Also the consistent dense mass-free quantities the
dynamics pins need (eigenvalues of M^-1 K).
"""
from __future__ import annotations

import itertools

import numpy as np


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def cmat(E, nu):
    lam, mu = lame(E, nu)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[np.arange(3), np.arange(3)] += 2 * mu
    C[3:, 3:] = np.eye(3) * mu
    return C


def tet_B(x):
    """x: [4,3] node coords. Returns (B [6, 12], V) from the barycentric map."""
    # solve for gradients of the linear shape functions: [1 x y z] a = e_l
    A = np.hstack([np.ones((4, 1)), x])
    coef = np.linalg.inv(A)         # columns: coefficients of N_l
    g = coef[1:, :].T               # [4, 3] gradient of N_l
    V = np.linalg.det(A) / 6.0
    B = np.zeros((6, 12))
    for l in range(4):
        gx, gy, gz = g[l]
        c = 3 * l
        B[0, c] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c], B[3, c + 1] = gy, gx
        B[4, c + 1], B[4, c + 2] = gz, gy
        B[5, c], B[5, c + 2] = gz, gx
    return B, V


def _edges_and_patches(elem_nodes):
    patches = {}
    for j, nd in enumerate(elem_nodes):
        for a, b in itertools.combinations(range(4), 2):
            key = tuple(sorted((int(nd[a]), int(nd[b]))))
            patches.setdefault(key, []).append(j)
    return patches


def assemble(X, elem_nodes, E, nu, Veff=None, grads_from=None, parts=None):
    """Dense K_ES and K_FEM for elements with node lists `elem_nodes`.

    X: [N, 3] coordinates of every node referenced.  E: scalar or one modulus
    per element; the smoothing domain of an edge then has the volume-averaged
    elasticity C_k = sum_j w_jk C(E_j).  Veff: per-element volume
    carried (defaults to the geometric volume).  grads_from: optional [ne, 4]
    node ids whose coordinates define each element's geometry (for split copies
    whose extra nodes sit on top of their twins the geometry is the same).
    """
    X = np.asarray(X, float)
    elem_nodes = np.asarray(elem_nodes)
    N = len(X)
    ne = len(elem_nodes)
    Ej = np.broadcast_to(np.asarray(E, float), (ne,))
    Cs = [cmat(e, nu) for e in Ej]
    Bs, Vs = [], []
    for j in range(ne):
        geo = elem_nodes[j] if grads_from is None else grads_from[j]
        B, V = tet_B(X[geo])
        Bs.append(B)
        Vs.append(V)
    Vs = np.array(Vs)
    Ve = Vs if Veff is None else np.asarray(Veff, float)
    dof = lambda nd: np.array([[3 * n, 3 * n + 1, 3 * n + 2] for n in nd]).ravel()
    K = np.zeros((3 * N, 3 * N))
    for key, pj in _edges_and_patches(elem_nodes).items():
        S = sum(Ve[j] for j in pj)
        if S == 0:
            continue
        Bt = np.zeros((6, 3 * N))
        Ck = np.zeros((6, 6))
        for j in pj:
            Bt[:, dof(elem_nodes[j])] += (Ve[j] / S) * Bs[j]
            Ck += (Ve[j] / S) * Cs[j]
        if parts is not None:
            for j in pj:
                parts[j] += (Ve[j] / 6.0) * Bt.T @ cmat(1.0, nu) @ Bt
        K += (S / 6.0) * Bt.T @ Ck @ Bt
    Kf = np.zeros((3 * N, 3 * N))
    for j in range(ne):
        d = dof(elem_nodes[j])
        Kf[np.ix_(d, d)] += Ve[j] * Bs[j].T @ Cs[j] @ Bs[j]
    return K, Kf


def modulus_parts(X, elem_nodes, nu, Veff=None, grads_from=None):
    """dK_ES/dE_j for every element j (dense), so that K_ES(E) = sum_j E_j K_j."""
    N = len(X)
    parts = [np.zeros((3 * N, 3 * N)) for _ in range(len(elem_nodes))]
    assemble(X, elem_nodes, 1.0, nu, Veff, grads_from, parts=parts)
    return parts


def lumped_mass(N, elem_nodes, Veff, rho):
    m = np.zeros(N)
    for j, nd in enumerate(elem_nodes):
        for n in nd:
            m[n] += rho * Veff[j] / 4.0
    return m


# ---------------------------------------------------------------- hexahedra

_HEX_SIGN = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                      [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], float)
# the six faces as local node quadruples, counter-clockwise seen from outside
_HEX_FACES = [(0, 3, 2, 1), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]
_HEX_EDGES = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
              (0, 4), (1, 5), (2, 6), (3, 7)]


def hex_surface_integrals(x):
    """x: [8, 3] hex nodes.  Returns (G [8, 3], V) with G_i = integral of grad N_i
    over the hex and V its volume, both from surface integrals (divergence
    theorem): G_i = sum over faces of int N_i n dS and V = (1/3) int x . n dS,
    each face a bilinear patch integrated with 2 x 2 Gauss points (exact)."""
    x = np.asarray(x, float)
    G = np.zeros((8, 3))
    V = 0.0
    a = 1.0 / np.sqrt(3.0)
    for f in _HEX_FACES:
        xf = x[list(f)]
        for s in (-a, a):
            for t in (-a, a):
                w = np.array([(1 - s) * (1 - t), (1 + s) * (1 - t), (1 + s) * (1 + t),
                              (1 - s) * (1 + t)]) / 4.0
                ds = np.array([-(1 - t), (1 - t), (1 + t), -(1 + t)]) / 4.0
                dt = np.array([-(1 - s), -(1 + s), (1 + s), (1 - s)]) / 4.0
                xs, xt = ds @ xf, dt @ xf
                ndS = np.cross(xs, xt)          # outward for this node order
                for q, i in enumerate(f):
                    G[i] += w[q] * ndS
                V += (w @ xf) @ ndS / 3.0
    return G, V


def hex_gradients_at(x, xi):
    """Gradients of the eight trilinear shape functions of the hex x [8, 3] at
    the natural point xi, by solving J^T g_i = dN_i/dxi (numpy)."""
    x = np.asarray(x, float)
    f = 1.0 + _HEX_SIGN * np.asarray(xi, float)          # [8, 3]
    dN = np.empty((8, 3))
    dN[:, 0] = _HEX_SIGN[:, 0] * f[:, 1] * f[:, 2] / 8.0
    dN[:, 1] = f[:, 0] * _HEX_SIGN[:, 1] * f[:, 2] / 8.0
    dN[:, 2] = f[:, 0] * f[:, 1] * _HEX_SIGN[:, 2] / 8.0
    J = x.T @ dN                                        # J[r, c] = dx_r / dxi_c
    return np.linalg.solve(J.T, dN.T).T


def _hex_B(g):
    B = np.zeros((6, 24))
    for l in range(8):
        gx, gy, gz = g[l]
        c = 3 * l
        B[0, c], B[1, c + 1], B[2, c + 2] = gx, gy, gz
        B[3, c], B[3, c + 1] = gy, gx
        B[4, c + 1], B[4, c + 2] = gz, gy
        B[5, c], B[5, c + 2] = gz, gx
    return B


def assemble_hex(X, hexes, E, nu):
    """Dense ES-H-FEM stiffness straight from Eq. strain_discretization: the
    smoothing domain of hex edge k collects the hexes j sharing it, each with
    its shape-function gradients at G_k, the edge's midpoint, and weight
    w_jk = V_j / S_k (S_k = sum of their volumes); V_k = S_k / 12 and
    K = sum_k V_k Bt_k^T C Bt_k with Bt_k = sum_j w_jk B_j(G_k).  Volumes from
    surface integrals (divergence theorem)."""
    X = np.asarray(X, float)
    hexes = np.asarray(hexes)
    N = len(X)
    C = cmat(E, nu)
    Vs = [hex_surface_integrals(X[h])[1] for h in hexes]
    patches = {}
    for j, h in enumerate(hexes):
        for q, (a, b) in enumerate(_HEX_EDGES):
            patches.setdefault(tuple(sorted((int(h[a]), int(h[b])))), []).append((j, q))
    dof = lambda nd: np.array([[3 * n, 3 * n + 1, 3 * n + 2] for n in nd]).ravel()
    K = np.zeros((3 * N, 3 * N))
    for pj in patches.values():
        S = sum(Vs[j] for j, _ in pj)
        Bt = np.zeros((6, 3 * N))
        for j, q in pj:
            a, b = _HEX_EDGES[q]
            G = 0.5 * (_HEX_SIGN[a] + _HEX_SIGN[b])   # midpoint of the edge
            Bt[:, dof(hexes[j])] += (Vs[j] / S) * _hex_B(hex_gradients_at(X[hexes[j]], G))
        K += (S / 12.0) * Bt.T @ C @ Bt
    return K, np.array(Vs)
