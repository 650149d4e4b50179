"""ctypes wrapper of the oracle library -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.cpp")

_i = C.c_int
_d = C.c_double
_p = C.c_void_p


def build(force=False):
    """Compile the oracle with g++ (plain FP64, no fused multiply-add)."""
    stale = not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "oracle.h")))
    if force or stale:
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-ffp-contract=off",
               "-o", LIB + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.orc_create.restype = _p
        L.orc_create.argtypes = [_i, _p, _i, _p, _d, _d, _d, _d, _i, _i]
        L.orc_create_hex.restype = _p
        L.orc_create_hex.argtypes = [_i, _p, _i, _p, _d, _d, _d, _d, _i]
        L.orc_error.restype = C.c_char_p
        L.orc_error.argtypes = [_p]
        L.orc_create_status.argtypes = [_p]
        L.orc_destroy.argtypes = [_p]
        L.orc_destroy.restype = None
        for name, args in [
            ("orc_set_traction", [_p, _i, _p, _p, _d]),
            ("orc_presplit", [_p, _i, _p, _p]),
            ("orc_critical_dt", [_p, _p]),
            ("orc_set_dt", [_p, _d]),
            ("orc_counts", [_p, _p]),
            ("orc_set_state", [_p, _p, _p]),
            ("orc_get_state", [_p, _p, _p, _p]),
            ("orc_internal_force", [_p, _p, _p]),
            ("orc_step", [_p, _i]),
            ("orc_energy", [_p, _p]),
            ("orc_splits", [_p, _i, _p, _p, _p]),
            ("orc_front_G", [_p, _i, _p, _p, _p]),
            ("orc_replay", [_p, _i, _p]),
            ("orc_masses", [_p, _p]),
            ("orc_loads", [_p, _p]),
            ("orc_elements", [_p, _p, _p, _p, _p]),
            ("orc_grad", [_p, _p]),
            ("orc_edges", [_p, _p, _p, _p, _p]),
            ("orc_elem_lambda_max", [_p, _p]),
            ("orc_sym_eig3", [_p, _p, _p]),
            ("orc_set_modulus", [_p, _p]),
            ("orc_set_frozen", [_p, _i]),
            ("orc_set_threads", [_p, _i]),
            ("orc_window_gradient", [_p, _i, _p, _p, _p, _p, _p]),
            ("orc_add_velocity_bc", [_p, _i, _p, _p, _p, _d, _p]),
            ("orc_strain_energy_grad", [_p, _p, _p]),
            ("orc_reactions", [_p, _i, _i, _p, _p, _p]),
            ("orc_hex_plane_masks", [_p]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = _i
        L.orc_lame.argtypes = [_d, _d, _p, _p]
        L.orc_lame.restype = None
        L.orc_stress_term.argtypes = [_p, _p, _i]
        L.orc_stress_term.restype = _d
        L.orc_crack_area.argtypes = [_p, _i]
        L.orc_crack_area.restype = _d
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


def lame(E, nu):
    lam, mu = C.c_double(), C.c_double()
    lib().orc_lame(E, nu, C.byref(lam), C.byref(mu))
    return lam.value, mu.value


def sym_eig3(sig6):
    s = _f64(sig6)
    w = np.zeros(3)
    v = np.zeros(9)
    lib().orc_sym_eig3(_ptr(s), _ptr(w), _ptr(v))
    return w, v.reshape(3, 3)


def stress_term(sig6, n, gsig=0):
    return lib().orc_stress_term(_ptr(_f64(sig6)), _ptr(_f64(n)), int(gsig))


def crack_area(X4, mask):
    return lib().orc_crack_area(_ptr(_f64(X4)), int(mask))


class Oracle:
    """One simulation of the oracle: mesh, material, loads, state."""

    def __init__(self, X, tets, E, nu, rho, Gc=np.inf, split_mode="phantom", gsig="principal",
                 hexes=False):
        self._X = _f64(X)
        self._t = _i32(tets)
        L = lib()
        if hexes:
            gs = {"principal": 0, "normal": 1}[gsig]
            self.c = L.orc_create_hex(len(self._X), _ptr(self._X), len(self._t), _ptr(self._t),
                                      float(E), float(nu), float(rho), float(Gc), gs)
        else:
            mode = {"phantom": 0, "erode": 1}[split_mode]
            gs = {"principal": 0, "normal": 1}[gsig]
            self.c = L.orc_create(len(self._X), _ptr(self._X), len(self._t), _ptr(self._t),
                                  float(E), float(nu), float(rho), float(Gc), mode, gs)
        st = L.orc_create_status(self.c)
        if st != 0:
            msg = L.orc_error(self.c).decode()
            L.orc_destroy(self.c)
            self.c = None
            raise OracleError(f"oracle create failed ({st}): {msg}")

    def __del__(self):
        if getattr(self, "c", None):
            lib().orc_destroy(self.c)
            self.c = None

    def _chk(self, r):
        if r != 0:
            raise OracleError(lib().orc_error(self.c).decode())

    @classmethod
    def from_mesh(cls, mesh, material, split_mode="phantom", gsig="principal", presplit=True,
                  traction=True, ramp_t0=0.0, Gc=None, E_tet=None):
        o = cls(mesh.X, mesh.tets, material["E"], material["nu"], material["rho"],
                material["Gc"] if Gc is None else Gc, split_mode, gsig)
        if E_tet is not None:
            o.set_modulus(E_tet)
        if traction and mesh.load_tris is not None:
            o.set_traction(mesh.load_tris, mesh.load_trac, ramp_t0)
        if presplit and mesh.presplit_tets is not None:
            o.presplit(mesh.presplit_tets, mesh.presplit_masks)
        return o

    @classmethod
    def hex_mesh(cls, mesh, material, traction=True, ramp_t0=0.0, Gc=None, gsig="principal",
                 presplit=True):
        """Oracle of a trilinear hexahedral mesh; cracks grow from the
        mesh's precracked hexes (crack plane indices)."""
        o = cls(mesh.X, mesh.hexes, material["E"], material["nu"], material["rho"],
                material["Gc"] if Gc is None else Gc, gsig=gsig, hexes=True)
        if traction and mesh.load_tris is not None:
            o.set_traction(mesh.load_tris, mesh.load_trac, ramp_t0)
        if presplit and getattr(mesh, "precrack_hexes", None) is not None:
            o.presplit(mesh.precrack_hexes, mesh.precrack_planes)
        return o

    def hex_plane_masks(self):
        out = np.zeros(23, dtype=np.int32)
        lib().orc_hex_plane_masks(_ptr(out))
        return out

    def set_traction(self, tri, t, ramp_t0=0.0):
        tri, t = _i32(tri), _f64(t)
        self._chk(lib().orc_set_traction(self.c, len(tri), _ptr(tri), _ptr(t), float(ramp_t0)))

    def presplit(self, tets, masks):
        tets = _i32(tets)
        masks = np.ascontiguousarray(masks, dtype=np.uint8)
        self._chk(lib().orc_presplit(self.c, len(tets), _ptr(tets), _ptr(masks)))

    def critical_dt(self):
        d = C.c_double()
        self._chk(lib().orc_critical_dt(self.c, C.byref(d)))
        return d.value

    def set_dt(self, dt):
        self._chk(lib().orc_set_dt(self.c, float(dt)))

    def counts(self):
        out = np.zeros(5, dtype=np.int32)
        lib().orc_counts(self.c, _ptr(out))
        return dict(nodes=int(out[0]), elems=int(out[1]), edges=int(out[2]),
                    splits=int(out[3]), fronts=int(out[4]))

    @property
    def n_nodes(self):
        return self.counts()["nodes"]

    def set_state(self, u=None, v=None):
        n = self.n_nodes
        uu = None if u is None else _f64(u, (n, 3))
        vv = None if v is None else _f64(v, (n, 3))
        self._chk(lib().orc_set_state(self.c, _ptr(uu), _ptr(vv)))

    def get_state(self):
        n = self.n_nodes
        u, v, a = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        self._chk(lib().orc_get_state(self.c, _ptr(u), _ptr(v), _ptr(a)))
        return u, v, a

    def internal_force(self, u):
        n = self.n_nodes
        u = _f64(u, (n, 3))
        f = np.zeros((n, 3))
        self._chk(lib().orc_internal_force(self.c, _ptr(u), _ptr(f)))
        return f

    def step(self, n):
        self._chk(lib().orc_step(self.c, int(n)))

    def energy(self):
        out = np.zeros(10)
        self._chk(lib().orc_energy(self.c, _ptr(out)))
        keys = ["step", "t", "KE", "SE", "Wext", "Ud", "Gmax", "n_split", "n_front", "n_nodes"]
        return dict(zip(keys, out.tolist()))

    def splits(self):
        n = C.c_int()
        lib().orc_splits(self.c, 0, None, None, C.byref(n))
        ev = np.zeros((max(n.value, 1), 4), dtype=np.int32)
        G = np.zeros(max(n.value, 1))
        self._chk(lib().orc_splits(self.c, n.value, _ptr(ev), _ptr(G), C.byref(n)))
        return ev[: n.value], G[: n.value]

    def front_G(self):
        n = C.c_int()
        lib().orc_front_G(self.c, 0, None, None, C.byref(n))
        tfl = np.zeros((max(n.value, 1), 3), dtype=np.int32)
        g = np.zeros((max(n.value, 1), 2))
        self._chk(lib().orc_front_G(self.c, n.value, _ptr(tfl), _ptr(g), C.byref(n)))
        return tfl[: n.value], g[: n.value]

    def set_modulus(self, E_tet):
        """Young's modulus of every original tet (split copies take their parent's)."""
        E = _f64(E_tet)
        if E.shape != (len(self._t),):
            raise OracleError("one modulus per tet")
        self._chk(lib().orc_set_modulus(self.c, _ptr(E)))

    def set_threads(self, n):
        """Threads of the element, edge and node loops; results are bitwise
        the same at any count."""
        self._chk(lib().orc_set_threads(self.c, int(n)))

    def set_frozen(self, on=True):
        self._chk(lib().orc_set_frozen(self.c, int(bool(on))))

    def strain_energy_grad(self, u=None):
        """dSE/dE per tet at fixed u (the explicit part; dSE/du is the internal force)."""
        uu = None if u is None else _f64(u, (self.n_nodes, 3))
        gE = np.zeros(len(self._t))
        self._chk(lib().orc_strain_energy_grad(self.c, _ptr(uu), _ptr(gE)))
        return gE

    def window_gradient(self, n_steps, gu=None, gv=None):
        """Run n fixed-topology steps; return (dJ/du0, dJ/dv0, dJ/dE) for
        J = gu . u_n + gv . v_n.  The state is left at the end of the window."""
        n = self.n_nodes
        gu = None if gu is None else _f64(gu, (n, 3))
        gv = None if gv is None else _f64(gv, (n, 3))
        gu0, gv0 = np.zeros((n, 3)), np.zeros((n, 3))
        gE = np.zeros(len(self._t))
        self._chk(lib().orc_window_gradient(self.c, int(n_steps), _ptr(gu), _ptr(gv), _ptr(gu0),
                                            _ptr(gv0), _ptr(gE)))
        return gu0, gv0, gE

    def add_velocity_bc(self, nodes, masks, v0, t0=0.0):
        """One group of prescribed velocities v0 (t/t0 ramp, then constant) on
        the dof bits of each node's mask; before the first step.  Returns the
        group id."""
        nodes, masks = _i32(nodes), _i32(masks)
        v0 = _f64(v0, (len(nodes), 3))
        g = C.c_int()
        self._chk(lib().orc_add_velocity_bc(self.c, len(nodes), _ptr(nodes), _ptr(masks), _ptr(v0),
                                            float(t0), C.byref(g)))
        return g.value

    def reactions(self, group=0):
        """(rows [n][6]: step, t, R_x, R_y, R_z, S(t); work of the group's reactions)."""
        n = C.c_int()
        w = C.c_double()
        self._chk(lib().orc_reactions(self.c, int(group), 0, None, C.byref(n), None))
        rows = np.zeros((max(n.value, 1), 6))
        self._chk(lib().orc_reactions(self.c, int(group), n.value, _ptr(rows), C.byref(n),
                                      C.byref(w)))
        return rows[: n.value], w.value

    def replay(self, ev3):
        ev3 = _i32(ev3).reshape(-1, 3)
        self._chk(lib().orc_replay(self.c, len(ev3), _ptr(ev3)))

    def masses(self):
        m = np.zeros(self.n_nodes)
        lib().orc_masses(self.c, _ptr(m))
        return m

    def loads(self):
        F = np.zeros((self.n_nodes, 3))
        lib().orc_loads(self.c, _ptr(F))
        return F

    def elements(self):
        ne = self.counts()["elems"]
        nodes = np.zeros((ne, 4), dtype=np.int32)
        Veff, V = np.zeros(ne), np.zeros(ne)
        parent = np.zeros(ne, dtype=np.int32)
        lib().orc_elements(self.c, _ptr(nodes), _ptr(Veff), _ptr(V), _ptr(parent))
        return dict(nodes=nodes, Veff=Veff, V=V, parent=parent)

    def grad(self):
        ne = self.counts()["elems"]
        g = np.zeros((ne, 4, 3))
        lib().orc_grad(self.c, _ptr(g))
        return g

    def edges(self, u=None):
        nE = self.counts()["edges"]
        nodes = np.zeros((nE, 2), dtype=np.int32)
        eps, sig = np.zeros((nE, 6)), np.zeros((nE, 6))
        uu = None if u is None else _f64(u, (self.n_nodes, 3))
        lib().orc_edges(self.c, _ptr(uu), _ptr(nodes), _ptr(eps), _ptr(sig))
        return nodes, eps, sig

    def elem_lambda_max(self):
        T0 = len(self._t)
        lam = np.zeros(T0)
        lib().orc_elem_lambda_max(self.c, _ptr(lam))
        return lam
