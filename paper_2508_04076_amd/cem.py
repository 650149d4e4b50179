"""Python binding of libcem (include/cem.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels of libcem.so; this module
only converts numpy arrays to pointers and back, and uses PyTorch for the HIP
stream (and optionally to own the state buffers).  If the shared library is
missing, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcem.so")

CEM_OK, CEM_EINVAL, CEM_ENOMEM, CEM_EHIP, CEM_EMESH, CEM_ECAPACITY, CEM_EUNSTABLE, CEM_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {-1: "CEM_EINVAL", -2: "CEM_ENOMEM", -3: "CEM_EHIP", -4: "CEM_EMESH",
               -5: "CEM_ECAPACITY", -6: "CEM_EUNSTABLE", -7: "CEM_ESTATE"}
PRECISION = {"fp64": 0, "mixed": 1}
SPLIT_MODE = {"phantom": 0, "erode": 1}
GSIG = {"principal": 0, "normal": 1}
LAYOUT = {"terms": 0, "stress_sums": 1, "tiles": 2, "tiles_fx": 3}

EXPORTS = [
    "cem_create", "cem_destroy", "cem_last_error", "cem_upload_mesh", "cem_upload_hex_mesh",
    "cem_set_traction",
    "cem_presplit", "cem_critical_dt", "cem_set_dt", "cem_bind_state", "cem_set_state",
    "cem_get_state", "cem_internal_force", "cem_step", "cem_replay_splits", "cem_read_energy",
    "cem_read_splits", "cem_read_front_G", "cem_save_state", "cem_load_state", "cem_counts",
    "cem_set_profiling", "cem_set_topology_mode", "cem_kernel_times", "cem_set_instances", "cem_set_dt_instances",
    "cem_critical_dt_instances", "cem_read_energy_instances", "cem_set_launch", "cem_autotune",
    "cem_add_velocity_bc", "cem_read_reactions", "cem_set_modulus", "cem_set_step",
    "cem_window_forward", "cem_window_backward", "cem_window_times", "cem_strain_energy_grad",
    "cem_set_precision", "cem_set_graph_steps", "cem_last_run", "cem_read_front_G_static",
    "cem_node_rows",
]


class cem_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("precision", C.c_int32),
                ("split_mode", C.c_int32), ("gsig", C.c_int32), ("max_splits", C.c_int32),
                ("graph_steps", C.c_int32)]


class cem_material(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double), ("Gc", C.c_double)]


class cem_energy(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("KE", C.c_double), ("SE", C.c_double),
                ("Wext", C.c_double), ("Ud", C.c_double), ("Gmax", C.c_double),
                ("n_split", C.c_int32), ("n_front", C.c_int32), ("n_nodes", C.c_int32),
                ("n_elems", C.c_int32)]


class cem_split_event(C.Structure):
    _fields_ = [("step", C.c_int32), ("tet", C.c_int32), ("side_mask", C.c_int32),
                ("pattern", C.c_int32), ("G", C.c_double)]


class cem_front_g(C.Structure):
    _fields_ = [("tet", C.c_int32), ("face", C.c_int32), ("lone", C.c_int32), ("pad", C.c_int32),
                ("G_I", C.c_double), ("G_II", C.c_double)]


class CemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library(path=LIB_PATH):
    """Load libcem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2508_04076_amd/build.py")
    # PyTorch ships its own HIP runtime.  Load it first so that libcem binds to
    # that same runtime instance: two HIP runtimes in one process cannot share
    # the device.
    import torch  # noqa: F401
    L = C.CDLL(path)
    p, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "cem_create": [C.POINTER(cem_options), C.POINTER(C.c_void_p)],
        "cem_destroy": [p],
        "cem_last_error": [p],
        "cem_upload_mesh": [p, i32, p, i32, p, C.POINTER(cem_material)],
        "cem_upload_hex_mesh": [p, i32, p, i32, p, C.POINTER(cem_material)],
        "cem_set_traction": [p, i32, p, p, d],
        "cem_presplit": [p, i32, p, p],
        "cem_critical_dt": [p, C.POINTER(C.c_double)],
        "cem_set_dt": [p, d],
        "cem_bind_state": [p, p, p, i64],
        "cem_set_state": [p, p, p],
        "cem_get_state": [p, p, p, p, C.POINTER(C.c_int32)],
        "cem_internal_force": [p, p, p],
        "cem_step": [p, i32],
        "cem_replay_splits": [p, i32, p],
        "cem_read_energy": [p, C.POINTER(cem_energy)],
        "cem_read_splits": [p, i32, p, C.POINTER(C.c_int32)],
        "cem_read_front_G": [p, i32, p, C.POINTER(C.c_int32)],
        "cem_save_state": [p, p, i64, C.POINTER(C.c_int64)],
        "cem_load_state": [p, p, i64],
        "cem_counts": [p, p],
        "cem_set_profiling": [p, i32],
        "cem_set_topology_mode": [p, i32],
        "cem_kernel_times": [p, p],
        "cem_set_instances": [p, i32, p, p],
        "cem_set_dt_instances": [p, p],
        "cem_critical_dt_instances": [p, p],
        "cem_read_energy_instances": [p, i32, p],
        "cem_set_launch": [p, i32, i32, i32],
        "cem_autotune": [p, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                         C.POINTER(C.c_int32), C.POINTER(C.c_double)],
        "cem_set_modulus": [p, i32, p],
        "cem_set_step": [p, i64],
        "cem_add_velocity_bc": [p, i32, p, p, p, d, C.POINTER(C.c_int32)],
        "cem_read_reactions": [p, i32, i32, p, C.POINTER(C.c_int32), C.POINTER(C.c_double)],
        "cem_window_forward": [p, i32, i32],
        "cem_window_backward": [p, p, p, p, p, p],
        "cem_window_times": [p, p],
        "cem_strain_energy_grad": [p, p, C.POINTER(C.c_double), p, p],
        "cem_set_precision": [p, i32],
        "cem_set_graph_steps": [p, i32],
        "cem_last_run": [p, p],
        "cem_read_front_G_static": [p, i32, p, C.POINTER(C.c_int32)],
        "cem_node_rows": [p, i32, p],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.cem_destroy.restype = None
    L.cem_last_error.restype = C.c_char_p
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(shape)


class Simulation:
    """One ES-T-FEM crack-element simulation on one GPU (a libcem context)."""

    def __init__(self, X, tets, material, precision="fp64", split_mode="phantom",
                 gsig="principal", max_splits=None, graph_steps=0, device=0, stream=None,
                 hexes=False):
        """tets: [T, 4] tetrahedra, or [H, 8] trilinear hexahedra with hexes=True."""
        self.lib = load_library()
        self.ctx = None
        X = _f64(X, (-1, 3))
        tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 8 if hexes else 4)
        if max_splits is None:  # a hex cracks at most once
            max_splits = len(tets) if hexes else max(len(tets) // 8, 64)
        self._torch_stream = None
        if stream is None:
            import torch
            self._torch_stream = torch.cuda.Stream(device=device)
            stream = self._torch_stream.cuda_stream
        opt = cem_options(int(device), C.c_void_p(int(stream)), PRECISION[precision],
                          SPLIT_MODE[split_mode], GSIG[gsig], int(max_splits), int(graph_steps))
        ctx = C.c_void_p()
        r = self.lib.cem_create(C.byref(opt), C.byref(ctx))
        if r != 0:
            raise CemError(r, "cem_create rejected the options")
        self.ctx = ctx
        mat = cem_material(float(material["E"]), float(material["nu"]), float(material["rho"]),
                           float(material.get("Gc", np.inf)))
        upload = self.lib.cem_upload_hex_mesh if hexes else self.lib.cem_upload_mesh
        self._chk(upload(self.ctx, len(X), _p(X), len(tets), _p(tets), C.byref(mat)))
        self.n_tets = len(tets)
        self.n_nodes0 = len(X)
        self.precision = precision

    @classmethod
    def from_mesh(cls, mesh, material, presplit=True, traction=True, ramp_t0=0.0, Gc=None,
                  E_tet=None, **kw):
        mat = dict(material)
        if Gc is not None:
            mat["Gc"] = Gc
        sim = cls(mesh.X, mesh.tets, mat, **kw)
        if E_tet is not None:
            sim.set_modulus(E_tet)
        if traction and mesh.load_tris is not None:
            sim.set_traction(mesh.load_tris, mesh.load_trac, ramp_t0)
        if presplit and mesh.presplit_tets is not None:
            sim.presplit(mesh.presplit_tets, mesh.presplit_masks)
        return sim

    @classmethod
    def from_hex_mesh(cls, mesh, material, traction=True, ramp_t0=0.0, Gc=None, presplit=True,
                      **kw):
        """Simulation of a trilinear hexahedral mesh (meshgen.HexMesh); cracks
        grow from the mesh's precracked hexes (crack plane indices)."""
        mat = dict(material)
        if Gc is not None:
            mat["Gc"] = Gc
        sim = cls(mesh.X, mesh.hexes, mat, hexes=True, **kw)
        if traction and mesh.load_tris is not None:
            sim.set_traction(mesh.load_tris, mesh.load_trac, ramp_t0)
        if presplit and getattr(mesh, "precrack_hexes", None) is not None:
            sim.presplit(mesh.precrack_hexes, mesh.precrack_planes)
        return sim

    def close(self):
        if self.ctx is not None:
            self.lib.cem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, r):
        if r != 0:
            msg = self.lib.cem_last_error(self.ctx) if self.ctx is not None else b""
            raise CemError(r, (msg or b"").decode())

    def set_traction(self, tri, t, ramp_t0=0.0):
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        t = _f64(t, (-1, 3))
        self._chk(self.lib.cem_set_traction(self.ctx, len(tri), _p(tri), _p(t), float(ramp_t0)))

    def presplit(self, tets, masks):
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        masks = np.ascontiguousarray(masks, dtype=np.uint8)
        self._chk(self.lib.cem_presplit(self.ctx, len(tets), _p(tets), _p(masks)))

    def critical_dt(self):
        d = C.c_double()
        self._chk(self.lib.cem_critical_dt(self.ctx, C.byref(d)))
        return d.value

    def set_dt(self, dt):
        self._chk(self.lib.cem_set_dt(self.ctx, float(dt)))

    def set_precision(self, precision):
        """Switch the force arithmetic ("fp64" or "mixed") keeping mesh and state."""
        self._chk(self.lib.cem_set_precision(self.ctx, PRECISION[precision]))
        self.precision = precision

    def set_graph_steps(self, k):
        """Steps per captured HIP graph from now on (0: plain launches)."""
        self._chk(self.lib.cem_set_graph_steps(self.ctx, int(k)))

    def last_run(self):
        """How the last step() call ran: steps, graph launches, steps per graph,
        steps as plain launches."""
        out = np.zeros(4, dtype=np.int64)
        self._chk(self.lib.cem_last_run(self.ctx, _p(out)))
        return dict(steps=int(out[0]), graph_launches=int(out[1]), graph_steps=int(out[2]),
                    plain_steps=int(out[3]))

    def counts(self):
        out = np.zeros(6, dtype=np.int32)
        self._chk(self.lib.cem_counts(self.ctx, _p(out)))
        return dict(nodes=int(out[0]), elems=int(out[1]), edges=int(out[2]), splits=int(out[3]),
                    fronts=int(out[4]), edges0=int(out[5]))

    @property
    def n_nodes(self):
        return self.counts()["nodes"]

    def bind_state(self, u, v):
        """Work in caller device tensors u, v of shape [capacity, 4] float64
        (rows in the internal node order, see node_rows); they must outlive
        the simulation."""
        for x in (u, v):
            if x.dtype.itemsize != 8 or x.dim() != 2 or x.shape[1] != 4 or not x.is_contiguous():
                raise ValueError("bind_state needs contiguous [capacity, 4] float64 tensors")
        self._chk(self.lib.cem_bind_state(self.ctx, C.c_void_p(u.data_ptr()),
                                          C.c_void_p(v.data_ptr()), int(min(u.shape[0], v.shape[0]))))
        self._bound = (u, v)

    def node_rows(self, n=None):
        """Internal row of each caller node (the first n nodes now)."""
        n = self.n_nodes if n is None else n
        out = np.zeros(n, dtype=np.int32)
        self._chk(self.lib.cem_node_rows(self.ctx, int(n), _p(out)))
        return out

    def set_state(self, u=None, v=None):
        n = self.n_nodes
        uu = None if u is None else _f64(u, (n, 3))
        vv = None if v is None else _f64(v, (n, 3))
        self._chk(self.lib.cem_set_state(self.ctx, _p(uu), _p(vv)))

    def get_state(self):
        n = self.n_nodes
        u, v, a = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros((n, 3))
        nn = C.c_int32()
        self._chk(self.lib.cem_get_state(self.ctx, _p(u), _p(v), _p(a), C.byref(nn)))
        return u, v, a

    def internal_force(self, u):
        n = self.n_nodes
        u = _f64(u, (n, 3))
        f = np.zeros((n, 3))
        self._chk(self.lib.cem_internal_force(self.ctx, _p(u), _p(f)))
        return f

    def step(self, n):
        self._chk(self.lib.cem_step(self.ctx, int(n)))

    def replay_splits(self, ev):
        ev = np.asarray(ev, dtype=np.int32).reshape(-1, 3)
        arr = (cem_split_event * max(len(ev), 1))()
        for i, (s, t, m) in enumerate(ev.tolist()):
            arr[i] = cem_split_event(s, t, m, 0, 0.0)
        self._chk(self.lib.cem_replay_splits(self.ctx, len(ev), C.cast(arr, C.c_void_p)))

    def energy(self):
        e = cem_energy()
        self._chk(self.lib.cem_read_energy(self.ctx, C.byref(e)))
        return {k: getattr(e, k) for k, _ in cem_energy._fields_}

    def splits(self):
        n = C.c_int32()
        self._chk(self.lib.cem_read_splits(self.ctx, 0, None, C.byref(n)))
        arr = (cem_split_event * max(n.value, 1))()
        self._chk(self.lib.cem_read_splits(self.ctx, n.value, C.cast(arr, C.c_void_p), C.byref(n)))
        ev = np.array([[a.step, a.tet, a.side_mask, a.pattern] for a in arr[: n.value]],
                      dtype=np.int32).reshape(-1, 4)
        G = np.array([a.G for a in arr[: n.value]], dtype=np.float64)
        return ev, G

    def front_G(self):
        n = C.c_int32()
        self._chk(self.lib.cem_read_front_G(self.ctx, 0, None, C.byref(n)))
        arr = (cem_front_g * max(n.value, 1))()
        self._chk(self.lib.cem_read_front_G(self.ctx, n.value, C.cast(arr, C.c_void_p), C.byref(n)))
        tfl = np.array([[a.tet, a.face, a.lone] for a in arr[: n.value]], dtype=np.int32).reshape(-1, 3)
        g = np.array([[a.G_I, a.G_II] for a in arr[: n.value]], dtype=np.float64).reshape(-1, 2)
        return tfl, g

    def front_G_static(self):
        """front_G through the allocation-free entry point (static staging)."""
        n = C.c_int32()
        self._chk(self.lib.cem_read_front_G_static(self.ctx, 0, None, C.byref(n)))
        arr = (cem_front_g * max(n.value, 1))()
        self._chk(self.lib.cem_read_front_G_static(self.ctx, n.value, C.cast(arr, C.c_void_p),
                                                   C.byref(n)))
        tfl = np.array([[a.tet, a.face, a.lone] for a in arr[: n.value]], dtype=np.int32).reshape(-1, 3)
        g = np.array([[a.G_I, a.G_II] for a in arr[: n.value]], dtype=np.float64).reshape(-1, 2)
        return tfl, g

    def save_state(self):
        used = C.c_int64()
        self._chk(self.lib.cem_save_state(self.ctx, None, 0, C.byref(used)))
        buf = np.zeros(used.value, dtype=np.uint8)
        self._chk(self.lib.cem_save_state(self.ctx, _p(buf), used.value, C.byref(used)))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._chk(self.lib.cem_load_state(self.ctx, _p(buf), len(buf)))

    def set_topology_mode(self, mode):
        """0 automatic, 1 one workgroup, 2 whole chip for split batches over 128."""
        self._chk(self.lib.cem_set_topology_mode(self.ctx, {"auto": 0, "single": 1, "chip": 2}.get(mode, mode)))

    def set_profiling(self, on=True):
        self._chk(self.lib.cem_set_profiling(self.ctx, 1 if on else 0))

    def kernel_times(self):
        out = np.zeros(7)
        self._chk(self.lib.cem_kernel_times(self.ctx, _p(out)))
        d = dict(zip(["total", "strain", "edge_stress", "front", "elem_force", "node_sum",
                      "topology"], out.tolist()))
        d["node"] = d["elem_force"] + d["node_sum"]
        return d

    # ---- batches
    def set_instances(self, node_off, tet_off):
        node_off = np.ascontiguousarray(node_off, dtype=np.int32)
        tet_off = np.ascontiguousarray(tet_off, dtype=np.int32)
        self.n_inst = len(node_off) - 1
        self._chk(self.lib.cem_set_instances(self.ctx, self.n_inst, _p(node_off), _p(tet_off)))

    def set_dt_instances(self, dt):
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        self._chk(self.lib.cem_set_dt_instances(self.ctx, _p(dt)))

    def critical_dt_instances(self):
        out = np.zeros(self.n_inst)
        self._chk(self.lib.cem_critical_dt_instances(self.ctx, _p(out)))
        return out

    def energy_instances(self):
        arr = (cem_energy * self.n_inst)()
        self._chk(self.lib.cem_read_energy_instances(self.ctx, self.n_inst,
                                                     C.cast(arr, C.c_void_p)))
        return [{k: getattr(e, k) for k, _ in cem_energy._fields_} for e in arr]

    def set_launch(self, grid_cap, lanes, layout="terms"):
        """Launch shape; layout "terms" or "stress_sums" (what the tet force
        pass hands to the node pass)."""
        self._chk(self.lib.cem_set_launch(self.ctx, int(grid_cap), int(lanes), LAYOUT[layout]))

    def autotune(self, trial_steps=10):
        g, l, lay, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._chk(self.lib.cem_autotune(self.ctx, int(trial_steps), C.byref(g), C.byref(l),
                                        C.byref(lay), C.byref(ms)))
        name = {v: k for k, v in LAYOUT.items()}[lay.value]
        return dict(grid_cap=g.value, lanes=l.value, layout=name, ms_per_step=ms.value)

    # ---- heterogeneous modulus and gradient windows
    def set_modulus(self, E_tet):
        """Young's modulus per tet (Pa, caller order); None: the scalar material E."""
        if E_tet is None:
            self._chk(self.lib.cem_set_modulus(self.ctx, 0, None))
            return
        E = np.ascontiguousarray(E_tet, dtype=np.float64).reshape(-1)
        self._chk(self.lib.cem_set_modulus(self.ctx, len(E), _p(E)))

    def set_step(self, step):
        """Step counter (time = step * dt for the load ramp); the state is kept."""
        self._chk(self.lib.cem_set_step(self.ctx, int(step)))

    def window_forward(self, n_steps, every=50):
        self._chk(self.lib.cem_window_forward(self.ctx, int(n_steps), int(every)))

    def window_backward(self, gu=None, gv=None):
        """(dJ/du0, dJ/dv0, dJ/dE) of J = gu . u_n + gv . v_n over the pending window."""
        n = self.n_nodes
        gu = None if gu is None else _f64(gu, (n, 3))
        gv = None if gv is None else _f64(gv, (n, 3))
        gu0, gv0, gE = np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(self.n_tets)
        self._chk(self.lib.cem_window_backward(self.ctx, _p(gu), _p(gv), _p(gu0), _p(gv0),
                                               _p(gE)))
        return gu0, gv0, gE

    def strain_energy_grad(self, u=None):
        """(SE, dSE/du, dSE/dE at fixed u) at displacement u (None: the current state)."""
        n = self.n_nodes
        uu = None if u is None else _f64(u, (n, 3))
        se = C.c_double()
        gu, gE = np.zeros((n, 3)), np.zeros(self.n_tets)
        self._chk(self.lib.cem_strain_energy_grad(self.ctx, _p(uu), C.byref(se), _p(gu), _p(gE)))
        return se.value, gu, gE

    def window_times(self):
        out = np.zeros(6)
        self._chk(self.lib.cem_window_times(self.ctx, _p(out)))
        return dict(zip(["total", "recompute", "strain2", "edge2", "elem_adj", "node_adj"],
                        out.tolist()))

    # ---- prescribed velocities
    def add_velocity_bc(self, nodes, masks, v0, t0=0.0):
        """One group of prescribed velocities (v0 t/t0 up to t0, then v0) on the
        dof bits of each node's mask; before the first step.  Returns the group id."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int32).reshape(-1)
        masks = np.ascontiguousarray(masks, dtype=np.int32).reshape(-1)
        v0 = _f64(v0, (len(nodes), 3))
        g = C.c_int32()
        self._chk(self.lib.cem_add_velocity_bc(self.ctx, len(nodes), _p(nodes), _p(masks), _p(v0),
                                               float(t0), C.byref(g)))
        return g.value

    def reactions(self, group=0):
        """(rows [n][6]: step, t, R_x, R_y, R_z, S(t); the group's reaction work)."""
        n, w = C.c_int32(), C.c_double()
        self._chk(self.lib.cem_read_reactions(self.ctx, int(group), 0, None, C.byref(n), None))
        rows = np.zeros((max(n.value, 1), 6))
        self._chk(self.lib.cem_read_reactions(self.ctx, int(group), n.value, _p(rows), C.byref(n),
                                              C.byref(w)))
        return rows[: n.value], w.value
