"""Seeded synthetic inputs shared by the HIP path, the oracle and the benches.

This module holds no arithmetic of the method: it only lays out structured
"Kuhn" tetrahedral grids, picks which tetrahedra form the pre-notch and on
which side of the notch each of their nodes lies, and lists the loaded
boundary triangles with their traction vectors.  Everything the method
computes from these arrays (volumes, gradients, masses, nodal loads, time
step) is computed separately by the GPU library and by the oracle.

The paper's benchmark meshes (Section 4.4, crack branching under tractions:
a 100 x 40 x 4 mm plate with a 50 mm edge notch at mid-height) are shown only
as figures, so structured grids of the same geometry stand in for them.  Each
hexahedral cell is cut into the six tetrahedra that follow the monotone lattice
paths from its lowest to its highest corner; every cube face is then split by
the diagonal through its lowest corner, so the grid is conforming.

Arrays follow the library's conventions: node coordinates float64 [N, 3],
tetrahedra int32 [T, 4] (positively oriented), 0-based ids.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np

# The six monotone paths through the unit cube, one per axis permutation.
_PERMS = list(itertools.permutations(range(3)))
_UNIT = np.eye(3, dtype=np.int64)


@dataclasses.dataclass
class Mesh:
    """A tetrahedral mesh plus the pieces of a benchmark set-up."""
    X: np.ndarray               # [N, 3] float64 node coordinates (m)
    tets: np.ndarray            # [T, 4] int32 node ids
    grid: tuple = None          # (nx, ny, nz) cell counts for structured grids
    h: tuple = None             # (hx, hy, hz) cell sizes
    presplit_tets: np.ndarray = None   # [P] int32 tet ids of the pre-notch
    presplit_masks: np.ndarray = None  # [P] uint8, bit l: local node l on side B
    load_tris: np.ndarray = None       # [F, 3] int32 loaded boundary triangles
    load_trac: np.ndarray = None       # [F, 3] float64 traction vectors (Pa)

    @property
    def n_nodes(self):
        return int(self.X.shape[0])

    @property
    def n_tets(self):
        return int(self.tets.shape[0])


def node_id(i, j, k, nx, ny):
    return i + (nx + 1) * (j + (ny + 1) * k)


def kuhn_box(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Structured grid of nx*ny*nz cells over [0,lx]x[0,ly]x[0,lz].

    Tet order: cell-major (cells in x-fastest order), six tets per cell in
    the fixed permutation order; every tet has a positive signed volume.
    """
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1),
                             np.arange(nz + 1), indexing="ij")
    # node id = i + (nx+1)*(j + (ny+1)*k): x fastest
    X = np.empty(((nx + 1) * (ny + 1) * (nz + 1), 3), dtype=np.float64)
    ids = node_id(ii, jj, kk, nx, ny).ravel()
    X[ids, 0] = (ii * hx).ravel()
    X[ids, 1] = (jj * hy).ravel()
    X[ids, 2] = (kk * hz).ravel()
    # the exact upper bounds, so boundary planes are exact
    X[ids[(ii == nx).ravel()], 0] = lx
    X[ids[(jj == ny).ravel()], 1] = ly
    X[ids[(kk == nz).ravel()], 2] = lz

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    # cell order x-fastest
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    ncell = ci.size
    tets = np.empty((ncell, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        corners = [np.zeros(3, dtype=np.int64)]
        for a in perm:
            corners.append(corners[-1] + _UNIT[a])
        # parity of the permutation decides the orientation of the path tet
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        if inv % 2 == 1:
            corners[2], corners[3] = corners[3], corners[2]
        for l, c in enumerate(corners):
            tets[:, p, l] = node_id(ci + c[0], cj + c[1], ck + c[2], nx, ny)
    mesh = Mesh(X=X, tets=tets.reshape(-1, 4).astype(np.int32),
                grid=(nx, ny, nz), h=(hx, hy, hz))
    return mesh


def kuhn_counts(nx, ny, nz):
    """Closed-form node / tet / edge / face counts of a Kuhn grid."""
    n = (nx + 1) * (ny + 1) * (nz + 1)
    t = 6 * nx * ny * nz
    axis = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    diag = nx * ny * (nz + 1) + nx * (ny + 1) * nz + (nx + 1) * ny * nz
    body = nx * ny * nz
    e = axis + diag + body
    # faces: each tet has 4, interior faces are shared by two
    bnd = 4 * (nx * ny + ny * nz + nx * nz)
    f = (4 * t + bnd) // 2
    return dict(nodes=n, tets=t, edges=e, faces=f, boundary_faces=bnd)


def cell_of_tet(mesh):
    """(i, j, k) cell index of every tet of a kuhn_box mesh (before permutation)."""
    nx, ny, nz = mesh.grid
    c = np.arange(mesh.n_tets) // 6
    return c % nx, (c // nx) % ny, c // (nx * ny)


def notch_presplit(mesh, axis_normal, plane_index, axis_len, len_cells, layers_below=1,
                   layers_above=0):
    """Pre-notch as pre-split tets.

    The notch plane is the grid plane `axis_normal` = plane_index (a cell
    boundary); it spans cells with index < len_cells along axis `axis_len` and
    the whole grid along the third axis.  The cut cell layers are the
    `layers_below` layers under the plane and `layers_above` layers over it.
    Each tet in a cut layer is partitioned by the level of its nodes inside
    its own layer: the nodes on the upper face of the layer form side B.  For
    the single layer directly below the plane this is "below the plane" versus
    "on the plane".  Every Kuhn tet crosses its layer once, so each partition
    is 1|3, 2|2 or 3|1.
    """
    cidx = cell_of_tet(mesh)
    cn = cidx[axis_normal]
    cl = cidx[axis_len]
    lo = plane_index - layers_below
    hi = plane_index + layers_above
    sel = np.nonzero((cn >= lo) & (cn < hi) & (cl < len_cells))[0]
    nx, ny, nz = mesh.grid
    # integer lattice coordinate of each node along the normal axis
    nid = mesh.tets[sel].astype(np.int64)
    if axis_normal == 0:
        lev = nid % (nx + 1)
    elif axis_normal == 1:
        lev = (nid // (nx + 1)) % (ny + 1)
    else:
        lev = nid // ((nx + 1) * (ny + 1))
    upper = lev > cn[sel][:, None]
    masks = (upper * (1 << np.arange(4))).sum(axis=1).astype(np.uint8)
    return sel.astype(np.int32), masks


def face_triangles(mesh, axis, side):
    """Boundary triangles on the grid face axis=min (side 0) or axis=max (side 1).

    Each boundary square is split by the diagonal through its lowest corner,
    which is the diagonal the Kuhn tets use, so every triangle is a tet face.
    """
    nx, ny, nz = mesh.grid
    n = [nx, ny, nz]
    a, b = [d for d in range(3) if d != axis]
    lvl = 0 if side == 0 else n[axis]
    ia, ib = np.meshgrid(np.arange(n[a]), np.arange(n[b]), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()

    def nid(da, db):
        c = [None, None, None]
        c[axis] = np.full_like(ia, lvl)
        c[a] = ia + da
        c[b] = ib + db
        return node_id(c[0], c[1], c[2], nx, ny)

    t1 = np.stack([nid(0, 0), nid(1, 0), nid(1, 1)], axis=1)
    t2 = np.stack([nid(0, 0), nid(0, 1), nid(1, 1)], axis=1)
    return np.concatenate([t1, t2]).astype(np.int32)


def add_tension(mesh, axis, traction_pa):
    """Opposite tractions +t on the max face and -t on the min face of `axis`."""
    top = face_triangles(mesh, axis, 1)
    bot = face_triangles(mesh, axis, 0)
    tv = np.zeros(3)
    tv[axis] = traction_pa
    mesh.load_tris = np.concatenate([top, bot]).astype(np.int32)
    mesh.load_trac = np.concatenate([np.tile(tv, (len(top), 1)),
                                     np.tile(-tv, (len(bot), 1))])
    return mesh


def jitter(mesh, amount=0.2, seed=0):
    """Move interior nodes by U(-amount, amount) * h per axis (seeded)."""
    rng = np.random.default_rng(seed)
    X = mesh.X
    lo, hi = X.min(axis=0), X.max(axis=0)
    interior = np.all((X > lo + 1e-12) & (X < hi - 1e-12), axis=1)
    h = np.asarray(mesh.h)
    d = rng.uniform(-amount, amount, size=X.shape) * h
    Xn = X.copy()
    Xn[interior] += d[interior]
    mesh.X = Xn
    return mesh


def permute(mesh, seed=1):
    """Random relabelling of nodes and tets (seeded); the geometry is unchanged."""
    rng = np.random.default_rng(seed)
    N, T = mesh.n_nodes, mesh.n_tets
    pn = rng.permutation(N)          # new id of old node i is inv... see below
    old_of_new = pn
    new_of_old = np.empty(N, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(N)
    pt = rng.permutation(T)          # new tet t is old tet pt[t]
    new_tet_of_old = np.empty(T, dtype=np.int64)
    new_tet_of_old[pt] = np.arange(T)
    X = mesh.X[old_of_new]
    tets = new_of_old[mesh.tets[pt]].astype(np.int32)
    out = Mesh(X=X, tets=tets, grid=None, h=mesh.h)
    if mesh.presplit_tets is not None:
        out.presplit_tets = new_tet_of_old[mesh.presplit_tets].astype(np.int32)
        out.presplit_masks = mesh.presplit_masks.copy()
        o = np.argsort(out.presplit_tets)
        out.presplit_tets = out.presplit_tets[o]
        out.presplit_masks = out.presplit_masks[o]
    if mesh.load_tris is not None:
        out.load_tris = new_of_old[mesh.load_tris].astype(np.int32)
        out.load_trac = mesh.load_trac.copy()
    out.node_new_of_old = new_of_old
    out.tet_new_of_old = new_tet_of_old
    return out


# --------------------------------------------------------------------------
# Benchmark set-ups.  Material of the crack-branching example (Section 4.4):
# E = 32 GPa, nu = 0.2, rho = 2450 kg/m^3, Gc = 3 J/m^2, 1 MPa traction.
# --------------------------------------------------------------------------
BRANCHING_MATERIAL = dict(E=32e9, nu=0.2, rho=2450.0, Gc=3.0)


def cube_notched(n=10, traction=1e6):
    """Unit cube of n^3 cells, half-plane notch z = 0.5 over x < 0.3,
    +-traction in z on the z faces (step load).  n=10: 6,000 tets."""
    m = kuhn_box(n, n, n, 1.0, 1.0, 1.0)
    m.presplit_tets, m.presplit_masks = notch_presplit(
        m, axis_normal=2, plane_index=n // 2, axis_len=0, len_cells=int(round(0.3 * n)))
    add_tension(m, 2, traction)
    return m


def plate_notched(nx=200, ny=80, nz=8, lx=0.1, ly=0.04, lz=0.004, notch_len=0.05,
                  traction=1e6, layers_below=1, layers_above=0):
    """Pre-notched plate: edge notch at mid-height y = ly/2 from x = 0 to notch_len,
    through the thickness; +-traction in y on the y faces.  Defaults: the
    100 x 40 x 4 mm plate at 0.5 mm cells, 768,000 tets."""
    m = kuhn_box(nx, ny, nz, lx, ly, lz)
    m.presplit_tets, m.presplit_masks = notch_presplit(
        m, axis_normal=1, plane_index=ny // 2, axis_len=0,
        len_cells=int(round(notch_len / lx * nx)), layers_below=layers_below,
        layers_above=layers_above)
    add_tension(m, 1, traction)
    return m


def block_notched(nx=400, ny=200, nz=100, h=0.5e-3, traction=1e6):
    """Large notched block: 400 x 200 x 100 cells at 0.5 mm (48,000,000 tets),
    notch plane y = 50 mm over x < 100 mm with four cut layers on each side
    (960,000 pre-split tets, 2% of the mesh)."""
    m = kuhn_box(nx, ny, nz, nx * h, ny * h, nz * h)
    m.presplit_tets, m.presplit_masks = notch_presplit(
        m, axis_normal=1, plane_index=ny // 2, axis_len=0, len_cells=nx // 2,
        layers_below=4, layers_above=4)
    add_tension(m, 1, traction)
    return m


def bar(n=100, lx=1.0, w=0.01):
    """Slender bar of n x 1 x 1 cells along x (for wave-speed checks)."""
    return kuhn_box(n, 1, 1, lx, w, w)


def random_displacement(n_nodes, scale=1e-6, seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_nodes, 3)) * scale


def union(meshes):
    """Disjoint union of meshes (a batch).  Returns the union mesh and the node
    and tet offsets of each member (member i owns nodes [node_off[i],
    node_off[i+1]) and tets [tet_off[i], tet_off[i+1]))."""
    node_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    tet_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    for i, mm in enumerate(meshes):
        node_off[i + 1] = node_off[i] + mm.n_nodes
        tet_off[i + 1] = tet_off[i] + mm.n_tets
    X = np.concatenate([mm.X for mm in meshes])
    tets = np.concatenate([mm.tets.astype(np.int64) + node_off[i] for i, mm in enumerate(meshes)])
    out = Mesh(X=X, tets=tets.astype(np.int32))
    ps = [mm.presplit_tets.astype(np.int64) + tet_off[i] for i, mm in enumerate(meshes)
          if mm.presplit_tets is not None]
    if ps:
        out.presplit_tets = np.concatenate(ps).astype(np.int32)
        out.presplit_masks = np.concatenate([mm.presplit_masks for mm in meshes
                                             if mm.presplit_tets is not None])
    lt = [mm.load_tris.astype(np.int64) + node_off[i] for i, mm in enumerate(meshes)
          if mm.load_tris is not None]
    if lt:
        out.load_tris = np.concatenate(lt).astype(np.int32)
        out.load_trac = np.concatenate([mm.load_trac for mm in meshes if mm.load_tris is not None])
    return out, node_off.astype(np.int32), tet_off.astype(np.int32)


def ensemble(n=64, tmin=20000, tmax=200000, seed=2):
    """Batch of n notched plates of the 100 x 40 x 4 mm geometry with seeded
    sizes T_i ~ U[tmin, tmax] tets (cells round(25 s) x round(10 s) x
    max(1, round(s)) with s = (T_i / 1500)^(1/3)) and tractions ~ U[0.5, 2] MPa."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(tmin, tmax, size=n)
    trac = rng.uniform(0.5e6, 2.0e6, size=n)
    meshes = []
    for Ti, ti in zip(T, trac):
        s = (Ti / 1500.0) ** (1.0 / 3.0)
        nx, ny, nz = int(round(25 * s)), int(round(10 * s)), max(1, int(round(s)))
        meshes.append(plate_notched(nx, ny, nz, traction=float(ti)))
    u, no, to = union(meshes)
    return u, no, to, meshes, trac


def plate_window(nx=130, ny=52, nz=5, traction=1e6):
    """Coarser notched plate for gradient windows: 100 x 40 x 4 mm at
    130 x 52 x 5 cells (0.77 x 0.77 x 0.8 mm), 202,800 tets, same notch rule
    and load as the default plate."""
    return plate_notched(nx=nx, ny=ny, nz=nz, traction=traction)


def modulus_field(n_tets, E0=32e9, sigma=0.1, seed=3):
    """Per-tet Young's modulus E_j = E0 exp(sigma z_j), z_j iid N(0, 1)."""
    rng = np.random.default_rng(seed)
    return E0 * np.exp(sigma * rng.standard_normal(n_tets))


@dataclasses.dataclass
class HexMesh:
    """A trilinear hexahedral mesh plus its loads."""
    X: np.ndarray               # [N, 3] float64 node coordinates (m)
    hexes: np.ndarray           # [H, 8] int32 node ids, bottom face 0-1-2-3 then top 4-7
    grid: tuple = None
    h: tuple = None
    load_tris: np.ndarray = None
    load_trac: np.ndarray = None
    precrack_hexes: np.ndarray = None   # [P] int32 hexes cracked before the run
    precrack_planes: np.ndarray = None  # [P] uint8 their crack plane indices

    @property
    def n_nodes(self):
        return int(self.X.shape[0])

    @property
    def n_hex(self):
        return int(self.hexes.shape[0])


def hex_box(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    """Structured grid of nx*ny*nz hexahedral cells (the node grid of
    kuhn_box); cell order x-fastest; node order per cell (i,j,k), (i+1,j,k),
    (i+1,j+1,k), (i,j+1,k), then the same at k+1 (positive orientation).
    Loaded faces use face_triangles: each boundary square as two triangles."""
    t = kuhn_box(nx, ny, nz, lx, ly, lz)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    off = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    hx = np.stack([node_id(ci + a, cj + b, ck + c, nx, ny) for a, b, c in off], axis=1)
    return HexMesh(X=t.X, hexes=hx.astype(np.int32), grid=(nx, ny, nz), h=t.h)


def hex_bar(n=100, lx=1.0, w=0.01):
    """Slender hexahedral bar of n x 1 x 1 cells along x."""
    return hex_box(n, 1, 1, lx, w, w)


def hex_notched(nx=12, ny=8, nz=2, lx=None, ly=None, lz=None, notch_cells=None, traction=1e6,
                h=1e-3):
    """Hex box of nx*ny*nz cells of size h, pulled by +-traction on its y
    faces, with a notch: the hexes of cell row j = ny // 2 with i < notch_cells
    (default nx // 3), through the thickness, precracked by their mid-plane
    normal to y (crack plane index 1)."""
    lx = nx * h if lx is None else lx
    ly = ny * h if ly is None else ly
    lz = nz * h if lz is None else lz
    m = hex_box(nx, ny, nz, lx, ly, lz)
    add_tension(m, 1, traction)
    n = nx // 3 if notch_cells is None else notch_cells
    i = np.arange(m.n_hex) % nx
    j = (np.arange(m.n_hex) // nx) % ny
    sel = np.nonzero((j == ny // 2) & (i < n))[0]
    m.precrack_hexes = sel.astype(np.int32)
    m.precrack_planes = np.full(len(sel), 1, dtype=np.uint8)
    return m
