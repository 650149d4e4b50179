"""Oracle pins of the hexahedral crack patterns III-VI (Section 3, the
parallelepiped patterns; the readings of the missing figure are listed with
the oracle).

What the text fixes, and how each pin ties the oracle to it:

- III and IV come from a front through the midpoints of two opposite edges of
  a face, V and VI from one through two neighbouring edges; III deactivates
  the hex, IV-VI leave the triangular-prism half.  The plane table (the cut
  edges of each of the 23 planes) is checked against the natural coordinates
  of the edge midpoints by brute force, and the region each plane cuts off
  against a sampled volume.
- G_III, G_IV and G_V follow Eq. G-I, G_VI follows Eq. G-II.  On cubes under
  a uniform uniaxial strain eps along d the rates have closed forms, with
  sigma = (lambda + 2 mu) eps the largest principal stress and |delta| the
  stretch of the front edges: an opposite-edge front with d normal to the
  mid-plane gives G_III = sigma |delta| and G_IV = sigma |delta| / 2 (normal
  at 45 degrees); a neighbouring-edge front with d normal to the wedge plane
  gives G_V = sigma |delta| and G_VI = (2/3) sigma |delta| (d . n = sqrt(2/3)).
- The cracked element keeps its edge-point gradients with the remaining
  volume: a lone hex's force is linear in that volume, so a deactivated hex
  gives none and a prism half gives exactly half.
- Ties: larger G wins, then the lower local face, then III, IV (-), IV (+),
  V, VI; G >= Gc cracks.  Fronts and first candidates are found here from the
  connectivity and the plane definitions, not from the oracle.
"""
import itertools

import numpy as np
import pytest

from oracle.oracle import Oracle, lame
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)

SIGN = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                 [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]])
EDGE = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
        (0, 4), (1, 5), (2, 6), (3, 7)]
MID = np.array([(SIGN[a] + SIGN[b]) / 2 for a, b in EDGE])


def planes():
    """The 23 crack planes c . xi = d in the oracle's index order: the three
    mid-planes, the twelve wedge planes, the eight corner planes."""
    out = []
    for a in range(3):
        c = np.zeros(3)
        c[a] = 1
        out.append((c, 0))
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        for sa in (-1, 1):
            for sb in (-1, 1):
                c = np.zeros(3)
                c[a], c[b] = sa, sb
                out.append((c, 1))
    for s in itertools.product((-1, 1), repeat=3):
        out.append((np.array(s, float), 2))
    return out


PLANES = planes()
CUT = [sum(1 << q for q in range(12) if MID[q] @ c == d) for c, d in PLANES]


def face_edges(f):
    axis, side = f // 2, (1 if f % 2 else -1)
    return [q for q in range(12) if all(SIGN[n][axis] == side for n in EDGE[q])]


def test_plane_table_by_brute_force():
    o = Oracle.hex_mesh(mg.hex_box(1, 1, 1), MAT)
    assert o.hex_plane_masks().tolist() == CUT
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 1, size=(200000, 3))
    for p, (c, d) in enumerate(PLANES):
        assert bin(CUT[p]).count("1") == (4 if p < 15 else 3)
        for f in range(6):  # a face is cut along two edges or not at all
            assert bin(CUT[p] & sum(1 << q for q in face_edges(f))).count("1") in (0, 2)
        frac = np.mean(pts @ c > d) if d > 0 else np.mean(pts @ c > 0)
        expect = 0.5 if d == 0 else (1 / 8 if d == 1 else 1 / 48)
        assert abs(frac - expect) < 3e-3, (p, frac)


def _stack(axis, h):
    n = [1, 1, 1]
    n[axis] = 2
    return mg.hex_box(*n, lx=n[0] * h, ly=n[1] * h, lz=n[2] * h)


def _uniaxial(X, d, eps):
    d = np.asarray(d, float) / np.linalg.norm(d)
    return eps * np.outer(X @ d, d), d


def test_opposite_edge_front_closed_forms():
    # hex 0 cracked by its mid-plane normal to y: its face x = +1 is cut at the
    # midpoints of its two y-edges, a front of hex 1 on opposite edges
    h, eps = 0.5, 1e-4
    m = _stack(0, h)
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.presplit([0], [1])
    u, _ = _uniaxial(m.X, [0, 1, 0], eps)
    o.set_state(u)
    lam, mu = lame(MAT["E"], MAT["nu"])
    sig = (lam + 2 * mu) * eps
    rows, g = o.front_G()
    # hex 1, its face x = -1 (local face 0): III (mid-plane y), IV (-x-y), IV (-x+y)
    assert rows.tolist() == [[1, 0, 1], [1, 0, 3], [1, 0, 4]]
    assert g[:, 1].tolist() == [3, 4, 4]
    assert g[0, 0] == pytest.approx(sig * eps * h, rel=1e-12)
    assert g[1, 0] == pytest.approx(sig * eps * h / 2, rel=1e-12)
    assert g[2, 0] == pytest.approx(sig * eps * h / 2, rel=1e-12)


def test_neighbouring_edge_front_closed_forms():
    # hex 0 cracked by the wedge plane +x -y = 1 (around its edge x = +1,
    # y = -1); its top face is cut on two neighbouring edges, a front of hex 1
    h, eps = 1.0, 2e-4
    m = _stack(2, h)
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.presplit([0], [5])
    u, d = _uniaxial(m.X, [1, -1, 0], eps)
    o.set_state(u)
    lam, mu = lame(MAT["E"], MAT["nu"])
    sig = (lam + 2 * mu) * eps
    rows, g = o.front_G()
    # hex 1, its face z = -1 (local face 4): V (plane +x -y = 1), VI (+x -y -z = 2)
    assert rows.tolist() == [[1, 4, 5], [1, 4, 19]]
    assert g[:, 1].tolist() == [5, 6]
    de = eps * h / np.sqrt(2)  # |delta| of each front edge (delta along d)
    c2 = 2.0 / 3.0             # (d . n_VI)^2, n_VI = (1, -1, -1) / sqrt 3
    assert g[0, 0] == pytest.approx(sig * de, rel=1e-12)
    assert g[1, 0] == pytest.approx(c2 * sig * de, rel=1e-12)


def test_remaining_volume_scales_a_lone_hex():
    m = mg.hex_box(1, 1, 1, 1e-2, 2e-2, 1.5e-2)
    rng = np.random.default_rng(4)
    m.X = m.X + rng.uniform(-1e-3, 1e-3, size=m.X.shape)
    u = mg.random_displacement(m.n_nodes, 1e-6, seed=2)
    f_all = Oracle.hex_mesh(m, MAT, traction=False).internal_force(u)
    assert np.abs(f_all).max() > 0
    for plane, frac in [(0, 0.0), (2, 0.0), (7, 0.5), (14, 0.5), (20, 0.5)]:
        o = Oracle.hex_mesh(m, MAT, traction=False)
        o.presplit([0], [plane])
        np.testing.assert_allclose(o.internal_force(u), frac * f_all, rtol=1e-12, atol=1e-12 * np.abs(f_all).max())
        ev, G = o.splits()
        assert ev.tolist() == [[0, 0, plane, 0]] and G.tolist() == [0.0]


def expected_first_candidates(m, cracked):
    """Front hexes and, per front hex, (lowest front face, its first candidate
    plane) from the connectivity: a face of a cracked hex with two cut edges
    is a front of the intact hex across it; its first candidate is III (the
    mid-plane along the two edges) for opposite edges, V (the wedge plane
    through both midpoints that contains the face normal) for neighbouring
    ones."""
    faces = {}
    for t, nd in enumerate(m.hexes):
        for f in range(6):
            key = tuple(sorted(int(nd[l]) for l in range(8) if SIGN[l][f // 2] == (1 if f % 2 else -1)))
            faces.setdefault(key, []).append((t, f))
    out = {}
    for s, p in cracked.items():
        for f in range(6):
            cut = [q for q in face_edges(f) if (CUT[p] >> q) & 1]
            if len(cut) != 2:
                continue
            key = tuple(sorted(int(m.hexes[s][l]) for l in range(8) if SIGN[l][f // 2] == (1 if f % 2 else -1)))
            for (t, fc) in faces[key]:
                if t == s or t in cracked:
                    continue
                gl = {tuple(sorted((int(m.hexes[s][EDGE[q][0]]), int(m.hexes[s][EDGE[q][1]])))) for q in cut}
                mine = sorted(q for q in range(12)
                              if tuple(sorted((int(m.hexes[t][EDGE[q][0]]), int(m.hexes[t][EDGE[q][1]])))) in gl)
                a = np.nonzero(MID[mine[0]] == 0)[0][0]
                b = np.nonzero(MID[mine[1]] == 0)[0][0]
                if a == b:
                    first = int(a)
                else:
                    k = fc // 2
                    first = next(pi for pi, (c, d) in enumerate(PLANES)
                                 if d == 1 and c[k] == 0 and MID[mine[0]] @ c == 1 and MID[mine[1]] @ c == 1)
                if t not in out or fc < out[t][0]:
                    out[t] = (fc, first)
    return out


def _cracked_block(seed=5):
    m = mg.hex_box(6, 5, 3, 6e-3, 5e-3, 3e-3)
    rng = np.random.default_rng(seed)
    hx = rng.choice(m.n_hex, size=12, replace=False)
    pl = rng.integers(0, 23, size=12)
    return m, {int(a): int(b) for a, b in zip(hx, pl)}


def test_ties_go_to_the_lower_face_then_the_first_candidate():
    # zero state from a ramped load: every rate is exactly 0 after one step,
    # so with Gc = 0 every front hex cracks, through its lowest front face
    # with that face's first candidate
    m, cracked = _cracked_block()
    mg.add_tension(m, 1, 1e6)
    want = expected_first_candidates(m, cracked)
    assert sum(1 for t in want) > 5
    o = Oracle.hex_mesh(m, MAT, ramp_t0=1e-3, Gc=0.0)
    o.presplit(list(cracked), list(cracked.values()))
    rows, g = o.front_G()
    assert sorted({int(r[0]) for r in rows}) == sorted(want)
    assert np.all(g[:, 0] == 0.0)
    o.set_dt(0.5 * o.critical_dt())
    o.step(1)
    ev, G = o.splits()
    dyn = ev[ev[:, 3] != 0]
    assert dyn[:, 1].tolist() == sorted(want)
    assert dyn[:, 2].tolist() == [want[t][1] for t in sorted(want)]
    assert np.all(G[ev[:, 3] != 0] == 0.0)


def test_griffith_test_holds_with_equality():
    m, cracked = _cracked_block(seed=6)
    mg.add_tension(m, 1, 1e6)
    def make(Gc):
        o = Oracle.hex_mesh(m, MAT, Gc=Gc)
        o.presplit(list(cracked), list(cracked.values()))
        return o
    dt = 0.5 * make(1e300).critical_dt()
    ref = make(1e300)
    ref.set_dt(dt)
    n = 0
    while True:
        ref.step(1)
        n += 1
        if ref.energy()["Gmax"] > 0 or n > 40:
            break
    Gs = ref.energy()["Gmax"]
    assert Gs > 0
    rows, g = ref.front_G()
    best = {}
    for (t, f, p), (val, pat) in zip(rows.tolist(), g.tolist()):
        if t not in best or val > best[t][0]:
            best[t] = (val, p, int(pat))
    assert max(b[0] for b in best.values()) == Gs
    want = [[n, t, b[1], b[2]] for t, b in sorted(best.items()) if b[0] == Gs]
    # unit cells of side h: a mid-plane crack has area h^2, a wedge plane
    # h^2 / sqrt 2, a corner plane sqrt(3) h^2 / 8; U_d = Gc times the area
    h = 1e-3
    area = lambda p: h * h if p < 3 else (h * h / np.sqrt(2) if p < 15 else np.sqrt(3) * h * h / 8)
    for Gc, expect in ((Gs, want), (np.nextafter(Gs, np.inf), [])):
        o = make(Gc)
        o.set_dt(dt)
        o.step(n)
        ev, G = o.splits()
        dyn = ev[ev[:, 3] != 0]
        assert dyn.tolist() == expect
        assert np.all(G[ev[:, 3] != 0] == Gs)
        assert o.energy()["Ud"] == pytest.approx(Gc * sum(area(p) for p in dyn[:, 2]), rel=1e-12)


def _shares_face(q, r):
    return any(all(SIGN[n][a] == SIGN[EDGE[q][0]][a] for n in EDGE[q] + EDGE[r])
               for a in range(3) if MID[q][a] != 0 and MID[r][a] != 0 and MID[q][a] == MID[r][a])


def test_candidates_by_brute_force_on_a_distorted_block():
    # every candidate's G from its plane alone: G1, G2 are the plane's cut edges
    # on the front face (lower local edge first), G3 (G4) the remaining cut edge
    # on a common face with G1 (G2), or G6; the stretches, the edge stresses of
    # the oracle's smoothing and the stress term then enter Eqs. G-I / G-II
    from oracle.oracle import stress_term
    m = mg.jitter(mg.hex_box(4, 4, 3, 4e-3, 4e-3, 3e-3), 0.2, seed=7)
    rng = np.random.default_rng(8)
    hx = rng.choice(m.n_hex, size=10, replace=False)
    pl = rng.integers(0, 23, size=10)
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.presplit(hx, pl)
    u = mg.random_displacement(m.n_nodes, 2e-6, seed=9) + 1e-4 * np.outer(m.X[:, 1], [0.3, 1.0, -0.2])
    o.set_state(u)
    en, _, sig = o.edges()
    eid = {tuple(sorted(map(int, e))): k for k, e in enumerate(en)}
    rows, g = o.front_G()
    assert len(rows) > 20 and set(g[:, 1]) == {3, 4, 5, 6}
    for (t, f, p), (G, pat) in zip(rows.tolist(), g.tolist()):
        nd = m.hexes[t]
        cut = [q for q in range(12) if (CUT[p] >> q) & 1]
        front = [q for q in cut if q in face_edges(f)]
        assert len(front) == 2
        q1, q2 = sorted(front)
        rest = [q for q in cut if q not in front]
        P = lambda q: 0.5 * (m.X[nd[EDGE[q][0]]] + m.X[nd[EDGE[q][1]]])
        def stretch(q):
            a, b = nd[EDGE[q][0]], nd[EDGE[q][1]]
            du, dX = u[b] - u[a], m.X[b] - m.X[a]
            return du if 2 * dX @ du + du @ du > 0 else np.zeros(3)
        s = lambda q, n: stress_term(sig[eid[tuple(sorted((int(nd[EDGE[q][0]]), int(nd[EDGE[q][1]]))))]], n)
        d1, d2 = stretch(q1), stretch(q2)
        if len(rest) == 1:
            assert pat == 6
            n = np.cross(P(q2) - P(q1), P(rest[0]) - P(q1))
            n /= np.linalg.norm(n)
            want = 0.5 * s(rest[0], n) * (abs(d1 @ n) + abs(d2 @ n))
        else:
            q3 = [r for r in rest if _shares_face(q1, r)]
            q4 = [r for r in rest if _shares_face(q2, r)]
            assert len(q3) == 1 and len(q4) == 1 and q3 != q4
            q3, q4 = q3[0], q4[0]
            n = np.cross(P(q4) - P(q1), P(q3) - P(q2))
            n /= np.linalg.norm(n)
            want = 0.5 * (s(q3, n) * abs(d1 @ n) + s(q4, n) * abs(d2 @ n))
            opposite = (MID[q1] == 0).tolist() == (MID[q2] == 0).tolist()
            assert pat == ((3 if p < 3 else 4) if opposite else 5)
        assert G == pytest.approx(want, rel=1e-11, abs=1e-300)


def test_shortening_front_edges_release_nothing():
    # the front edges shorten under compression along y: delta = 0, G = 0
    h, eps = 0.5, 1e-4
    m = _stack(0, h)
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.presplit([0], [1])
    u, _ = _uniaxial(m.X, [0, 1, 0], -eps)
    o.set_state(u)
    rows, g = o.front_G()
    assert len(rows) == 3 and np.all(g[:, 0] == 0.0)


@pytest.mark.parametrize("d, plane, pattern, area", [
    ([1, -1, -1], 19, 6, np.sqrt(3) / 8),   # along VI's normal: G_VI = sigma |delta| > G_V
    ([1, -1, 0], 5, 5, 1 / np.sqrt(2)),     # along V's normal: G_V = sigma |delta| > G_VI
])
def test_the_larger_of_V_and_VI_cracks_and_books_its_area(d, plane, pattern, area):
    # the stack of the neighbouring-edge case, strained along the normal of one
    # candidate: that one wins (ratio 3/2), and U_d = Gc times its surface, the
    # corner triangle (sqrt 3 / 8) h^2 or the wedge quad h^2 / sqrt 2
    h, eps = 1e-3, 1e-3
    m = _stack(2, h)
    o = Oracle.hex_mesh(m, MAT, traction=False)
    o.presplit([0], [5])
    u, _ = _uniaxial(m.X, d, eps)
    o.set_state(u)
    o.set_dt(0.25 * o.critical_dt())
    o.step(1)
    ev, G = o.splits()
    assert ev.tolist() == [[0, 0, 5, 0], [1, 1, plane, pattern]]
    assert G[1] > MAT["Gc"]
    assert o.energy()["Ud"] == pytest.approx(MAT["Gc"] * area * h * h, rel=1e-12)
