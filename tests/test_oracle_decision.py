"""Oracle pins of the split decision (Section 3 and the Griffith test of
Section 2.1) and of its stress term near tied principal stresses.

- Ties: with every release rate exactly 0 and Gc = 0, every crack-front tet
  splits (G >= Gc holds with equality), through its lowest local front face,
  with pattern I (ties go to the lower face, then pattern I before II).  The
  expected splits come from the mesh's own faces, not from the oracle.
- Equality: with Gc set to the largest release rate of a step, exactly the
  tets that reach it split in that step; with the next larger double, none.
- Stress term: sigma_1 |P_1 n| against the closed form of a tensor built from
  a known rotation, for relative gaps between the two largest principal
  stresses from 1e-13 to 1e-2 (eigenvalues within 1e-6 max|lambda| form one
  eigenspace).
"""
import numpy as np

from oracle.oracle import Oracle, stress_term
from paper_2508_04076_amd import meshgen as mg

MAT = dict(mg.BRANCHING_MATERIAL)


def expected_fronts(tets, presplit, masks):
    """Crack fronts by the definition of Section 3, from the connectivity: for
    each face of a pre-split tet whose nodes lie on both sides of its cut, the
    intact tet across it, that tet's local face index (its opposite local
    node) and the node of the face alone on its side.  {tet: [(face, lone)]}."""
    faces = {}
    for t, nd in enumerate(tets):
        for f in range(4):
            key = tuple(sorted(int(nd[l]) for l in range(4) if l != f))
            faces.setdefault(key, []).append((t, f))
    split = {int(t): int(m) for t, m in zip(presplit, masks)}
    out = {}
    for s, m in split.items():
        for f in range(4):
            ls = [l for l in range(4) if l != f]
            bits = [(m >> l) & 1 for l in ls]
            if bits[0] == bits[1] == bits[2]:
                continue
            lone = ls[[i for i in range(3) if bits.count(bits[i]) == 1][0]]
            key = tuple(sorted(int(tets[s][l]) for l in ls))
            for (t, fc) in faces[key]:
                if t != s and t not in split:
                    out.setdefault(t, []).append((fc, int(tets[s][lone])))
    return out


def _positively_oriented(X, tets):
    d = np.einsum("ij,ij->i", np.cross(X[tets[:, 1]] - X[tets[:, 0]], X[tets[:, 2]] - X[tets[:, 0]]),
                  X[tets[:, 3]] - X[tets[:, 0]])
    return bool((d > 0).all())


def test_ties_go_to_the_lower_face_then_pattern_I():
    # ramped load from rest: the state after the first step is still zero, so
    # every front's G_I and G_II are exactly 0; with Gc = 0 all of them pass
    m = mg.cube_notched(5)
    assert _positively_oriented(m.X, m.tets)
    # every other notch tet pre-split: intact tets between two split ones
    # have two or three fronts, so the face order is tested
    m.presplit_tets, m.presplit_masks = m.presplit_tets[::2], m.presplit_masks[::2]
    fr = expected_fronts(m.tets, m.presplit_tets, m.presplit_masks)
    assert sum(len(v) > 1 for v in fr.values()) > 0
    o = Oracle.from_mesh(m, MAT, ramp_t0=1e-3, Gc=0.0)
    o.set_dt(0.5 * o.critical_dt())
    o.step(1)
    tfl, g = o.front_G()
    ev, G = o.splits()
    dyn = ev[ev[:, 3] != 0]
    want = []
    for t in sorted(fr):
        face, lone = min(fr[t])
        l2 = [int(x) for x in m.tets[t]].index(lone)
        want.append([1, t, (1 << l2) | (1 << face), 1])
    assert dyn.tolist() == want
    assert np.all(G[ev[:, 3] != 0] == 0.0)


def _best_per_tet(m, tfl, g):
    """(G, mask, pattern) per candidate in face order, ties to the lower face
    and to pattern I; masks from the local indices of the mesh connectivity."""
    best = {}
    for (t, f, lone), (gI, gII) in zip(tfl.tolist(), g.tolist()):
        l2 = [int(x) for x in m.tets[t]].index(lone)
        for val, mask, pat in ((gI, (1 << l2) | (1 << f), 1), (gII, 1 << l2, 2)):
            if t not in best or val > best[t][0]:
                best[t] = (val, mask, pat)
    return best


def test_griffith_test_holds_with_equality():
    m = mg.cube_notched(5)
    assert _positively_oriented(m.X, m.tets)
    dt = 0.5 * Oracle.from_mesh(m, MAT).critical_dt()
    # reference run: no split passes (Gc finite but out of reach), G recorded
    ref = Oracle.from_mesh(m, MAT, Gc=1e300)
    ref.set_dt(dt)
    gmax = []
    for n in range(1, 40):
        ref.step(1)
        gmax.append(ref.energy()["Gmax"])
        if gmax[-1] > 0:
            break
    n = len(gmax)
    assert gmax[-1] > 0 and all(x == 0 for x in gmax[:-1])
    tfl, g = ref.front_G()
    best = _best_per_tet(m, tfl, g)
    Gs = max(b[0] for b in best.values())
    assert Gs == gmax[-1]
    want = [[n, t, b[1], b[2]] for t, b in sorted(best.items()) if b[0] == Gs]
    for Gc, expect in ((Gs, want), (np.nextafter(Gs, np.inf), [])):
        o = Oracle.from_mesh(m, MAT, Gc=Gc)
        o.set_dt(dt)
        o.step(n)
        ev, G = o.splits()
        dyn = ev[ev[:, 3] != 0]
        assert dyn.tolist() == expect, (Gc, dyn.tolist(), expect)
        assert np.all(G[ev[:, 3] != 0] == Gs)


def _voigt(S):
    return [S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[1, 2], S[0, 2]]


def test_stress_term_across_the_tie_gap():
    rng = np.random.default_rng(21)
    scale = 3e6
    for gap in (0.0, 1e-13, 1e-11, 1e-9, 1e-7, 5e-7, 2e-6, 1e-5, 1e-4, 1e-2):
        for _ in range(25):
            Q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
            lam = scale * np.array([1.0, 1.0 - gap, -0.3])
            S = (Q * lam) @ Q.T
            n = rng.standard_normal(3)
            n /= np.linalg.norm(n)
            s = stress_term(_voigt(S), n)
            if gap <= 5e-7:
                # one eigenspace spanned by q1 and q2: the part of n normal to q3
                want = scale * np.sqrt(max(0.0, 1.0 - (Q[:, 2] @ n) ** 2))
                tol = 1e-12 * scale
            else:
                want = scale * abs(Q[:, 0] @ n)
                # the eigenvector moves by rounding over the gap
                tol = (1e-12 + 1e-14 / gap) * scale
            assert abs(s - want) <= tol, (gap, s, want)
    # three equal principal stresses: every direction is principal
    for _ in range(10):
        Q = np.linalg.qr(rng.standard_normal((3, 3)))[0]
        S = (Q * (scale * np.array([1.0, 1.0 - 1e-12, 1.0 + 1e-12]))) @ Q.T
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        assert abs(stress_term(_voigt(S), n) - scale) < 1e-10 * scale
