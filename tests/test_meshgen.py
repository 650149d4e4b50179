"""Synthetic input generator: closed-form counts and geometry (CPU)."""
import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg


def _edges(t):
    e = np.concatenate([t[:, [0, 1]], t[:, [0, 2]], t[:, [0, 3]], t[:, [1, 2]], t[:, [1, 3]],
                        t[:, [2, 3]]])
    return np.unique(np.sort(e, axis=1), axis=0)


def _faces(t):
    f = np.concatenate([t[:, [1, 2, 3]], t[:, [0, 2, 3]], t[:, [0, 1, 3]], t[:, [0, 1, 2]]])
    return np.unique(np.sort(f, axis=1), axis=0, return_counts=True)


def _vol(X, t):
    a = X[t[:, 1]] - X[t[:, 0]]
    b = X[t[:, 2]] - X[t[:, 0]]
    c = X[t[:, 3]] - X[t[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


@pytest.mark.parametrize("g", [(1, 1, 1), (2, 3, 4), (10, 10, 10), (7, 2, 5)])
def test_kuhn_counts_closed_form(g):
    m = mg.kuhn_box(*g)
    cnt = mg.kuhn_counts(*g)
    assert m.n_nodes == cnt["nodes"] == (g[0] + 1) * (g[1] + 1) * (g[2] + 1)
    assert m.n_tets == cnt["tets"] == 6 * g[0] * g[1] * g[2]
    assert len(_edges(m.tets)) == cnt["edges"]
    faces, mult = _faces(m.tets)
    assert len(faces) == cnt["faces"]
    assert mult.max() <= 2 and (mult == 1).sum() == cnt["boundary_faces"]
    # Euler characteristic of a ball: V - E + F - T = 1
    assert cnt["nodes"] - cnt["edges"] + cnt["faces"] - cnt["tets"] == 1


def test_paper_workload_sizes():
    assert mg.kuhn_counts(10, 10, 10)["edges"] == 7930
    c1 = mg.kuhn_counts(200, 80, 8)
    assert (c1["nodes"], c1["tets"], c1["edges"]) == (146529, 768000, 951008)
    c4 = mg.kuhn_counts(400, 200, 100)
    assert (c4["nodes"], c4["tets"], c4["edges"]) == (8140701, 48000000, 56420700)


def test_orientation_and_volume():
    m = mg.kuhn_box(3, 4, 5, 0.3, 0.2, 0.1)
    V = _vol(m.X, m.tets)
    assert V.min() > 0
    assert abs(V.sum() - 0.3 * 0.2 * 0.1) < 1e-15
    mj = mg.jitter(mg.kuhn_box(4, 4, 4), 0.2, seed=0)
    V = _vol(mj.X, mj.tets)
    assert V.min() > 0 and abs(V.sum() - 1.0) < 1e-13


def test_notch_and_loads():
    m = mg.cube_notched(10)
    assert len(m.presplit_tets) == 180
    pc = np.array([bin(x).count("1") for x in m.presplit_masks])
    assert set(pc) <= {1, 2, 3}
    # side B = nodes on the notch plane z = 0.5
    for t, mk in zip(m.presplit_tets[:30], m.presplit_masks[:30]):
        z = m.X[m.tets[t], 2]
        assert all(((mk >> l) & 1) == (z[l] > 0.45) for l in range(4))
    p = mg.plate_notched()
    assert len(p.presplit_tets) == 4800
    # loaded faces are tet faces
    faces, _ = _faces(p.tets)
    fs = {tuple(f) for f in faces.tolist()}
    assert all(tuple(sorted(tr)) in fs for tr in p.load_tris.tolist())
    # total applied force: +1 MPa * 0.1 * 0.004 on top, minus on bottom
    A = 0.5 * np.linalg.norm(np.cross(p.X[p.load_tris[:, 1]] - p.X[p.load_tris[:, 0]],
                                      p.X[p.load_tris[:, 2]] - p.X[p.load_tris[:, 0]]), axis=1)
    top = p.load_trac[:, 1] > 0
    assert abs((A[top] * p.load_trac[top, 1]).sum() - 1e6 * 0.1 * 0.004) < 1e-6


def test_permutation_is_relabelling():
    m = mg.cube_notched(4)
    p = mg.permute(m, seed=1)
    assert np.allclose(np.sort(_vol(p.X, p.tets)), np.sort(_vol(m.X, m.tets)))
    assert len(p.presplit_tets) == len(m.presplit_tets)
