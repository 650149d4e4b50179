"""The 768,000-tet notched plate through the onset of dynamic splitting and
branching, GPU (through the C-ABI) against the oracle's run stored in
tests/golden/plate_768k_splits.json (written by
tests/golden/make_plate_768k.py, which calls only the oracle).

Identical split events (step, tet, side mask, pattern) over the whole run,
release rates of the dynamic splits within 1e-9, u and v at the stored node
sample within 1e-8 relative L2, energies within 1e-8; in the force layout
and launch shape the bench's autotuner picks for this plate (stress sums)
and in the term layout, both under HIP graphs.
"""
import json
import os

import numpy as np
import pytest

from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plate_768k_splits.json")


def _hex2(rows):
    return np.array([[float.fromhex(x) for x in r] for r in rows])


@pytest.mark.parametrize("launch", [(8192, 8, "stress_sums"), (2048, 4, "terms")])
def test_plate_split_events_match_the_oracle_through_fracture(launch):
    from paper_2508_04076_amd.cem import Simulation
    d = json.load(open(GOLD))
    print(f"\n[case] plate 768k, {d['steps']} steps against the stored oracle run, launch {launch}",
          flush=True)
    mesh = mg.plate_notched()
    mat = d["material"]
    sim = Simulation.from_mesh(mesh, mat, ramp_t0=d["ramp_t0"], max_splits=200000, graph_steps=50)
    sim.set_launch(*launch)
    sim.set_dt(float.fromhex(d["dt_hex"]))
    sim.step(d["steps"])
    ev, G = sim.splits()
    want = np.array(d["events"], dtype=np.int32)
    assert (want[:, 3] > 0).sum() > 1000
    assert ev.shape == want.shape, (ev.shape, want.shape)
    assert np.array_equal(ev, want)
    Gw = np.array([float.fromhex(x) for x in d["G"]])
    dyn = want[:, 3] > 0
    assert np.allclose(G[dyn], Gw[dyn], rtol=1e-9, atol=0)
    u, v, _ = sim.get_state()
    assert u.shape[0] == d["n_nodes_end"]
    idx = np.array(d["sample_nodes"])
    for got, key in ((u, "u_sample"), (v, "v_sample")):
        w = _hex2(d[key])
        assert np.linalg.norm(got[idx] - w) <= 1e-8 * np.linalg.norm(w), key
    assert abs(np.linalg.norm(u) / d["u_l2"] - 1) < 1e-8
    e, eo = sim.energy(), d["energy_end"]
    for k in ("KE", "SE", "Wext", "Ud"):
        assert abs(e[k] - eo[k]) <= 1e-8 * abs(eo[k]), (k, e[k], eo[k])
    assert int(e["n_split"]) == len(want)
    sim.close()
