"""Batches: many independent simulations in one launch per pass (GPU)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_04076_amd import meshgen as mg

pytestmark = pytest.mark.gpu
MAT = dict(mg.BRANCHING_MATERIAL)


def _members():
    a = mg.cube_notched(4, traction=1.5e6)
    b = mg.cube_notched(5, traction=0.8e6)
    c = mg.plate_notched(24, 10, 2, 0.012, 0.005, 0.001, 0.006, traction=1.2e6)
    return [a, b, c]


def _split_rows(ev, tet_off, i):
    """Rows of the batch's split records that belong to member i."""
    return np.nonzero((ev[:, 1] >= tet_off[i]) & (ev[:, 1] < tet_off[i + 1]))[0]


def test_batch_matches_standalone_bitwise_and_oracle():
    from paper_2508_04076_amd.cem import Simulation
    print("\n[case] batch of 3 vs standalone, 150 steps", flush=True)
    members = _members()
    un, node_off, tet_off = mg.union(members)
    batch = Simulation(un.X, un.tets, MAT, max_splits=un.n_tets // 4, graph_steps=25)
    batch.set_instances(node_off, tet_off)
    batch.set_traction(un.load_tris, un.load_trac)
    batch.presplit(un.presplit_tets, un.presplit_masks)
    dtc = batch.critical_dt_instances()
    dts = 0.5 * dtc
    batch.set_dt_instances(dts)
    batch.step(150)
    ub, vb, _ = batch.get_state()
    evb, Gb = batch.splits()
    eb = batch.energy_instances()
    N0u = un.n_nodes
    for i, mm in enumerate(members):
        solo = Simulation.from_mesh(mm, MAT, max_splits=mm.n_tets // 4)
        assert abs(solo.critical_dt() - dtc[i]) <= 1e-15 * dtc[i]
        solo.set_dt(dts[i])
        solo.step(150)
        us, vs, _ = solo.get_state()
        evs, _ = solo.splits()
        rows = _split_rows(evb, tet_off, i)
        ev_i = evb[rows].copy()
        ev_i[:, 1] -= tet_off[i]
        assert np.array_equal(ev_i, evs)
        # original nodes, then the member's extra nodes in its own split order
        n0 = mm.n_nodes
        ext = np.concatenate([N0u + 4 * r + np.arange(4) for r in rows]) if len(rows) else \
            np.zeros(0, dtype=np.int64)
        ubi = np.concatenate([ub[node_off[i]:node_off[i + 1]], ub[ext]])
        vbi = np.concatenate([vb[node_off[i]:node_off[i + 1]], vb[ext]])
        assert np.array_equal(ubi, us) and np.array_equal(vbi, vs), f"member {i} not bitwise"
        es = solo.energy()
        for k in ("KE", "SE", "Wext", "Ud"):
            assert abs(eb[i][k] - es[k]) <= 1e-12 * max(abs(es[k]), 1e-30), (i, k)
        assert eb[i]["n_split"] == es["n_split"] and eb[i]["n_front"] == es["n_front"]
        assert eb[i]["Gmax"] == es["Gmax"] and eb[i]["n_nodes"] == es["n_nodes"]
        if i == 0:
            orc = Oracle.from_mesh(mm, MAT)
            orc.set_dt(dts[i])
            orc.step(150)
            uo, _, _ = orc.get_state()
            assert np.linalg.norm(us - uo) <= 1e-10 * np.linalg.norm(uo)
            eo, _ = orc.splits()
            assert np.array_equal(eo, evs)
        solo.close()
    batch.close()


def test_autotune_keeps_state_and_picks_a_valid_shape():
    from paper_2508_04076_amd.cem import Simulation
    print("\n[case] autotune on a batch of 3", flush=True)
    members = _members()
    un, node_off, tet_off = mg.union(members)
    sim = Simulation(un.X, un.tets, MAT, max_splits=un.n_tets // 4)
    sim.set_instances(node_off, tet_off)
    sim.set_traction(un.load_tris, un.load_trac)
    sim.presplit(un.presplit_tets, un.presplit_masks)
    sim.set_dt_instances(0.5 * sim.critical_dt_instances())
    sim.step(20)
    u0, v0, _ = sim.get_state()
    best = sim.autotune(trial_steps=5)
    assert best["grid_cap"] in (1024, 2048, 4096, 8192) and best["lanes"] in (4, 8, 16)
    assert best["layout"] in ("terms", "stress_sums", "tiles")
    assert best["ms_per_step"] > 0
    u1, v1, _ = sim.get_state()
    assert np.array_equal(u0, u1) and np.array_equal(v0, v1)
    # the tuned shape runs the same physics as the default shape (up to the
    # rounding order of the node sums)
    sim.step(40)
    ua, _, _ = sim.get_state()
    ref = Simulation(un.X, un.tets, MAT, max_splits=un.n_tets // 4)
    ref.set_instances(node_off, tet_off)
    ref.set_traction(un.load_tris, un.load_trac)
    ref.presplit(un.presplit_tets, un.presplit_masks)
    ref.set_dt_instances(0.5 * ref.critical_dt_instances())
    ref.set_launch(best["grid_cap"], best["lanes"], best["layout"])
    ref.step(60)
    ur, _, _ = ref.get_state()
    # the same splits in both runs (the node counts say so), then the same field
    assert ua.shape == ur.shape
    assert np.array_equal(sim.splits()[0], ref.splits()[0])
    assert np.linalg.norm(ua - ur) <= 1e-9 * np.linalg.norm(ur)
    sim.close()
    ref.close()


def test_full_ensemble_members_match_the_oracle():
    """The 64-plate ensemble at full size (7.1M tets, seeded sizes 20k-200k and
    tractions 0.5-2 MPa, 1 us ramp) under graphs: three members (the smallest,
    a middle one and the largest) against the oracle run of that member alone,
    over the first 30 steps (the pre-split notch included)."""
    from paper_2508_04076_amd.cem import Simulation
    print("\n[case] 64-plate ensemble, 30 graph steps, members against the oracle", flush=True)
    un, node_off, tet_off, members, trac = mg.ensemble(64)
    sim = Simulation(un.X, un.tets, MAT, precision="fp64", max_splits=un.n_tets // 4,
                     graph_steps=10)
    sim.set_instances(node_off, tet_off)
    sim.set_traction(un.load_tris, un.load_trac, 1e-6)
    sim.presplit(un.presplit_tets, un.presplit_masks)
    dts = 0.5 * sim.critical_dt_instances()
    sim.set_dt_instances(dts)
    sim.step(30)
    ub, vb, _ = sim.get_state()
    sizes = np.array([m.n_tets for m in members])
    pick = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    for i in pick:
        o = Oracle.from_mesh(members[i], MAT, ramp_t0=1e-6)
        o.set_threads(8)
        o.set_dt(dts[i])
        o.step(30)
        n0 = members[i].n_nodes
        uo, vo, _ = o.get_state()
        uo, vo = uo[:n0], vo[:n0]  # the original nodes (extra nodes: the notch copies)
        assert np.all(o.splits()[0][:, 3] == 0)  # no dynamic split in 30 steps
        ui, vi = ub[node_off[i]:node_off[i + 1]], vb[node_off[i]:node_off[i + 1]]
        err = np.linalg.norm(ui - uo) / np.linalg.norm(uo)
        print(f"  member {i}: {members[i].n_tets} tets, rel L2 u {err:.2e}", flush=True)
        assert err < 1e-10 and np.linalg.norm(vi - vo) < 1e-10 * np.linalg.norm(vo)
    sim.close()
