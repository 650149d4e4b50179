"""Writes plate_768k_splits.json: the oracle's run of the notched plate
(100 x 40 x 4 mm, 200 x 80 x 8 cells x 6 tets = 768,000 tets, 50 mm edge notch
at mid-height pre-split, +-1 MPa traction in y ramped over 1 us, FP64,
dt = 0.5 dt_crit) through the onset of dynamic splitting and branching.

Only the oracle and the seeded mesh generator are called.  The file holds
every split event (step, tet, side mask, pattern, G), the energies at the
end, dt bitwise (hex), and u and v at a seeded sample of nodes (original
and extra) at the end.

    python tests/golden/make_plate_768k.py [--steps 2400] [--threads 8]

About 20 minutes on 8 threads (the oracle's threads give the same bits at
any count).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2508_04076_amd import meshgen as mg  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plate_768k_splits.json")
RAMP_T0 = 1e-6
N_SAMPLE = 1500


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2400)
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    mat = dict(mg.BRANCHING_MATERIAL)
    mesh = mg.plate_notched()
    orc = Oracle.from_mesh(mesh, mat, ramp_t0=RAMP_T0)
    orc.set_threads(a.threads)
    dt = 0.5 * orc.critical_dt()
    orc.set_dt(dt)
    t0 = time.time()
    done = 0
    while done < a.steps:
        n = min(100, a.steps - done)
        orc.step(n)
        done += n
        e = orc.energy()
        print(f"step {done}: splits {int(e['n_split'])}, Gmax {e['Gmax']:.4g}, "
              f"{time.time() - t0:.0f} s", flush=True)
    ev, G = orc.splits()
    u, v, _ = orc.get_state()
    rng = np.random.default_rng(7)
    n0 = mesh.n_nodes
    samp = np.sort(np.concatenate([
        rng.choice(n0, size=min(N_SAMPLE, n0), replace=False),
        np.arange(n0, u.shape[0])[rng.permutation(u.shape[0] - n0)[:N_SAMPLE // 3]],
    ])).astype(int)
    doc = {
        "workload": "notched plate 100x40x4 mm, 200x80x8 cells x 6 tets (768,000 tets), "
                    "50 mm edge notch at mid-height, +-1 MPa in y ramped over 1 us, FP64, "
                    "dt = 0.5 dt_crit, phantom-node splitting, principal-stress G",
        "written_by": "tests/golden/make_plate_768k.py (oracle only)",
        "material": mat,
        "ramp_t0": RAMP_T0,
        "steps": a.steps,
        "dt_hex": float(dt).hex(),
        "n_nodes_end": int(u.shape[0]),
        "events": [[int(x) for x in r] for r in ev],
        "G": [float(x).hex() for x in G],
        "energy_end": {k: float(x) for k, x in orc.energy().items()},
        "u_l2": float(np.linalg.norm(u)),
        "v_l2": float(np.linalg.norm(v)),
        "sample_nodes": samp.tolist(),
        "u_sample": [[float(x).hex() for x in r] for r in u[samp]],
        "v_sample": [[float(x).hex() for x in r] for r in v[samp]],
    }
    with open(a.out, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
        f.write("\n")
    dyn = int((ev[:, 3] != 0).sum())
    print(f"wrote {a.out}: {len(ev)} events ({dyn} dynamic), {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
