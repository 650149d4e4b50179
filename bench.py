"""Throughput of the ES-T-FEM crack-element step on one MI355X.

Default workload: the notched plate of the paper's crack-branching example
(Section 4.4) on a synthetic structured mesh, 100 x 40 x 4 mm at 200 x 80 x 8
cells x 6 tets = 768,000 tets, 1 MPa traction ramped over 1 us, splitting on.
A step is the whole hot path: strain pass, edge stress pass, crack-front pass
with flag compaction, node force + Newmark pass, topology update.

Prints one JSON line (rank 0).  Phases:
  0. the library's autotuner picks the launch shape (force layout, grid,
     lanes) on a warmed-up copy;
  1. FP64 run, plain launches with per-pass HIP events on the library's
     stream: warmup, then --steps steps (per-pass durations and the roofline
     of the dominant pass; reported as "per_pass_run");
  2. the same steps as captured HIP graphs, and again as plain launches,
     both without events: value and ms_per_step are the faster of the two
     (which one wins varies from one machine to another; both are reported
     under "modes"),
     each bitwise equal to run 1;
  3. mixed precision with the FP64 split schedule replayed (its own tuned
     shape): throughput and relative L2 error of u against the FP64 run;
  4. the CPU oracle on a bounded sample (cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tet-steps/sec and HBM GB/s, FP32-mixed vs FP64 at stated displacement error"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per tet-step of each pass (compulsory traffic of the
# three-pass formulation with stored gradients; FP64 / mixed).
ALG_BYTES = {
    "fp64": {"strain": 149.0, "edge_stress": 146.0, "node": 200.0},
    "mixed": {"strain": 85.0, "edge_stress": 88.0, "node": 130.0},
}
# the node pass is two launches: per-element force terms (with the crack-front
# workgroups riding along), then per-node sums
KERNEL_NAMES = {"strain": ["k_strain"], "edge_stress": ["k_edge_stress"],
                "node": ["k_elem_force_front", "k_node"]}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    from paper_2508_04076_amd import meshgen as mg
    if name == "plate":
        return mg.plate_notched(), 1e-6, ("notched plate 100x40x4 mm, 200x80x8 cells x 6 tets "
                                         "(768,000 tets), 50 mm edge notch at mid-height, "
                                         "1 MPa traction ramped over 1 us")
    if name == "cube":
        return mg.cube_notched(10), 0.0, ("unit cube 10x10x10 cells x 6 tets (6,000 tets), "
                                          "notch z=0.5 over x<0.3, 1 MPa step traction")
    if name == "block8m":
        return mg.block_notched(220, 110, 55), 1e-6, (
            "notched block 220x110x55 cells x 6 tets at 0.5 mm (7,986,000 tets), "
            "8 pre-split layers over half the length, 1 MPa ramped")
    if name == "block":
        return mg.block_notched(), 1e-6, ("notched block 400x200x100 cells x 6 tets at 0.5 mm "
                                          "(48,000,000 tets), 2% pre-split, 1 MPa ramped")
    if name == "dirichlet":
        m = mg.plate_notched()
        m.load_tris, m.load_trac = None, None
        return m, 0.0, ("notched plate 100x40x4 mm, 200x80x8 cells x 6 tets (768,000 tets), "
                        "velocity-driven: face y = 40 mm at +0.2 m/s in y ramped over 1 us, "
                        "face y = 0 held in y")
    raise SystemExit(f"unknown workload {name}")


def velocity_groups(name, mesh):
    """Prescribed-velocity groups of a workload: (nodes, dof masks, v0 [n][3], t0)."""
    if name != "dirichlet":
        return []
    y = mesh.X[:, 1]
    top = np.nonzero(np.abs(y - y.max()) < 1e-12)[0]
    bot = np.nonzero(np.abs(y - y.min()) < 1e-12)[0]
    vt = np.zeros((len(top), 3))
    vt[:, 1] = 0.2
    return [(top, np.full(len(top), 2), vt, 1e-6),
            (bot, np.full(len(bot), 2), np.zeros((len(bot), 3)), 0.0)]


def kernel_source_hash():
    """SHA-256 over every HIP source and header of the library (file name and
    contents, in name order): the kernels, their helpers and the host runtime,
    whose node and element order also set the traffic."""
    d = os.path.join(ROOT, "paper_2508_04076_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode() + b"\0" + open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def copy_peak_gbs(nbytes=1 << 30, reps=10):
    """Read+write GB/s of a plain device-to-device copy of nbytes (torch's
    current stream, timed with events after three untimed copies)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def counters_for(kernel_src_hash, workload="plate"):
    """HBM traffic per launch of `workload` from the committed rocprofv3 counter
    summaries (profiles/hbm_counters.json, else hbm_counters_<workload>.json),
    if they were taken on the current kernel source."""
    for name in ("hbm_counters.json", f"hbm_counters_{workload}.json"):
        p = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(p):
            continue
        try:
            d = json.load(open(p))
        except Exception:
            continue
        if d.get("workload") != workload:
            continue
        return d if d.get("kernel_source_sha256") == kernel_src_hash else None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="plate",
                    choices=["plate", "cube", "block8m", "block", "ensemble", "window",
                             "dirichlet", "hex", "hexblock"])
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps for the CPU baseline (0: about 15 s of work)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--launch", default="",
                    help="fixed launch shape grid_cap,lanes,layout (e.g. 2048,4,stress_sums) "
                         "instead of the autotuner")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="ensemble workload only (default mixed)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes, 5 times "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n,
                          "launches": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(it would shard by node slabs with a halo exchange per step)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_04076_amd import meshgen as mg
    from paper_2508_04076_amd.cem import Simulation

    mat = dict(mg.BRANCHING_MATERIAL)
    if args.workload == "ensemble":
        return bench_ensemble(args)
    if args.workload == "window":
        return bench_window(args)
    if args.workload in ("hex", "hexblock"):
        return bench_hex(args)
    mesh, ramp, desc = workload(args.workload)
    T = mesh.n_tets
    log(f"workload {args.workload}: {T} tets, {mesh.n_nodes} nodes")
    K, W = args.steps, args.warmup
    if not args.no_graph:
        W = max(W, args.graph_steps)  # the first graph is captured in the warm-up
    max_splits = max(T // 8, len(mesh.presplit_tets) + 20000)

    tuned = {}

    groups = velocity_groups(args.workload, mesh)

    def make(precision, graph):
        s_ = Simulation.from_mesh(mesh, mat, ramp_t0=ramp, precision=precision,
                                  max_splits=max_splits, graph_steps=graph, device=0)
        for g_ in groups:
            s_.add_velocity_bc(*g_)
        if tuned:
            s_.set_launch(tuned["grid_cap"], tuned["lanes"], tuned["layout"])
        return s_

    # ---- 0. launch shape from the library's autotuner, on a warmed-up copy
    gs = 0 if args.no_graph else args.graph_steps
    sim = make("fp64", 0)
    dt = 0.5 * sim.critical_dt()
    if args.launch:
        g_, l_, lay_ = args.launch.split(",")
        tuned.update(grid_cap=int(g_), lanes=int(l_), layout=lay_)
        sim.set_launch(tuned["grid_cap"], tuned["lanes"], tuned["layout"])
    elif not args.no_tune:
        sim.set_dt(dt)
        sim.step(W)
        tuned.update(sim.autotune(trial_steps=10))
        log(f"autotuned launch: {tuned}")
        sim.close()
        sim = make("fp64", 0)

    # ---- 1. FP64, plain launches with per-pass HIP events on the library's
    # stream: the kernel times of the roofline (and the timed region when
    # graphs are off)
    sim.set_dt(dt)
    log(f"dt = {dt:.6e} s; warmup {W} steps")
    sim.set_profiling(True)
    sim.step(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = sim.kernel_times()
    reaction = None
    if groups:
        rows, work = sim.reactions(0)
        reaction = {"driven_face_reaction_N_last": rows[-1, 2:5].tolist(),
                    "driven_face_work_J": work, "rows": len(rows)}
    u64, _, _ = sim.get_state()
    e64 = sim.energy()
    ev64, _ = sim.splits()
    log(f"fp64 (plain launches, per-pass events): "
        f"{wall * 1e3 / K:.4f} ms/step, {T * K / wall:.4e} tet-steps/s, splits {e64['n_split']}")
    per_launch = {k: kt[k] / K for k in ("strain", "edge_stress", "front", "elem_force",
                                          "node_sum", "node", "topology")}
    sim.close()

    # ---- 2. FP64 as captured HIP graphs without events, same steps: the
    # timed region of `value` (tet-steps/s over graph replays)
    graph, handover = None, None
    if not args.no_graph and gs > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = make("fp64", gs)
        torch.cuda.synchronize()
        t_up = time.perf_counter() - t0
        g.set_dt(dt)
        g.step(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(K)
        torch.cuda.synchronize()
        gw = time.perf_counter() - t0
        t0 = time.perf_counter()
        ug, vg, _ = g.get_state()
        t_rd = time.perf_counter() - t0
        graph = {"ms_per_step": gw * 1e3 / K, "tet_steps_per_s": T * K / gw,
                 "graph_steps": gs,
                 "bitwise_equal_to_per_pass_run": bool(np.array_equal(ug, u64))}
        log(f"fp64 graphs without events: {gw * 1e3 / K:.4f} ms/step, {T * K / gw:.4e} tet-steps/s")
        t0 = time.perf_counter()
        g.set_state(ug, vg)
        torch.cuda.synchronize()
        t_wr = time.perf_counter() - t0
        # the boundary's host hand-overs, outside the timed region of `value`
        handover = {
            "mesh_upload_s": t_up, "state_readback_ms": t_rd * 1e3, "state_set_ms": t_wr * 1e3,
            "tet_steps_per_s_with_readback": T * K / (gw + t_rd),
            "tet_steps_per_s_with_upload_and_readback": T * K / (t_up + gw + t_rd),
            "note": ("mesh upload = host preprocessing (order, edges, patches, node lists) plus "
                     "host-to-device copies, once per run; readback = u, v, a to host; "
                     f"rates over the {K} timed graph steps"),
        }
        log(f"host hand-over: upload {t_up:.2f} s, state readback {t_rd * 1e3:.2f} ms, "
            f"set {t_wr * 1e3:.2f} ms")
        g.close()

    # ---- 2b. the same steps as plain launches without events: the library's
    # other execution mode (graph_steps 0)
    plain = None
    if not args.no_graph and gs > 0:
        p_ = make("fp64", 0)
        p_.set_dt(dt)
        p_.step(W)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_.step(K)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t0
        up, _, _ = p_.get_state()
        plain = {"ms_per_step": pw * 1e3 / K, "tet_steps_per_s": T * K / pw,
                 "bitwise_equal_to_per_pass_run": bool(np.array_equal(up, u64))}
        log(f"fp64 plain launches without events: {pw * 1e3 / K:.4f} ms/step, "
            f"{T * K / pw:.4e} tet-steps/s")
        p_.close()

    # ---- 3. mixed precision, FP64 split schedule replayed
    mixed = None
    if not args.no_mixed:
        mx = make("mixed", args.graph_steps if not args.no_graph else 0)
        mx.set_dt(dt)
        sched = ev64[ev64[:, 3] > 0][:, :3]
        if len(sched):
            mx.replay_splits(sched)
        mx.step(W)
        tuned_mx = None
        if not args.launch and not args.no_tune:
            # its own launch shape (the tuner restores the state after each trial)
            tuned_mx = mx.autotune(trial_steps=10)
            log(f"autotuned launch (mixed): {tuned_mx}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mx.step(K)
        torch.cuda.synchronize()
        mw = time.perf_counter() - t0
        um, _, _ = mx.get_state()
        err = float(np.linalg.norm(um - u64) / np.linalg.norm(u64))
        mixed = {"tet_steps_per_s": T * K / mw, "ms_per_step": mw * 1e3 / K,
                 "rel_l2_u_vs_fp64": err, "steps_compared": W + K,
                 "split_schedule": "fp64 run replayed", "dtype": "f32 force / f64 state",
                 "autotune": tuned_mx}
        log(f"mixed: {mw * 1e3 / K:.4f} ms/step, {T * K / mw:.4e} tet-steps/s, "
            f"rel L2 u err {err:.3e}")
        mx.close()

    # ---- roofline of the dominant pass (largest average time per step)
    dom = max(("strain", "edge_stress", "node"), key=lambda k: per_launch[k])
    dur_s = per_launch[dom] * 1e-3
    alg = ALG_BYTES["fp64"][dom] * T
    achieved = alg / dur_s / 1e9
    cnt = counters_for(kernel_source_hash(), args.workload)
    if cnt and cnt.get("layout", "terms") != tuned.get("layout", "terms"):
        cnt = None  # counters of the other force layout
    traffic = None
    if cnt and cnt.get("workload") == args.workload and \
            all(k in cnt.get("kernels", {}) for k in KERNEL_NAMES[dom]):
        traffic = sum(cnt["kernels"][k]["hbm_bytes_per_launch"] for k in KERNEL_NAMES[dom])
    roofline = {"bound": "hbm", "kernel": "+".join(KERNEL_NAMES[dom]), "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic, "alg_bytes_per_tet": ALG_BYTES["fp64"][dom],
                "avg_launch_ms": per_launch[dom]}

    # ---- HBM GB/s of the step: model bytes x rate ("effective"), and counted
    # bytes (rocprofv3 counters of this source) over each pass's event time,
    # against the spec and a device copy measured here
    per_pass_run = {"ms_per_step": wall * 1e3 / K, "tet_steps_per_s": T * K / wall,
                    "launch": "plain launches with per-pass HIP events (the kernel times above)"}
    modes = {k: v for k, v in (("graphs", graph), ("plain", plain)) if v}
    if modes:
        best = max(modes, key=lambda k: modes[k]["tet_steps_per_s"])
        value, ms_step = modes[best]["tet_steps_per_s"], modes[best]["ms_per_step"]
        launch_desc = (f"HIP graphs of {gs} steps, no events" if best == "graphs"
                       else "plain launches, no events")
        if len(modes) > 1:
            launch_desc += " (the faster of graphs and plain launches here; both under 'modes')"
    else:
        value, ms_step = per_pass_run["tet_steps_per_s"], per_pass_run["ms_per_step"]
        launch_desc = per_pass_run["launch"]
    hbm = {"spec_gbs": HBM_PEAK_GBS, "copy_peak_gbs": copy_peak_gbs(),
           "effective_gbs_fp64": sum(ALG_BYTES["fp64"].values()) * value / 1e9,
           "alg_bytes_per_tet_fp64": sum(ALG_BYTES["fp64"].values())}
    if mixed:
        hbm["effective_gbs_mixed"] = sum(ALG_BYTES["mixed"].values()) * mixed["tet_steps_per_s"] / 1e9
    if cnt and cnt.get("workload") == args.workload and \
            all(k in cnt.get("kernels", {}) for p_ in KERNEL_NAMES for k in KERNEL_NAMES[p_]):
        counted, tb, tt = {}, 0.0, 0.0
        for p_, names in KERNEL_NAMES.items():
            b_ = sum(cnt["kernels"][k]["hbm_bytes_per_launch"] for k in names)
            counted[p_] = {"bytes_per_launch": b_, "gbs": b_ / (per_launch[p_] * 1e-3) / 1e9}
            tb += b_
            tt += per_launch[p_] * 1e-3
        hbm["counted"] = counted
        hbm["counted_gbs_s_e_f"] = tb / tt / 1e9
        hbm["counted_note"] = ("bytes from FETCH_SIZE and WRITE_SIZE (scaled by a plain copy) at "
                               "the library's default launch shape; times from this run's events")

    # ---- 4. CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        from oracle.oracle import Oracle
        o = Oracle.from_mesh(mesh, mat, ramp_t0=ramp)
        for g_ in groups:
            o.add_velocity_bc(*g_)
        o.set_dt(dt)
        n_cpu = args.cpu_steps
        if n_cpu <= 0:
            t0 = time.perf_counter()
            o.step(1)
            one = time.perf_counter() - t0
            n_cpu = max(1, min(200, int(20.0 / max(one, 1e-6))))
            done = 1
        else:
            done = 0
        log(f"oracle: {n_cpu} steps on the host")
        t0 = time.perf_counter()
        o.step(n_cpu - done)
        el = time.perf_counter() - t0
        n_timed = n_cpu - done
        if n_timed == 0:
            n_timed, el = 1, one
        cpu = {"value": T * n_timed / el, "unit": "tet-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_timed} steps of the same workload from t=0 (single-threaded FP64 "
                         f"C++ oracle, {el:.1f} s)",
               "host_cpus": os.cpu_count()}

    out = {
        "metric": METRIC, "value": value, "unit": "tet-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "tets": T, "nodes": mesh.n_nodes,
                   "dt_s": dt, "splits_after_run": int(e64["n_split"]),
                   "launch": launch_desc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": per_launch,
        "hbm": hbm,
        "autotune": tuned or None,
        "per_pass_run": per_pass_run,
        "modes": modes or None,
        "mixed": mixed,
        "host_handover": handover,
    }
    if reaction:
        out["reactions"] = reaction
    print(json.dumps(out), flush=True)


def bench_ensemble(args):
    """64 notched plates of seeded sizes 20k-200k tets and tractions 0.5-2 MPa,
    stepped together as one batch (one launch per pass, captured graphs), each
    with its own time step; launch shape picked by the library's autotuner."""
    import torch
    from paper_2508_04076_amd import meshgen as mg
    from paper_2508_04076_amd.cem import Simulation

    mat = dict(mg.BRANCHING_MATERIAL)
    prec = args.precision or "mixed"
    un, node_off, tet_off, members, trac = mg.ensemble(64)
    T = un.n_tets
    log(f"ensemble: 64 plates, {T} tets, {un.n_nodes} nodes, precision {prec}")
    K, W = args.steps, args.warmup
    if not args.no_graph:
        W = max(W, args.graph_steps)  # the first graph is captured in the warm-up
    gs = 0 if args.no_graph else args.graph_steps
    # every tet splits at most once: capacity T can never run out, however far
    # the high-traction members fragment
    sim = Simulation(un.X, un.tets, mat, precision=prec, max_splits=T, graph_steps=gs)
    sim.set_instances(node_off, tet_off)
    sim.set_traction(un.load_tris, un.load_trac, 1e-6)
    sim.presplit(un.presplit_tets, un.presplit_masks)
    dts = 0.5 * sim.critical_dt_instances()
    sim.set_dt_instances(dts)
    sim.step(W)
    tuned = sim.autotune(trial_steps=10)
    log(f"autotuned launch: {tuned}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    e = sim.energy_instances()
    value = T * K / wall
    log(f"ensemble {prec}: {wall * 1e3 / K:.4f} ms/step, {value:.4e} tet-steps/s")
    sim.set_profiling(True)
    sim.step(min(K, 200))
    kt = sim.kernel_times()
    nK = min(K, 200)
    per = {k: kt[k] / nK for k in ("strain", "edge_stress", "front", "elem_force", "node_sum",
                                    "node", "topology")}
    alg = ALG_BYTES[prec]["node"] * T
    achieved = alg / (per["node"] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "tet-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": wall * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 force / f64 state" if prec == "mixed"
        else "f64", "data": "synthetic",
        "config": {"workload": "batch of 64 notched plates, 20k-200k tets each (seed 2), "
                               "tractions 0.5-2 MPa, one launch per pass",
                   "tets": T, "instances": 64, "dt_range_s": [float(dts.min()), float(dts.max())],
                   "launch": f"HIP graphs of {gs} steps; autotuned grid {tuned['grid_cap']}, "
                             f"{tuned['lanes']} lanes per node",
                   "splits_after_run": int(sum(x["n_split"] for x in e))},
        "roofline": {"bound": "hbm", "kernel": "k_elem_force+k_node", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_tet": ALG_BYTES[prec]["node"],
                     "avg_launch_ms": per["node"]},
        "cpu_baseline": None,
        "kernels_ms_per_step": per,
        "autotune": tuned,
    }
    sim.close()
    print(json.dumps(out), flush=True)

# Algorithmic bytes per tet of one reverse step, from the same per-pass
# figures: the reverse strain pass gathers two displacement fields and writes
# two strain records (S with the u gather and the write doubled); the reverse
# edge pass sums two patches and also writes z and reads 1/S (E with the V_eff
# eps read doubled, plus z, einvV and einv0 per edge at E/T = 1.24); the
# reverse force pass is F plus z (per edge), gE read+write (per tet) and the
# extra adjoint node state (p, q read+write, lambda write, N/T = 0.19).
ADJ_BYTES = {
    "fp64": {"strain2": 16 + 80 + 2 * 4.6 + 2 * 48, "edge2": 29 + 2 * 48 + 59 + 3 * 10,
             "force2": 200 + 10 + 16 + 5},
    "mixed": {"strain2": 16 + 40 + 2 * 4.6 + 2 * 24, "edge2": 29 + 2 * 24 + 30 + 3 * 5,
              "force2": 130 + 5 + 16 + 5},
}


def bench_window(args):
    """Gradient window on the 202,800-tet notched plate (130 x 52 x 5 cells)
    with a lognormal per-tet modulus (E = 32 GPa exp(0.1 z), seed 3): 500
    fixed-topology steps forward with a checkpoint every 50, then the reverse
    sweep (segment recompute + reverse steps) giving dJ/dE, dJ/du0, dJ/dv0 for
    J = SE(u_500), the strain energy at the window's end (dJ/dE = the explicit
    dSE/dE at fixed u plus the window adjoint with gu = K u_500).  A step here
    is one forward step plus its share of the backward."""
    import torch
    from paper_2508_04076_amd import meshgen as mg
    from paper_2508_04076_amd.cem import Simulation

    mat = dict(mg.BRANCHING_MATERIAL)
    prec = args.precision or "fp64"
    n_win, every = 500, 50
    mesh = mg.plate_window()
    E = mg.modulus_field(mesh.n_tets, mat["E"], 0.1, seed=3)
    T = mesh.n_tets
    log(f"window: {T} tets, {mesh.n_nodes} nodes, {n_win} steps, checkpoint every {every}, {prec}")
    sim = Simulation.from_mesh(mesh, mat, ramp_t0=1e-6, precision=prec, E_tet=E,
                               max_splits=4000, graph_steps=args.graph_steps)
    dt = 0.5 * sim.critical_dt()
    sim.set_dt(dt)
    n = sim.n_nodes
    zero = np.zeros((n, 3))
    # launch shape (force layout, grid, lanes) for the forward and reverse passes
    tuned = None
    if args.launch:
        g_, l_, lay_ = args.launch.split(",")
        sim.set_launch(int(g_), int(l_), lay_)
        tuned = {"grid_cap": int(g_), "lanes": int(l_), "layout": lay_}
    elif not args.no_tune:
        sim.step(every)
        tuned = sim.autotune(trial_steps=10)
        log(f"autotuned launch: {tuned}")

    def one(n_steps, profiled):
        sim.set_profiling(profiled)
        sim.set_state(zero, zero)
        sim.set_step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.window_forward(n_steps, every)
        t1 = time.perf_counter()
        se, gu, g_exp = sim.strain_energy_grad()
        g = sim.window_backward(gu, None)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, (g[0], g[1], g[2] + g_exp, se)

    one(every, False)  # warm-up: graphs, buffers
    f_s, b_s, _ = one(n_win, False)
    value = T * n_win / (f_s + b_s)
    log(f"window: forward {f_s * 1e3:.2f} ms, backward {b_s * 1e3:.2f} ms, "
        f"{value:.4e} tet-steps/s (forward + backward)")
    # timed region with per-kernel HIP events (plain launches)
    fp, bp, g = one(n_win, True)
    wt = sim.window_times()
    per = {k: wt[k] / n_win for k in ("strain2", "edge2", "elem_adj", "node_adj")}
    per["force2"] = per["elem_adj"] + per["node_adj"]
    per["recompute_step"] = wt["recompute"] / n_win
    alg = ADJ_BYTES[prec]
    rows = {k: alg[k] * T / (per[k] * 1e-3) / 1e9 for k in ("strain2", "edge2", "force2")}
    dom = max(("strain2", "edge2", "force2"), key=lambda k: per[k])
    names = {"strain2": "k_strain2", "edge2": "k_edge2", "force2": "k_elem_adj+k_node_adj"}
    cpu = None
    if not args.no_cpu:
        cpu = window_cpu_baseline(mesh, mat, E, dt, np.random.default_rng(9).standard_normal((n, 3)))
    out = {
        "metric": "adjoint window tet-steps/s (forward + backward, checkpointed)",
        "value": value, "unit": "tet-steps/s", "n_gpus": 1, "steps": n_win, "warmup": every,
        "ms_per_step": (f_s + b_s) * 1e3 / n_win, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32 force / f64 state",
        "data": "synthetic",
        "config": {"workload": "gradient window: notched plate 100x40x4 mm at 130x52x5 cells "
                               "(202,800 tets), lognormal modulus sigma 0.1 (seed 3), 500 steps, "
                               "checkpoint every 50, J = strain energy at step 500",
                   "forward_ms": f_s * 1e3, "backward_ms": b_s * 1e3,
                   "profiled_forward_ms": fp * 1e3, "profiled_backward_ms": bp * 1e3,
                   "dJ_dE_norm": float(np.linalg.norm(g[2])), "J": g[3]},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": rows[dom],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rows[dom] / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_tet": alg[dom],
                     "avg_launch_ms": per[dom]},
        "reverse_kernels_ms_per_step": per,
        "reverse_kernels_gbs": rows,
        "autotune": tuned,
        "cpu_baseline": cpu,
    }
    sim.close()
    print(json.dumps(out), flush=True)


def window_cpu_baseline(mesh, mat, E, dt, gu, n_steps=8):
    """The oracle's window gradient on the same mesh for a few steps."""
    from oracle.oracle import Oracle
    t0 = time.perf_counter()
    o = Oracle.from_mesh(mesh, mat, ramp_t0=1e-6, E_tet=E)
    o.set_dt(dt)
    t1 = time.perf_counter()
    o.window_gradient(n_steps, gu, None)
    t2 = time.perf_counter()
    log(f"oracle window: setup {t1 - t0:.1f} s, {n_steps} steps fwd+bwd {t2 - t1:.1f} s")
    return {"value": mesh.n_tets * n_steps / (t2 - t1), "unit": "tet-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_steps}-step window forward + reverse on the same 202,800-tet mesh "
                      "(oracle setup excluded)"}


# Algorithmic bytes per hex-step of the hexahedral passes (compulsory traffic,
# FP64 / mixed), with E/H = 3 edges and N/H = 1 node per hex on a structured
# grid: strain = ids 32 + G 192 + u gather 32 + write V eps 48; edge = CSR
# 4 (E/H) + 48 + read V eps 48 + write sigma 48 (E/H) + einvV 8 (E/H);
# force = ids 84 (12 edge ids 48, node lists 36) + G 192 + read sigma 48 (E/H)
# + u, v read+write 96 + 1/m 8.  The per-hex stress sum handed from the element
# pass to the node pass is an intermediate, not counted.
HEX_BYTES = {
    "fp64": {"strain": 32 + 192 + 32 + 48, "edge_stress": 12 + 48 + 48 + 144 + 24,
             "node": 84 + 192 + 144 + 96 + 8},
    "mixed": {"strain": 32 + 192 + 32 + 24, "edge_stress": 12 + 48 + 24 + 72 + 12,
              "node": 84 + 192 + 72 + 96 + 8},
}


def bench_hex(args):
    """Trilinear hexahedra (ES-H-FEM, factor 1/12): the notched-plate geometry
    at 200 x 80 x 8 hex cells (128,000 hexes, 1 MPa ramped over 1 us), or a
    400 x 200 x 100 block (8,000,000 hexes).  No splitting (hexahedra do not
    split).  A step: strain, edge stress, element force + node update."""
    import torch
    from paper_2508_04076_amd import meshgen as mg
    from paper_2508_04076_amd.cem import Simulation

    mat = dict(mg.BRANCHING_MATERIAL)
    if args.workload == "hex":
        mesh = mg.add_tension(mg.hex_box(200, 80, 8, 0.1, 0.04, 0.004), 1, 1e6)
        desc = ("plate 100x40x4 mm as 200x80x8 trilinear hex cells (128,000 hexes), "
                "1 MPa traction ramped over 1 us, no splitting")
    else:
        mesh = mg.add_tension(mg.hex_box(400, 200, 100, 0.2, 0.1, 0.05), 1, 1e6)
        desc = ("block 200x100x50 mm as 400x200x100 trilinear hex cells (8,000,000 hexes), "
                "1 MPa traction ramped over 1 us, no splitting")
    H = mesh.n_hex
    K, W = args.steps, args.warmup
    if not args.no_graph:
        W = max(W, args.graph_steps)  # the first graph is captured in the warm-up
    log(f"hex workload {args.workload}: {H} hexes, {mesh.n_nodes} nodes")
    out_runs = {}
    for prec in ("fp64", "mixed"):
        if prec == "mixed" and args.no_mixed:
            continue
        for graph in (False, True):
            if graph and args.no_graph:
                continue
            sim = Simulation.from_hex_mesh(mesh, mat, ramp_t0=1e-6, precision=prec,
                                           graph_steps=args.graph_steps if graph else 0)
            dt = 0.5 * sim.critical_dt()
            sim.set_dt(dt)
            sim.set_profiling(not graph)
            sim.step(W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(K)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            run = {"ms_per_step": wall * 1e3 / K, "hex_steps_per_s": H * K / wall, "dt_s": dt}
            if not graph:
                kt = sim.kernel_times()
                run["kernels_ms_per_step"] = {k: kt[k] / K for k in
                                              ("strain", "edge_stress", "node", "topology")}
                run["u"] = sim.get_state()[0]
            out_runs[(prec, graph)] = run
            log(f"hex {prec} {'graphs' if graph else 'plain+events'}: {wall * 1e3 / K:.4f} ms/step, "
                f"{H * K / wall:.4e} hex-steps/s")
            sim.close()
    base = out_runs[("fp64", False)]
    per = base["kernels_ms_per_step"]
    dom = max(("strain", "edge_stress", "node"), key=lambda k: per[k])
    achieved = HEX_BYTES["fp64"][dom] * H / (per[dom] * 1e-3) / 1e9
    names = {"strain": "k_strain_hex", "edge_stress": "k_edge_stress",
             "node": "k_elem_force_hex+k_node"}
    mixed = None
    if ("mixed", False) in out_runs:
        um, u64 = out_runs[("mixed", False)]["u"], base["u"]
        mixed = {"hex_steps_per_s": out_runs[("mixed", False)]["hex_steps_per_s"],
                 "ms_per_step": out_runs[("mixed", False)]["ms_per_step"],
                 "graph_hex_steps_per_s": out_runs.get(("mixed", True), {}).get("hex_steps_per_s"),
                 "rel_l2_u_vs_fp64": float(np.linalg.norm(um - u64) / np.linalg.norm(u64))}
    cpu = None
    if not args.no_cpu:
        from oracle.oracle import Oracle
        o = Oracle.hex_mesh(mesh, mat, ramp_t0=1e-6)
        o.set_dt(base["dt_s"])
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        n_cpu = max(1, min(100, int(15.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        o.step(n_cpu)
        el = time.perf_counter() - t0
        cpu = {"value": H * n_cpu / el, "unit": "hex-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"{n_cpu} steps of the same hex workload after one warm-up step "
                         f"(single-threaded FP64 oracle, {el:.1f} s)"}
    timed = out_runs.get(("fp64", True), base)
    out = {
        "metric": "hex-steps/sec (ES-H-FEM), FP64 and FP32-mixed",
        "value": timed["hex_steps_per_s"], "unit": "hex-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": timed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "hexes": H, "nodes": mesh.n_nodes, "dt_s": base["dt_s"],
                   "launch": (f"HIP graphs of {args.graph_steps} steps, no events"
                              if timed is not base else "plain launches with per-pass HIP events")},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_hex": HEX_BYTES["fp64"][dom],
                     "avg_launch_ms": per[dom]},
        "kernels_ms_per_step": per,
        "per_pass_run": {"hex_steps_per_s": base["hex_steps_per_s"], "ms_per_step": base["ms_per_step"],
                         "launch": "plain launches with per-pass HIP events (the kernel times above)"},
        "mixed": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)



if __name__ == "__main__":
    main()
