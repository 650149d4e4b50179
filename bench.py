"""Throughput of the ES-T-FEM crack-element step on one MI355X.

Default workload: the large notched block, 400 x 200 x 100 cells of 0.5 mm x
6 tets = 48,000,000 tets (8,140,701 nodes), notch plane y = 50 mm over
x < 100 mm with 960,000 pre-split tets (2%), +-1 MPa traction in y ramped
over 1 us, splitting on; the headline precision is FP32 forces with FP64
state, FP64 is reported beside it.  A step is the whole hot path: strain
pass, edge stress pass, crack-front pass with flag compaction, node force +
Newmark pass, topology update.  `--workload plate` is the 768,000-tet notched
plate of the crack-branching example (Section 4.4), FP64 headline.

Prints one JSON line.  The mesh is uploaded once; every timed run starts
from one checkpoint:
  0. FP64 from t = 0 through --advance steps (past the onset of dynamic
     splitting) and --warmup steps: checkpoint C0;
  1. per precision (FP64, then mixed on the same state): the library's
     autotuner picks the launch shape from C0; then --steps steps from C0
     three times: plain launches with per-pass HIP events on the library's
     stream (kernel durations, roofline), HIP graphs of min(--graph-steps,
     --steps) steps, plain launches; `value` is the faster of the last two
     in the headline precision, each bitwise equal to the events run;
  2. mixed precision from t = 0 to the end of the window with the FP64 split
     schedule replayed (relative L2 error of u), and free-running (split
     events that differ);
  3. the CPU oracle on a bounded sample at one thread and every core.
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
# the force pass is two launches: per-element force terms (with the crack-front
# workgroups riding along), then per-node sums; in the tiled layout, the
# crack-front launch, the tiled force + node launch and the node pass of the
# split copies' extra nodes
KERNEL_NAMES = {"strain": ["k_strain"], "edge_stress": ["k_edge_stress"],
                "node": ["k_elem_force_front", "k_node"]}
KERNEL_NAMES_TILES = dict(KERNEL_NAMES, node=["k_front", "k_force_tile", "k_node"])
KERNEL_NAMES_TILES_FX = dict(KERNEL_NAMES, node=["k_front", "k_force_fx", "k_node"])


def kernel_names(layout):
    return {"tiles": KERNEL_NAMES_TILES, "tiles_fx": KERNEL_NAMES_TILES_FX}.get(layout, KERNEL_NAMES)
# steps before the warm-up by default: past the onset of dynamic splitting
DEFAULT_ADVANCE = {"block": 1000, "block8m": 600, "plate": 600, "dirichlet": 600, "cube": 200}


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


def counters_for(kernel_src_hash, workload, precision, layout):
    """HBM traffic per launch from the committed rocprofv3 counter summary
    profiles/hbm_counters_<workload>_<precision>_<layout>.json, if it was taken
    on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"hbm_counters_{workload}_{precision}_{layout}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("workload") != workload or d.get("precision") != precision:
        return None
    if d.get("kernel_source_sha256") != kernel_src_hash or d.get("layout", "terms") != layout:
        return None
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="block",
                    choices=["plate", "cube", "block8m", "block", "ensemble", "window",
                             "dirichlet", "hex", "hexblock"])
    ap.add_argument("--advance", type=int, default=-1,
                    help="steps before the warm-up, to put the timed window past the onset of "
                         "dynamic splitting (-1: the workload's default)")
    ap.add_argument("--headline", default=None, choices=["fp64", "mixed"],
                    help="precision of `value` (default: mixed for the blocks, else fp64)")
    ap.add_argument("--graph-steps", type=int, default=50,
                    help="steps per HIP graph (capped at --steps)")
    ap.add_argument("--no-error", action="store_true",
                    help="skip the mixed-versus-FP64 runs from t = 0 (counter runs)")
    ap.add_argument("--error-steps", type=int, default=0,
                    help="length of the mixed-versus-FP64 error runs from t = 0 (default: to the "
                         "end of the timed window)")
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
    K, W = args.steps, args.warmup
    head = args.headline or ("mixed" if args.workload in ("block", "block8m") else "fp64")
    if args.no_mixed:
        head = "fp64"
    adv = args.advance if args.advance >= 0 else DEFAULT_ADVANCE.get(args.workload, 0)
    gs = 0 if args.no_graph else min(args.graph_steps, K)
    n_pre = len(mesh.presplit_tets) if mesh.presplit_tets is not None else 0
    max_splits = n_pre + max(T // 50, 20000)
    log(f"workload {args.workload}: {T} tets, {mesh.n_nodes} nodes; headline {head}; "
        f"advance {adv}, warmup {W}, timed {K} steps, graphs of {gs}")
    groups = velocity_groups(args.workload, mesh)

    # ---- one upload; every run below rewinds to a checkpoint
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = Simulation.from_mesh(mesh, mat, ramp_t0=ramp, precision="fp64",
                               max_splits=max_splits, graph_steps=0, device=0)
    for g_ in groups:
        sim.add_velocity_bc(*g_)
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t0
    log(f"mesh upload {t_up:.1f} s")
    dt = 0.5 * sim.critical_dt()
    sim.set_dt(dt)
    ck_init = sim.save_state() if not (args.no_mixed or args.no_error) else None
    # run up to the timed window (past the onset of dynamic splitting where the
    # load reaches the notch in time), then the warm-up steps
    done = 0
    while done < adv:
        n = min(250, adv - done)
        sim.step(n)
        done += n
        e = sim.energy()
        log(f"advance: step {done}, splits {e['n_split']} ({e['n_split'] - n_pre} dynamic), "
            f"fronts {e['n_front']}, Gmax {e['Gmax']:.3g}")
    sim.step(W)
    ck0 = sim.save_state()
    step0 = int(sim.energy()["step"])

    def timed(prec_ck, graph, profiled=False):
        """K steps from the checkpoint; returns seconds, final u, energy, last-run record."""
        sim.load_state(prec_ck)
        sim.set_graph_steps(graph)
        sim.set_profiling(profiled)
        torch.cuda.synchronize()
        t0_ = time.perf_counter()
        sim.step(K)
        torch.cuda.synchronize()
        wall_ = time.perf_counter() - t0_
        sim.set_profiling(False)
        return wall_, sim.get_state()[0], sim.energy(), sim.last_run()

    def one_precision(prec, ck):
        """Autotuned shape, per-pass events run, graph run, plain run."""
        res = {}
        tuned_ = None
        if args.launch:
            g_, l_, lay_ = args.launch.split(",")
            sim.set_launch(int(g_), int(l_), lay_)
            tuned_ = {"grid_cap": int(g_), "lanes": int(l_), "layout": lay_, "source": "--launch"}
        elif not args.no_tune:
            sim.load_state(ck)
            sim.set_graph_steps(0)
            tuned_ = sim.autotune(trial_steps=10)
            log(f"autotuned launch ({prec}): {tuned_}")
        wall_, u_pp, e_, _ = timed(ck, 0, profiled=True)
        kt = sim.kernel_times()
        res["per_pass"] = {"ms_per_step": wall_ * 1e3 / K, "tet_steps_per_s": T * K / wall_,
                           "launch": "plain launches with per-pass HIP events"}
        res["kernels_ms_per_step"] = {k: kt[k] / K for k in ("strain", "edge_stress", "front",
                                                             "elem_force", "node_sum", "node",
                                                             "topology")}
        log(f"{prec} per-pass events: {wall_ * 1e3 / K:.4f} ms/step")
        modes_ = {}
        for name, graph in (("graphs", gs), ("plain", 0)):
            if name == "graphs" and gs == 0:
                continue
            w_, u_, e2, lr = timed(ck, graph)
            modes_[name] = {"ms_per_step": w_ * 1e3 / K, "tet_steps_per_s": T * K / w_,
                            "graph_launches": lr["graph_launches"], "graph_steps": lr["graph_steps"],
                            "plain_steps": lr["plain_steps"],
                            "bitwise_equal_to_per_pass_run": bool(np.array_equal(u_, u_pp))}
            log(f"{prec} {name}: {w_ * 1e3 / K:.4f} ms/step, {T * K / w_:.4e} tet-steps/s ({lr})")
        best_ = max(modes_, key=lambda k: modes_[k]["tet_steps_per_s"])
        res.update(modes=modes_, best=best_, autotune=tuned_, u_end=u_pp,
                   splits_in_window=int(e_["n_split"]) - n_split0, energy=e_)
        return res

    n_split0 = int(sim.energy()["n_split"])
    runs = {"fp64": one_precision("fp64", ck0)}
    ev64, _ = sim.splits()
    u64_end = runs["fp64"]["u_end"]
    host = {"mesh_upload_s": t_up}
    t0 = time.perf_counter()
    ug, _, _ = sim.get_state()
    host["state_readback_ms"] = (time.perf_counter() - t0) * 1e3
    mixed_err = None
    if not args.no_mixed:
        # the same state in mixed precision: switch the arithmetic, keep the rest
        sim.load_state(ck0)
        sim.set_precision("mixed")
        ck0m = sim.save_state()
        runs["mixed"] = one_precision("mixed", ck0m)
        um = runs["mixed"]["u_end"]
        win_err = float(np.linalg.norm(um - u64_end) / np.linalg.norm(u64_end))
    if not args.no_mixed and not args.no_error:
        # from t = 0 with the FP64 split schedule replayed, and free-running
        n_all = max(step0 + K, args.error_steps)
        sim.set_graph_steps(gs)
        if n_all > step0 + K:
            # a longer FP64 reference run from t = 0
            sim.set_precision("fp64")
            sim.load_state(ck_init)
            t0 = time.perf_counter()
            sim.step(n_all)
            log(f"fp64 reference: {n_all} steps from t = 0 in {time.perf_counter() - t0:.1f} s")
            ev64, _ = sim.splits()
            u64_end = sim.get_state()[0]
        sim.set_precision("fp64")
        sim.load_state(ck_init)
        sim.set_precision("mixed")
        sched = ev64[ev64[:, 3] > 0][:, :3]
        if len(sched):
            sim.replay_splits(sched)
        sim.step(n_all)
        ur, _, _ = sim.get_state()
        rep_err = float(np.linalg.norm(ur - u64_end) / np.linalg.norm(u64_end))
        sim.set_precision("fp64")
        sim.load_state(ck_init)
        sim.set_precision("mixed")
        sim.step(n_all)
        evf, _ = sim.splits()
        a64 = {tuple(r) for r in ev64[:, :3].tolist()}
        af = {tuple(r) for r in evf[:, :3].tolist()}
        mixed_err = {"rel_l2_u_vs_fp64_from_t0_schedule_replayed": rep_err,
                     "steps_from_t0": n_all,
                     "rel_l2_u_vs_fp64_over_timed_window_same_start": win_err,
                     "free_running_split_events": {"fp64": len(a64), "mixed": len(af),
                                                   "only_fp64": len(a64 - af),
                                                   "only_mixed": len(af - a64)}}
        log(f"mixed error: {mixed_err}")
    sim.close()
    del ck_init, ck0

    # ---- roofline of the dominant pass of the headline precision
    hr = runs[head]
    per = hr["kernels_ms_per_step"]
    dom = max(("strain", "edge_stress", "node"), key=lambda k: per[k])

    def roof(prec, r_):
        p_ = r_["kernels_ms_per_step"]
        ach = ALG_BYTES[prec][dom] * T / (p_[dom] * 1e-3) / 1e9
        lay = (r_["autotune"] or {}).get("layout", "terms")
        kn = kernel_names(lay)
        cnt_ = counters_for(kernel_source_hash(), args.workload, prec, lay)
        tr = None
        if cnt_ and all(k in cnt_["kernels"] for k in kn[dom]):
            tr = sum(cnt_["kernels"][k]["hbm_bytes_per_launch"] for k in kn[dom])
        return {"bound": "hbm", "kernel": "+".join(kn[dom]), "achieved": ach, "layout": lay,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": tr, "alg_bytes_per_tet": ALG_BYTES[prec][dom],
                "avg_launch_ms": p_[dom], "precision": prec}, cnt_

    roofline, cnt = roof(head, hr)
    hbm = {"spec_gbs": HBM_PEAK_GBS, "copy_peak_gbs": copy_peak_gbs()}
    for prec, r_ in runs.items():
        v_ = r_["modes"][r_["best"]]["tet_steps_per_s"]
        hbm[f"effective_gbs_{prec}"] = sum(ALG_BYTES[prec].values()) * v_ / 1e9
        hbm[f"alg_bytes_per_tet_{prec}"] = sum(ALG_BYTES[prec].values())
        lay = (r_["autotune"] or {}).get("layout", "terms")
        kn = kernel_names(lay)
        c_ = counters_for(kernel_source_hash(), args.workload, prec, lay)
        if c_ and all(k in c_["kernels"] for p_ in kn for k in kn[p_]):
            counted, tb, tt = {}, 0.0, 0.0
            for p_, names in kn.items():
                b_ = sum(c_["kernels"][k]["hbm_bytes_per_launch"] for k in names)
                t_ = r_["kernels_ms_per_step"][p_] * 1e-3
                counted[p_] = {"bytes_per_launch": b_, "gbs": b_ / t_ / 1e9}
                tb += b_
                tt += t_
            hbm[f"counted_{prec}"] = counted
            hbm[f"counted_gbs_s_e_f_{prec}"] = tb / tt / 1e9

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.workload, mesh, mat, ramp, groups)

    best = hr["best"]
    value, ms_step = hr["modes"][best]["tet_steps_per_s"], hr["modes"][best]["ms_per_step"]
    mb = hr["modes"][best]
    if mb["graph_launches"] > 0:
        launch_desc = (f"{mb['graph_launches']} HIP graph launch(es) of {mb['graph_steps']} steps"
                       + (f" + {mb['plain_steps']} plain steps" if mb["plain_steps"] else "")
                       + ", no events")
    else:
        launch_desc = "plain launches, no events"
    if len(hr["modes"]) > 1:
        launch_desc += " (the faster of graphs and plain launches here; both under 'modes')"

    def strip(r_):
        return {k: v for k, v in r_.items() if k not in ("u_end", "energy")}

    other = [p for p in runs if p != head]
    out = {
        "metric": METRIC, "value": value, "unit": "tet-steps/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 force / f64 state" if head == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": desc, "tets": T, "nodes": mesh.n_nodes, "dt_s": dt,
                   "precision": head,
                   "timed_window_steps": [step0 + 1, step0 + K],
                   "steps_before_window": {"advance": adv, "warmup": W},
                   "dynamic_splits_before_window": n_split0 - n_pre,
                   "dynamic_splits_in_window": hr["splits_in_window"],
                   "launch": launch_desc},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels_ms_per_step": per,
        "hbm": hbm,
        head: strip(hr),
        "mixed_error": mixed_err,
        "host_handover": host,
    }
    for p_ in other:
        out[p_] = strip(runs[p_])
        out[p_]["tet_steps_per_s"] = runs[p_]["modes"][runs[p_]["best"]]["tet_steps_per_s"]
        out[p_]["roofline"] = roof(p_, runs[p_])[0]
    print(json.dumps(out), flush=True)


def cpu_baseline(name, mesh, mat, ramp, groups):
    """The oracle on the host at one thread and at every core of this process's
    CPU share (threads give the same bits), each for about 12 s of stepping
    from t = 0.  The 48M and 8M blocks are too large for the oracle in a
    bench's time: their sample is a 100 x 50 x 25-cell block of the same
    construction (750,000 tets: same cell size, material, load and notch
    rule), whose per-tet cost is the block's."""
    from oracle.oracle import Oracle
    from paper_2508_04076_amd import meshgen as mg
    if name in ("block", "block8m"):
        sm = mg.block_notched(100, 50, 25)
        sample = "100x50x25-cell notched block of the same construction (750,000 tets)"
    else:
        sm = mesh
        sample = "the same mesh"
    o = Oracle.from_mesh(sm, mat, ramp_t0=ramp)
    for g_ in groups:
        o.add_velocity_bc(*g_)
    o.set_dt(0.5 * o.critical_dt())
    o.step(1)  # initial acceleration and first step, untimed
    ncpu = min(16, len(os.sched_getaffinity(0)))
    res = {}
    for nt in sorted({1, ncpu}):
        o.set_threads(nt)
        t0 = time.perf_counter()
        o.step(1)
        one = time.perf_counter() - t0
        n = max(1, min(400, int(12.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        o.step(n)
        el = time.perf_counter() - t0
        res[nt] = (sm.n_tets * n / el, n, el)
        log(f"oracle, {nt} thread(s): {res[nt][0]:.4e} tet-steps/s ({n} steps, {el:.1f} s)")
    v, n, el = res[ncpu]
    v1, n1, el1 = res[1]
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = "unknown"
    return {"value": v, "unit": "tet-steps/s", "cores": ncpu, "kind": "oracle",
            "sample": f"{n} steps of the {sample}, from step 2 (FP64 C++ oracle, "
                      f"{ncpu} threads, {el:.1f} s)",
            "single_thread": {"value": v1, "steps": n1, "seconds": el1},
            "host_cpu_model": model, "host_cpus_visible": os.cpu_count()}


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
                   "launch": f"HIP graphs of {gs} steps; autotuned {tuned['layout']} layout, "
                             f"grid {tuned['grid_cap']}, {tuned['lanes']} lanes per node",
                   "splits_after_run": int(sum(x["n_split"] for x in e))},
        "roofline": {"bound": "hbm", "kernel": "+".join(kernel_names(tuned["layout"])["node"]),
                     "layout": tuned["layout"], "achieved": achieved,
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
# grid.  Each hex has one strain record per edge point (12 x 48 / 24 B) and
# recomputes its gradients from the corner coordinates.  strain = hex nodes 32
# + X gather 32 + u gather 32 + V 8 + write 12 records; edge = CSR offsets 12
# + 12 entries 48 + read the 12 records + write sigma (E/H) + einvV (E/H);
# force = hex nodes 32 + 12 edge ids 48 + 8 list positions 32 + X 32 + V 8 +
# sigma (E/H) + node lists 32 + u, v read+write 96 + 1/m 8.  The nodal terms
# handed from the element pass to the node pass are an intermediate, not
# counted.
HEX_BYTES = {
    "fp64": {"strain": 32 + 32 + 32 + 8 + 12 * 48, "edge_stress": 12 + 48 + 12 * 48 + 144 + 24,
             "node": 32 + 48 + 32 + 32 + 8 + 144 + 32 + 96 + 8},
    "mixed": {"strain": 32 + 32 + 32 + 8 + 12 * 24, "edge_stress": 12 + 48 + 12 * 24 + 72 + 12,
              "node": 32 + 48 + 32 + 32 + 8 + 72 + 32 + 96 + 8},
}


def bench_hex(args):
    """Trilinear hexahedra (ES-H-FEM, factor 1/12): the notched-plate geometry
    at 200 x 80 x 8 hex cells (128,000 hexes, 1 MPa ramped over 1 us), or a
    400 x 200 x 100 block (8,000,000 hexes), each with a notch of precracked
    hexes (mid-planes normal to y through the middle cell row, over the first
    half of the plate or third of the block).  A step: strain, edge stress,
    hex crack pass, element force + node update, crack topology."""
    import torch
    from paper_2508_04076_amd import meshgen as mg
    from paper_2508_04076_amd.cem import Simulation

    mat = dict(mg.BRANCHING_MATERIAL)
    if args.workload == "hex":
        mesh = mg.hex_notched(200, 80, 8, 0.1, 0.04, 0.004, notch_cells=100, traction=1e6)
        desc = ("plate 100x40x4 mm as 200x80x8 trilinear hex cells (128,000 hexes), "
                "1 MPa traction ramped over 1 us, 800 precracked notch hexes")
    else:
        mesh = mg.hex_notched(400, 200, 100, 0.2, 0.1, 0.05, notch_cells=133, traction=1e6)
        desc = ("block 200x100x50 mm as 400x200x100 trilinear hex cells (8,000,000 hexes), "
                "1 MPa traction ramped over 1 us, 13,300 precracked notch hexes")
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
            run = {"ms_per_step": wall * 1e3 / K, "hex_steps_per_s": H * K / wall, "dt_s": dt,
                   "cracks": sim.counts()["splits"]}
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
                   "cracked_hexes_after_run": timed["cracks"],
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
