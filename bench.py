"""Benchmark: batched scene generation on one MI355X.

One step = one whole generation pass (sample -> exact check -> first-valid
selection -> commit -> retries) over every scene of the workload, inputs
already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched-4096]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operation counts per unit of work, fixed for reporting:
#   sphere-sphere pair   11  (3 sub + 5 for the squared distance + 2 for the
#                             squared threshold + 1 compare)
#   sphere-box test      26  (yaw boxes)
#   trilinear sample     45
#   sphere transform     10
# The roofline fraction counts the tests the method executes at these units.
# The place kernel's bounding-sphere pretests (box, object and sphere culls)
# are reported beside it, at the same units, as overhead: they decide no
# candidate by themselves.
FLOP_PAIR, FLOP_BOX, FLOP_GRID, FLOP_XFORM = 11, 26, 45, 10
PEAK_FP32_VALU_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 FP32 FLOP/clk (published MI355X figure)

WORKLOADS = {
    "batched-4096": dict(desc="4096 scenes; 2.0x1.0 m support at a random world pose; 20 objects "
                              "x 64 spheres (r~U[0.01,0.05] m, centres in a cube of side "
                              "U[0.05,0.25] m); 1024 candidates per attempt; 16 oriented cuboids "
                              "(half extents U[0.05,0.5] m, random yaw); margin 5 mm; 10 retries",
                         make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                      fromlist=["x"]).batched_scenes(4096, seed=seed),
                         ncand=1024, cpu_scenes=160, learned=True, dense=True, tune=True),
    "table-1": dict(desc="1 scene; 1.2x0.8 m table; 8 objects x 32 spheres; 256 candidates; "
                         "4 cuboids; margin 5 mm; 10 retries",
                    make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                 fromlist=["x"]).table_scene(seed=seed),
                    ncand=256, cpu_scenes=1, tune=True),
    "uneven-16384": dict(desc="16384 uneven scenes in one autotuned persistent launch: objects "
                              "U{5..60}, spheres per object U{16..256}, candidates per attempt "
                              "U{512..4096}, cuboids U{4..32}; support 2.0x1.0 m scaled by "
                              "sqrt(N/20); margin 5 mm; 10 retries",
                         make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                      fromlist=["x"]).uneven_batch(16384, seed=seed),
                         ncand=1024, cpu_scenes=24, tune=True, graph=True),
    "shelves-65536": dict(desc="65536 scenes x 6 stacked 0.8x0.4 m shelves; 100 objects x 128 "
                               "spheres (r~U[0.005,0.02] m, centres in a cube of side "
                               "U[0.03,0.08] m), round-robin over the shelves; furniture as "
                               "64^3 signed-distance grids (one shared asset, 6 instances per "
                               "scene), trilinear; 2048 candidates per attempt; margin 5 mm; "
                               "10 retries; autotuned launch",
                          make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                       fromlist=["x"]).shelf_scenes(65536, seed=seed),
                          ncand=2048, cpu_scenes=0, tune=True),
    "relations-4096": dict(desc="4096 scenes on a 2.0x1.0 m support with 4 cuboids; 8 objects x 32 "
                                "spheres with object-object relations: within 0.45 m of object 0 "
                                "inside a pi/4 cone (face_to), beyond 0.5 m, 0.35+-0.03 m from "
                                "object 1 in a pi/2 cone, in the middle of objects 0-2, within "
                                "0.3 m of that one (face_to); ratio_on_support 1 / 0.5 on the "
                                "free objects; 256 candidates per attempt; margin 5 mm; 10 retries",
                           make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                        fromlist=["x"]).relation_scenes(4096, seed=seed),
                           ncand=256, cpu_scenes=0, tune=True),
    "reach-4096": dict(desc="4096 robot tables (1.2x0.8 m, 4 cuboids, robot base 0.15 m off the "
                            "near edge); 8 objects x 32 spheres that must be reachable on a "
                            "24x9x64x64 base-symmetric 4-D map (6 from above, 2 at 45 deg); 256 "
                            "candidates per attempt; margin 5 mm; 10 retries",
                       make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                    fromlist=["x"]).reach_scenes(4096, seed=seed),
                       ncand=256, cpu_scenes=0, tune=True),
    "stable-4096": dict(desc="4096 tables (1.6x1.0 m, 6 cuboids); 12 objects x 32 spheres, of "
                             "every three one turning about z only, one resting on a face of its "
                             "bounding box (6 stable poses weighted by face area), one in one of "
                             "12 rotations uniform on SO(3); 256 candidates per attempt; margin "
                             "5 mm; 10 retries",
                        make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                     fromlist=["x"]).stable_scenes(4096, seed=seed),
                        ncand=256, cpu_scenes=0, tune=True),
    "uneven-shelves-65536": dict(desc="learned proposal + uneven batching on dense multi-support "
                                      "scenes: 65536 shelf units (6 stacked 0.8x0.4 m shelves, "
                                      "64^3 SDF grids, trilinear); objects U{40..100} per scene "
                                      "(round-robin over the shelves), spheres U{64..128} per object "
                                      "(r~U[0.005,0.02] m), candidates U{1024..2048} per attempt; "
                                      "margin 5 mm; 10 retries; plain autotuned, learned top-64 "
                                      "ticks; network trained on labels harvested from plain runs "
                                      "on 3 x 64 other scenes",
                                 make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                              fromlist=["x"]).uneven_shelf_scenes(
                                     65536, seed=seed),
                                 ncand=2048, cpu_scenes=0, tune=True),
    "drawers-4096": dict(desc="4096 two-drawer cabinets at random world poses; drawers are "
                              "prismatic joints with travel U[0, 0.35] m drawn per scene by the "
                              "batched forward kinematics, which moves their walls (boxes) and "
                              "bottoms (supports); 4 objects x 32 spheres per drawer (cube side "
                              "U[0.04,0.12] m, r~U[0.01,0.03] m); 256 candidates per attempt; "
                              "6 static cabinet boards; margin 5 mm; 10 retries",
                         make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                      fromlist=["x"]).drawer_scenes(4096, seed=seed),
                         ncand=256, cpu_scenes=0, tune=True),
}


def recorded_traffic(key: str, path: str = None):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE runs kept in
    profiles/traffic.json -- only while the kernel's sources are the ones those
    counters were taken on (else None)."""
    import hashlib
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[key]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def dense_equivalent(b, db, ncand, retries=10):
    """Dense-equivalent work of a generation: the FLOP a dense check of
    every candidate a first-valid scan must decide would compute (entries up
    to and including the accepted one; all (R+1) C entries of an object that
    fails), at 11 per sphere pair, 26 per sphere-box test, 10 per sphere
    transform -- for the last generation in `db` (plain records)."""
    _, rec = db.records()
    n_placed = db.n_placed.cpu().numpy()
    status = db.status.cpu().numpy()
    obj_off = np.asarray(b.obj_off, np.int64)
    sph_off = np.asarray(b.sph_off, np.int64)
    nbox = np.diff(np.asarray(b.box_off, np.int64))
    C = np.asarray(b.obj_ncand, np.int64) if b.obj_ncand is not None else None
    flop = 0
    for s in range(b.n_scenes):
        o0 = obj_off[s]
        last = min(int(n_placed[s]) + (1 if status[s] == 2 else 0), int(obj_off[s + 1] - o0))
        for j in range(last):
            o = o0 + j
            c = int(C[o]) if C is not None else ncand
            a, i = int(rec[o, 0]), int(rec[o, 1])
            decided = a * c + i + 1 if i >= 0 else (retries + 1) * c
            S = int(sph_off[o + 1] - sph_off[o])
            P = int(sph_off[o] - sph_off[o0])
            flop += decided * S * (11 * P + 26 * int(nbox[s]) + 10)
    return flop


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def learned_leg(ctx, db, b, W, args, stream, plain_rate):
    """The learned-proposal form on the same scenes: harvest labels from plain
    runs on three other seeds of the workload, train the network on the device
    (untimed), then time generation with top-64 proposals and the uniform
    fallback exactly like the plain leg."""
    import torch
    from paper_2512_16896_amd import learned as L
    from paper_2512_16896_amd import scn
    t0 = time.perf_counter()
    parts = []
    for k in range(3):
        tb = W["make"](100 + k)
        tdb = scn.DeviceBatch(tb, "cuda:0")
        scn.generate_scenes(ctx, tdb, scn.GenArgs(seed=500 + k, default_ncand=W["ncand"]))
        parts.append(L.harvest(ctx, tdb, seed=900 + k, labels_per_state=64))
        del tdb
    data = L.merge(parts)
    del parts
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = scn.Network()
    net.init(ctx, 1)
    t0 = time.perf_counter()
    log = L.train(ctx, net, data, steps=6000, batch=256, lr=1e-3, log_every=3000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_labels = int(data.bins.numel())
    del data
    gen = lambda step: scn.generate_scenes_learned(
        ctx, db, scn.GenArgs(seed=1000 + step, default_ncand=W["ncand"]), net, top_k=64)
    for i in range(max(args.warmup, 1)):
        gen(-1 - i)
    torch.cuda.synchronize()
    ctx.reset_counters()
    steps = args.steps
    t0 = time.perf_counter()
    for k in range(steps):
        gen(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = ctx.read_counters()
    _, rec = db.records()
    prop = rec[:, 0] == -2
    placed = rec[:, 1] >= 0
    rate = cnt["valid_scenes"] / wall
    return {"value": rate, "unit": "valid scenes/s", "ms_per_step": 1e3 * wall / steps,
            "valid_fraction": cnt["valid_scenes"] / (b.n_scenes * steps),
            "candidate_checks_per_s": cnt["candidates"] / wall,
            "vs_plain": rate / plain_rate,
            "placed_by_proposal": float(prop.sum() / max(placed.sum(), 1)),
            "rank0_accepted": float((prop & (rec[:, 1] == 0)).sum() / max(placed.sum(), 1)),
            "training": {"labels": n_labels, "harvest_s": t_harvest, "steps": 6000, "batch": 256,
                         "train_s": t_train, "loss_first": log[0][1], "loss_last": log[-1][1]}}


def dense_leg(ctx, db, b, default_ncand, stream, seed=77, reps=3):
    """scn_check_batch in distance mode over a whole generation's states: for
    every object position j, all candidates of object j of every scene (its
    per-object candidate count) against the scene's boxes and its first
    min(j, placed) objects (the placement of the last plain run in `db`).
    Times the check launches only, with HIP events on the launch stream."""
    import torch
    from paper_2512_16896_amd import scn
    n = b.n_scenes
    final = db.n_placed.clone()
    fin = final.cpu().numpy().astype(np.int64)
    obj_off = np.asarray(b.obj_off, np.int64)
    sph_off = np.asarray(b.sph_off, np.int64)
    ncand = (np.asarray(b.obj_ncand, np.int64) if b.obj_ncand is not None
             else np.full(b.n_objects, default_ncand, np.int64))
    nobj = obj_off[1:] - obj_off[:-1]
    nbox = np.diff(np.asarray(b.box_off, np.int64))
    dev = torch.device("cuda", 0)
    pairs = boxes = xf = cands = 0
    launches = []
    for j in range(int(nobj.max())):
        live = nobj > j
        o = np.where(live, obj_off[:-1] + j, -1)
        C = np.where(live, ncand[np.maximum(o, 0)], 0)
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(C)
        total, cmax = int(off[-1]), int(C.max())
        oi = torch.as_tensor(o.astype(np.int32), device=dev)
        cand_off = torch.as_tensor(off.astype(np.int32), device=dev)
        npl = torch.as_tensor(np.minimum(fin, j).astype(np.int32), device=dev)
        poses = scn.sample_poses(ctx, db, oi, cand_off, total, cmax, seed, 0)
        launches.append((oi, cand_off, total, cmax, npl, poses))
        S = (sph_off[o + 1] - sph_off[o])[live]
        P = (sph_off[obj_off[:-1] + np.minimum(j, fin)] - sph_off[obj_off[:-1]])[live]
        pairs += int(np.sum(C[live] * S * P))
        boxes += int(np.sum(C[live] * S * nbox[live]))
        xf += int(np.sum(C[live] * S))
        cands += total
    ms = []
    torch.cuda.synchronize()
    ctx.reset_counters()
    for rep in range(reps):
        tot = 0.0
        for oi, cand_off, total, cmax, npl, poses in launches:
            db.n_placed.copy_(npl)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            scn.check_batch(ctx, db, oi, cand_off, total, cmax, poses)
            e1.record(stream)
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        ms.append(tot)
    cnt = ctx.read_counters()
    db.n_placed.copy_(final)
    t = min(ms) * 1e-3
    flop = FLOP_PAIR * pairs + FLOP_BOX * boxes + FLOP_XFORM * xf
    return {"candidate_checks_per_s": cands / t, "pairs_per_s": pairs / t,
            "ms_per_pass": 1e3 * t, "launches": len(launches), "candidates": cands,
            "refined_fraction": cnt["check_refined"] / (reps * max(cands, 1)),
            "roofline": {"bound": "alu", "achieved": flop / t / 1e12,
                         "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                         "frac": flop / t / 1e12 / PEAK_FP32_VALU_TFLOPS,
                         "traffic": recorded_traffic(f"k_check dense {b.name}"),
                         "kernel": "k_check (dense, distance mode)",
                         "kernel_ms_per_launch": 1e3 * t / len(launches)}}


def plain_leg(ctx, b, W, steps, warmup, schedule=0):
    """Time `steps` whole plain generations of batch b (inputs resident in HBM
    before the timed region), after `warmup` untimed ones.  Returns the result
    fields, the device batch and the schedule that ran."""
    import torch
    from paper_2512_16896_amd import scn
    db = scn.DeviceBatch(b, "cuda:0")
    stream = torch.cuda.current_stream()
    graph = 1 if W.get("graph") else 0
    gen = lambda step: scn.generate_scenes(
        ctx, db, scn.GenArgs(seed=1000 + step, default_ncand=W["ncand"], schedule=schedule,
                             use_graph=graph))
    tuned = None
    if W.get("tune") and schedule == 0:
        progress(f"autotuning {b.name or ''}")
        tuned = ctx.autotune(db, scn.GenArgs(seed=999, default_ncand=W["ncand"]))
    sched_run = tuned[0] if tuned else (schedule or scn.DEFAULT_SCHEDULE)
    for i in range(warmup):
        gen(-1 - i)
    torch.cuda.synchronize()
    ctx.reset_counters()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        gen(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = ctx.read_counters()     # the place kernel counts the scenes it finished
    launch_ms = float(np.mean([a.elapsed_time(z) for a, z in ev]))
    per = {k: v / steps for k, v in cnt.items() if k != "error_word"}
    # executed method tests at the fixed units, per launch
    flop = (FLOP_PAIR * per["sphere_pairs"] + FLOP_BOX * per["box_pairs"] +
            FLOP_GRID * per["grid_samples"] + FLOP_XFORM * per["transforms"])
    pre = FLOP_BOX * per["box_culls"] + FLOP_PAIR * (per["object_culls"] + per["sphere_culls"])
    achieved = flop / (launch_ms * 1e-3) / 1e12
    n = b.n_scenes
    out = {
        "value": cnt["valid_scenes"] / wall, "unit": "valid scenes/s",
        "ms_per_step": 1e3 * wall / steps,
        "launch": "hipGraph replay" if graph else "direct",
        "schedule": (f"autotuned 0x{tuned[0]:x}" if tuned else
                     (f"0x{schedule:x}" if schedule else f"default 0x{scn.DEFAULT_SCHEDULE:x}")),
        "valid_fraction": cnt["valid_scenes"] / (n * steps),
        "candidate_checks_per_s": cnt["candidates"] / wall,
        "counters_per_step": per,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU_TFLOPS,
                     "traffic": recorded_traffic(f"k_place {b.name} 0x{sched_run:x}"),
                     "kernel": "k_place (fused place kernel)", "kernel_ms": launch_ms,
                     "flop_per_launch": flop,
                     "units": "executed tests: 11/pair, 26/sphere-box, 45/trilinear, "
                              "10/transform"},
        "pretests": {"flop_per_launch": pre,
                     "tflops": pre / (launch_ms * 1e-3) / 1e12,
                     "frac_if_counted": (flop + pre) / (launch_ms * 1e-3) / 1e12
                     / PEAK_FP32_VALU_TFLOPS,
                     "note": "bounding-sphere box/object/sphere pretests (overhead, not in frac)"},
    }
    return out, db, stream


def host_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(b, W, n_all=64, n_one=2, warm=2, runs=5):
    """The FP64 oracle as it stands, on the host cores: the first n_all scenes
    with every core, the first n_one with one thread; median of `runs` timed
    runs after `warm` untimed ones."""
    import oracle
    from paper_2512_16896_amd import scenegen as sg
    oracle.build(force=False)
    threads = oracle.max_threads()

    def timed(k, nthreads):
        sub, ids = sg.subset(b, np.arange(min(k, b.n_scenes)))
        oracle.set_threads(nthreads)
        ts, last = [], None
        for r in range(warm + runs):
            t = time.perf_counter()
            last = oracle.generate(sub, seed=1000, default_ncand=W["ncand"], scene_id=ids)
            if r >= warm:
                ts.append(time.perf_counter() - t)
        med = float(np.median(ts))
        v = int(np.sum(last["status"] == 1))
        return {"valid_scenes_per_s": v / med, "scenes_per_s": sub.n_scenes / med,
                "candidate_checks_per_s": float(np.sum(last["n_cand"])) / med,
                "median_s": med, "scenes": sub.n_scenes, "valid": v, "threads": nthreads}

    allc = timed(n_all, threads)
    one = timed(n_one, 1)
    oracle.set_threads(threads)
    return {"value": allc["valid_scenes_per_s"], "unit": "valid scenes/s", "cores": threads,
            "kind": "oracle",
            "sample": f"scenes 0..{allc['scenes'] - 1} of the same workload, seed 1000, median of "
                      f"{runs} runs after {warm} warm-ups ({allc['median_s']:.2f} s, "
                      f"{allc['valid']} valid); one thread: scenes 0..{one['scenes'] - 1}",
            "host_cpu": host_model(), "all_cores": allc, "one_thread": one}


def extra_workload(ctx, name, steps, warmup, dense_scenes=0):
    """Another workload's plain generation (and optionally the dense check on
    a sample of its scenes), reported as an extra key of the same line."""
    import torch
    from paper_2512_16896_amd import scenegen as sg
    W = WORKLOADS[name]
    progress(f"building {name}")
    b = W["make"](0)
    b.name = name
    progress(f"timing {name}")
    out, db, stream = plain_leg(ctx, b, W, steps, warmup)
    out["config"] = W["desc"]
    if name == "table-1":
        ms = out["roofline"]["kernel_ms"]
        out["us_per_scene"] = 1e3 * ms
        out["us_per_object"] = 1e3 * ms / b.n_objects
    del db
    torch.cuda.empty_cache()
    if dense_scenes:
        progress(f"dense check on {dense_scenes} scenes of {name}")
        rng = np.random.default_rng(5)
        pick = np.sort(rng.choice(b.n_scenes, dense_scenes, replace=False))
        sub, _ = sg.subset(b, pick)
        sub.name = name
        del b
        from paper_2512_16896_amd import scn
        sdb = scn.DeviceBatch(sub, "cuda:0")
        scn.generate_scenes(ctx, sdb, scn.GenArgs(seed=1000, default_ncand=W["ncand"]))
        d = dense_leg(ctx, sdb, sub, W["ncand"], stream, reps=2)
        d["sample"] = f"{dense_scenes} random scenes (rng seed 5) of the {name} batch"
        out["dense_check"] = d
        del sdb
        torch.cuda.empty_cache()
    return out


def drawers_leg(ctx, steps, warmup):
    """Articulated scenes: the batched forward kinematics (joint values, links,
    moved rows; timed alone with HIP events) and then the plain generation on
    the moved drawers."""
    import torch
    from paper_2512_16896_amd import scn
    W = WORKLOADS["drawers-4096"]
    progress("building drawers-4096")
    b = W["make"](0)
    b.name = "drawers-4096"
    db = scn.DeviceBatch(b, "cuda:0")
    J = scn.Joints(b.params["art"])
    stream = torch.cuda.current_stream()
    for i in range(3):
        scn.forward_kinematics(ctx, J, db, seed=50 + i)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(20)]
    for k in range(20):
        ev[k][0].record(stream)
        scn.forward_kinematics(ctx, J, db, seed=60 + k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ctx.read_counters()
    fk_ms = float(np.mean([a.elapsed_time(z) for a, z in ev]))
    nj = int(J.joint.shape[0])
    rows = int(J.box_link.numel() + J.sup_link.numel())
    db.refresh_geometry()
    b.box = db.box.cpu().numpy()[:b.n_boxes]
    b.sup = db.sup.cpu().numpy()
    del db
    out, db, _ = plain_leg(ctx, b, W, steps, warmup)
    out["config"] = W["desc"]
    out["forward_kinematics"] = {"us_per_call": 1e3 * fk_ms, "joints": nj, "rows": rows,
                                 "joints_per_s": nj / (fk_ms * 1e-3),
                                 "note": "joint values, link poses and moved box/support rows "
                                         "of all 4096 scenes per call (three launches)"}
    del db
    torch.cuda.empty_cache()
    return out


def reach_query_leg(ctx, n=1 << 22):
    """scn_reach_query alone: n queries (random robot bases, object poses and
    approach angles) against the synthetic map; queries per second."""
    import torch
    from paper_2512_16896_amd import scn, scenegen as sg
    m, g = sg.reach_map()
    rng = np.random.default_rng(1)
    robot = np.zeros((n, 12), np.float32)
    robot[:, 0] = robot[:, 4] = robot[:, 8] = 1.0
    pose = np.zeros((n, 12), np.float32)
    yaw = rng.uniform(0, 2 * np.pi, n)
    pose[:, 0], pose[:, 1], pose[:, 3], pose[:, 4], pose[:, 8] = \
        np.cos(yaw), -np.sin(yaw), np.sin(yaw), np.cos(yaw), 1.0
    pose[:, 9:] = rng.uniform(-1, 1, (n, 3))
    dev = torch.device("cuda", 0)
    dm = torch.tensor(m.ravel(), device=dev)
    tr, tp = torch.tensor(robot, device=dev), torch.tensor(pose, device=dev)
    th = torch.tensor(rng.uniform(0, 1.5, n).astype(np.float32), device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        scn.reach_query(ctx, dm, g, tr, tp, th)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        scn.reach_query(ctx, dm, g, tr, tp, th)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    return {"queries": n, "us_per_call": 1e3 * ms, "queries_per_s": n / (ms * 1e-3),
            "bytes_per_query": 12 * 4 * 2 + 4 + 1,
            "hbm_gbs": n * (12 * 4 * 2 + 4 + 1) / (ms * 1e-3) / 1e9}


def shelves_learned_leg(ctx, steps=3, warmup=1):
    """The dense multi-support configuration with the learned proposal and
    uneven batching combined: the plain leg (autotuned), then labels from
    plain runs on 3 x 64 other scenes, 2000 training steps, and the learned
    generation of the same batch (same metric and counters)."""
    import torch
    from paper_2512_16896_amd import learned as L
    from paper_2512_16896_amd import scenegen as sg
    from paper_2512_16896_amd import scn
    name = "uneven-shelves-65536"
    W = WORKLOADS[name]
    progress(f"building {name}")
    b = W["make"](0)
    b.name = name
    progress(f"timing {name} (plain)")
    out, db, stream = plain_leg(ctx, b, W, steps, warmup)
    out["config"] = W["desc"]
    progress(f"{name}: harvest and training")
    t0 = time.perf_counter()
    parts = []
    for k in range(3):
        tb = sg.uneven_shelf_scenes(64, seed=100 + k, chunk=64)
        tdb = scn.DeviceBatch(tb, "cuda:0")
        scn.generate_scenes(ctx, tdb, scn.GenArgs(seed=500 + k, default_ncand=W["ncand"]))
        parts.append(L.harvest(ctx, tdb, seed=900 + k, labels_per_state=16))
        del tdb
    data = L.merge(parts)
    del parts
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = scn.Network()
    net.init(ctx, 1)
    t0 = time.perf_counter()
    log = L.train(ctx, net, data, steps=2000, batch=256, lr=1e-3, log_every=1000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    n_labels = int(data.bins.numel())
    del data
    gen = lambda step: scn.generate_scenes_learned(
        ctx, db, scn.GenArgs(seed=1000 + step, default_ncand=W["ncand"]), net, top_k=64)
    progress(f"timing {name} (learned)")
    for i in range(warmup):
        gen(-1 - i)
    torch.cuda.synchronize()
    ctx.reset_counters()
    t0 = time.perf_counter()
    for k in range(steps):
        gen(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    cnt = ctx.read_counters()
    _, rec = db.records()
    prop = rec[:, 0] == -2
    placed = rec[:, 1] >= 0
    rate = cnt["valid_scenes"] / wall
    out["learned"] = {
        "value": rate, "unit": "valid scenes/s", "ms_per_step": 1e3 * wall / steps,
        "valid_fraction": cnt["valid_scenes"] / (b.n_scenes * steps),
        "candidate_checks_per_s": cnt["candidates"] / wall, "vs_plain": rate / out["value"],
        "placed_by_proposal": float(prop.sum() / max(placed.sum(), 1)),
        "rank0_accepted": float((prop & (rec[:, 1] == 0)).sum() / max(placed.sum(), 1)),
        "training": {"labels": n_labels, "harvest_s": t_harvest, "steps": 2000, "batch": 256,
                     "train_s": t_train, "loss_first": log[0][1], "loss_last": log[-1][1]}}
    del db
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched-4096", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", type=lambda v: int(v, 0), default=0)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and timing the learned-proposal form")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads' lines (table-1, uneven-16384, shelves-65536)")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-check legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(scenes would shard across GPUs with no exchange; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_16896_amd import scn

    W = WORKLOADS[args.workload]
    progress(f"building {args.workload}")
    b = W["make"](args.seed)
    b.name = args.workload
    progress("uploading and timing")
    torch.cuda.set_device(0)
    ctx = scn.Context(0)
    leg, db, stream = plain_leg(ctx, b, W, args.steps, args.warmup, args.schedule)
    n = b.n_scenes
    out = {
        "metric": "valid scenes/sec + candidate-pose checks/sec (plain vs learned proposal)",
        "value": leg["value"], "unit": "valid scenes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W['desc']}", "scenes": n,
                   "objects": int(b.n_objects), "method": "plain (uniform candidates)"},
    }
    out.update({k: v for k, v in leg.items() if k not in ("value", "unit", "ms_per_step")})
    dq = dense_equivalent(b, db, W["ncand"])
    kms = leg["roofline"]["kernel_ms"]
    out["dense_equivalent"] = {
        "flop_per_step": dq, "tflops": dq / (kms * 1e-3) / 1e12,
        "x_fp32_peak": dq / (kms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS,
        "note": "dense FLOP of the candidates a first-valid scan decides (last step), over the "
                "place kernel's time; culling makes it exceed the peak"}
    if W.get("dense") and not args.no_dense:
        progress("dense check")
        out["dense_check"] = dense_leg(ctx, db, b, W["ncand"], stream)
    if W.get("learned") and not args.no_learned:
        progress("learned form: harvest, training, timing")
        out["learned"] = learned_leg(ctx, db, b, W, args, stream, leg["value"])
    if not args.no_cpu_baseline and W["cpu_scenes"] > 0:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(b, W)
    del db
    torch.cuda.empty_cache()
    if args.workload == "batched-4096" and not args.no_extra:
        out["table_1"] = extra_workload(ctx, "table-1", 200, 20)
        out["uneven_16384"] = extra_workload(ctx, "uneven-16384", 10, 2,
                                             dense_scenes=0 if args.no_dense else 512)
        out["shelves_65536"] = extra_workload(ctx, "shelves-65536", 5, 1)
        out["uneven_shelves_65536"] = shelves_learned_leg(ctx)
        out["drawers_4096"] = drawers_leg(ctx, 20, 3)
        out["relations_4096"] = extra_workload(ctx, "relations-4096", 20, 3)
        out["stable_4096"] = extra_workload(ctx, "stable-4096", 20, 3)
        out["reach_4096"] = extra_workload(ctx, "reach-4096", 20, 3)
        out["reach_4096"]["reach_query"] = reach_query_leg(ctx)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
