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

# Algorithmic FP32 operation counts per unit of work (flag-mode tests):
#   sphere-sphere pair : 3 sub + 5 (squared distance) + 2 (threshold) + 1 cmp = 11
#   sphere-box pair    : 3 sub + 15 (box-frame rotation) + 3 (|q|-h) + 3 (max 0)
#                        + 5 (squared norm) + 1 cmp = 30
#   sphere transform   : 4 + 4 + 1 (yaw + position) + 18 (support pose) = 27
#   box pretest        : the sphere-box test applied to the bounding sphere = 30
#   object pretest     : bounding sphere vs bounding sphere, like a pair = 11
FLOP_PAIR, FLOP_BOX, FLOP_XFORM, FLOP_BOXCULL, FLOP_OBJCULL = 11, 30, 27, 30, 11
# Distance mode (scn_check_batch with clearances): the pair is 3 sub + 5 (squared
# distance) + 1 sqrt + 1 sub + 1 min = 11; the box adds the signed part of the
# SDF to the flag form: 30 + 1 sqrt + 3 (max of the excess, min 0, add) + 1 sub
# + 1 min - 1 cmp = 35.
FLOP_PAIR_DIST, FLOP_BOX_DIST = 11, 35
PEAK_FP32_VALU_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 FP32 FLOP/clk (published MI355X figure)

WORKLOADS = {
    "batched-4096": dict(desc="4096 scenes; 2.0x1.0 m support at a random world pose; 20 objects "
                              "x 64 spheres (r~U[0.01,0.05] m, centres in a cube of side "
                              "U[0.05,0.25] m); 1024 candidates per attempt; 16 oriented cuboids "
                              "(half extents U[0.05,0.5] m, random yaw); margin 5 mm; 10 retries",
                         make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                      fromlist=["x"]).batched_scenes(4096, seed=seed),
                         ncand=1024, cpu_scenes=160, learned=True, dense=True),
    "table-1": dict(desc="1 scene; 1.2x0.8 m table; 8 objects x 32 spheres; 256 candidates; "
                         "4 cuboids; margin 5 mm; 10 retries",
                    make=lambda seed: __import__("paper_2512_16896_amd.scenegen",
                                                 fromlist=["x"]).table_scene(seed=seed),
                    ncand=256, cpu_scenes=1),
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
}


def recorded_traffic(key: str):
    """HBM bytes per launch from the rocprofv3 FETCH_SIZE/WRITE_SIZE runs kept in
    profiles/traffic.json -- only while the kernel's sources are the ones those
    counters were taken on (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[key]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def dense_equivalent(b, db, ncand, retries=10):
    """Survey definition of the generation roofline: the FLOP a dense check of
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


def dense_leg(ctx, db, b, W, stream, seed=77):
    """scn_check_batch in distance mode over a whole generation's states: for
    every object position j, all candidates of object j of every scene against
    the scene's boxes and its first min(j, placed) objects (the placement of the
    last plain run).  Times the check launches only."""
    import torch
    from paper_2512_16896_amd import scn
    n, C = b.n_scenes, W["ncand"]
    final = db.n_placed.clone()
    fin = final.cpu().numpy().astype(np.int64)
    obj_off = np.asarray(b.obj_off, np.int64)
    sph_off = np.asarray(b.sph_off, np.int64)
    nobj = obj_off[1:] - obj_off[:-1]
    nbox = np.diff(np.asarray(b.box_off, np.int64))
    cand_off = torch.arange(0, (n + 1) * C, C, dtype=torch.int32, device="cuda:0")
    dnobj = torch.as_tensor(nobj, dtype=torch.int32, device="cuda:0")
    doff = db.obj_off[:-1]
    pairs = boxes = xf = 0
    launches = []
    for j in range(int(nobj.max())):
        oi = torch.where(dnobj > j, doff + j, torch.full_like(dnobj, -1)).to(torch.int32)
        npl = torch.minimum(final, torch.full_like(final, j))
        poses = scn.sample_poses(ctx, db, oi, cand_off, n * C, C, seed, 0)
        launches.append((oi, npl, poses))
        live = nobj > j
        o = obj_off[:-1][live] + j
        S = sph_off[o + 1] - sph_off[o]
        P = sph_off[obj_off[:-1][live] + np.minimum(j, fin[live])] - sph_off[obj_off[:-1][live]]
        pairs += int(np.sum(C * S * P))
        boxes += int(np.sum(C * S * nbox[live]))
        xf += int(np.sum(C * S))
    ms = []
    for rep in range(3):
        tot = 0.0
        for oi, npl, poses in launches:
            db.n_placed.copy_(npl)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            scn.check_batch(ctx, db, oi, cand_off, n * C, C, poses)
            e1.record(stream)
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        ms.append(tot)
    db.n_placed.copy_(final)
    t = min(ms) * 1e-3
    flop = FLOP_PAIR_DIST * pairs + FLOP_BOX_DIST * boxes + FLOP_XFORM * xf
    return {"candidate_checks_per_s": n * C * len(launches) / t, "pairs_per_s": pairs / t,
            "ms_per_pass": 1e3 * t, "launches": len(launches),
            "roofline": {"bound": "alu", "achieved": flop / t / 1e12,
                         "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                         "frac": flop / t / 1e12 / PEAK_FP32_VALU_TFLOPS,
                         "traffic": recorded_traffic(f"k_check dense {b.name}"),
                         "kernel": "k_check (dense, distance mode)"}}


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
    progress("uploading")
    torch.cuda.set_device(0)
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b, "cuda:0")
    stream = torch.cuda.current_stream()
    graph = 1 if W.get("graph") else 0
    gen = lambda step: scn.generate_scenes(
        ctx, db, scn.GenArgs(seed=1000 + step, default_ncand=W["ncand"], schedule=args.schedule,
                             use_graph=graph))

    tuned = None
    if W.get("tune") and args.schedule == 0:
        progress("autotuning")
        tuned = ctx.autotune(db, scn.GenArgs(seed=999, default_ncand=W["ncand"]))
    # the schedule the timed launches run
    sched_run = tuned[0] if tuned else (args.schedule or scn.DEFAULT_SCHEDULE)
    progress("timing")
    for i in range(args.warmup):
        gen(-1 - i)
    torch.cuda.synchronize()
    ctx.reset_counters()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        gen(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cnt = ctx.read_counters()     # the place kernel counts the scenes it finished
    valid = cnt["valid_scenes"]
    wall = t1 - t0
    launch_ms = float(np.mean([a.elapsed_time(z) for a, z in ev]))
    steps = args.steps
    flop_per_launch = (FLOP_PAIR * cnt["sphere_pairs"] + FLOP_BOX * cnt["box_pairs"] +
                       FLOP_XFORM * cnt["transforms"] + FLOP_BOXCULL * cnt["box_culls"] +
                       FLOP_OBJCULL * (cnt["object_culls"] + cnt["sphere_culls"])) / steps
    achieved_tflops = flop_per_launch / (launch_ms * 1e-3) / 1e12
    n = b.n_scenes
    out = {
        "metric": "valid scenes/sec + candidate-pose checks/sec (plain vs learned proposal)",
        "value": valid / wall,
        "unit": "valid scenes/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {W['desc']}", "scenes": n,
                   "objects": int(b.n_objects), "method": "plain (uniform candidates)"},
        "launch": "hipGraph replay" if graph else "direct",
        "schedule": (f"autotuned 0x{tuned[0]:x}" if tuned else
                     (f"0x{args.schedule:x}" if args.schedule
                      else f"default 0x{scn.DEFAULT_SCHEDULE:x}")),
        "valid_fraction": valid / (n * steps),
        "candidate_checks_per_s": cnt["candidates"] / wall,
        "counters_per_step": {k: v / steps for k, v in cnt.items() if k != "error_word"},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP32_VALU_TFLOPS,
                     "traffic": recorded_traffic(f"k_place {args.workload} 0x{sched_run:x}"),
                     "kernel": "k_place (fused place kernel)",
                     "kernel_ms": launch_ms},
    }
    dq = dense_equivalent(b, db, W["ncand"])
    out["dense_equivalent"] = {
        "flop_per_step": dq, "tflops": dq / (launch_ms * 1e-3) / 1e12,
        "x_fp32_peak": dq / (launch_ms * 1e-3) / 1e12 / PEAK_FP32_VALU_TFLOPS,
        "note": "dense FLOP of the candidates a first-valid scan decides (last step), over the "
                "place kernel's time; culling makes it exceed the peak"}
    if W.get("dense"):
        progress("dense check")
        out["dense_check"] = dense_leg(ctx, db, b, W, stream)
    if W.get("learned") and not args.no_learned:
        progress("learned form: harvest, training, timing")
        out["learned"] = learned_leg(ctx, db, b, W, args, stream, valid / wall)
    if not args.no_cpu_baseline and W["cpu_scenes"] > 0:
        progress("cpu baseline")
        import oracle
        from paper_2512_16896_amd import scenegen as sg
        k = min(W["cpu_scenes"], n)
        pick = np.arange(k)
        sub, ids = sg.subset(b, pick)
        oracle.build(force=False)
        threads = oracle.max_threads()
        tc = time.perf_counter()
        ref = oracle.generate(sub, seed=1000, default_ncand=W["ncand"], scene_id=ids)
        tc = time.perf_counter() - tc
        v = int(np.sum(ref["status"] == 1))
        out["cpu_baseline"] = {"value": v / tc, "unit": "valid scenes/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"scenes 0..{k - 1} of the same workload, seed 1000, "
                                         f"{tc:.1f} s, {v} valid"}
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
