"""GPU: dense multi-shelf scenes with voxel-SDF furniture (trilinear grids)
against the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import CLR_TOL, BAND, MARGIN, audit_placements, compare_generation, objects_of
from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_2512_16896_amd import scn
    ctx = scn.Context(0)
    yield scn, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _results(db):
    import torch
    torch.cuda.synchronize()
    rec_f, rec_i = db.records()
    return db.status.cpu().numpy(), db.n_placed.cpu().numpy(), rec_i, rec_f, db.placed.cpu().numpy()


def _audit_grids(b, placed, npl, margin=MARGIN, tol=CLR_TOL):
    """Every placed sphere keeps the margin from the furniture field too."""
    import oracle
    for s in range(b.n_scenes):
        o0 = b.obj_off[s]
        for j in range(int(npl[s])):
            o = o0 + j
            for q in placed[b.sph_off[o]:b.sph_off[o + 1]].astype(np.float64):
                for g in range(b.grid_off[s], b.grid_off[s + 1]):
                    G = b.grid[g].astype(np.float64)
                    pg = G[:9].reshape(3, 3) @ q[:3] + G[9:12]
                    v = oracle.grid_sample(b.grid_vals[b.grid_src[g]], G[12:15], G[15], pg)
                    assert v - q[3] >= margin - tol


def test_small_shelves_match_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.shelf_scenes(12, seed=3)
    ref = orc.generate(b, seed=5)
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=5))
    status, npl, rec_i, rec_f, placed = _results(db)
    n_cmp, n_band = compare_generation(b, ref, status, rec_i, rec_f)
    assert n_cmp > 0.9 * b.n_objects
    c = ctx.read_counters()
    assert c["grid_samples"] > 0
    audit_placements(sg.subset(b, [0, 1])[0], placed[:2 * 100 * 128], npl[:2])
    _audit_grids(sg.subset(b, [0])[0], placed[:100 * 128], npl[:1])


def test_check_batch_with_grids_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.shelf_scenes(6, seed=4)
    gen = orc.generate(b, seed=1)
    rng = np.random.default_rng(1)
    n_placed = np.minimum(gen["n_placed"], rng.integers(0, 100, size=b.n_scenes)).astype(np.int32)
    obj_idx = (b.obj_off[:-1] + np.minimum(n_placed, 99)).astype(np.int32)
    C = rng.integers(50, 200, size=b.n_scenes)
    cand_off = np.zeros(b.n_scenes + 1, np.int32)
    cand_off[1:] = np.cumsum(C)
    poses = sg.random_poses(rng, int(cand_off[-1]), 0.42, 0.22, z=(0.0, 0.2))
    placed = np.nan_to_num(gen["placed"], nan=0.0).astype(np.float32)
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed))
    db.n_placed.copy_(torch.tensor(n_placed))
    clr, col = scn.check_batch(ctx, db, torch.tensor(obj_idx, device="cuda"),
                               torch.tensor(cand_off, device="cuda"), int(cand_off[-1]), int(C.max()),
                               [torch.tensor(p, device="cuda") for p in poses])
    ref = orc.check(b, obj_idx, cand_off, n_placed, placed.astype(np.float64),
                    [p.astype(np.float64) for p in poses])
    clr = clr.cpu().numpy().astype(np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(clr), fin)
    assert np.max(np.abs(clr[fin] - ref[fin])) < CLR_TOL
    clear = np.abs(ref - MARGIN) >= BAND
    assert np.array_equal(col.cpu().numpy()[clear].astype(bool), (ref < MARGIN)[clear])


@pytest.mark.parametrize("sched", [0x008, 0x028 | 0xF00, 0x110])
def test_shelf_launch_modes_identical(dev, sched):
    scn, ctx, torch = dev
    b = sg.shelf_scenes(40, seed=6)
    a = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, a, scn.GenArgs(seed=9, schedule=0x004 | 0xF00))
    c = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, c, scn.GenArgs(seed=9, schedule=sched))
    for u, v in zip(_results(a), _results(c)):
        assert np.array_equal(u, v, equal_nan=True)


def test_full_shelves_65536_sampled(dev, orc):
    """65536 scenes x 6 shelves x 100 objects x 128 spheres with voxel-SDF
    bays: the tuned launch on the device; 16 sampled scenes replayed by the
    oracle through all 100 objects, 256 scenes audited in FP64 (boxes, grids,
    placed spheres); properties checked on all scenes."""
    scn, ctx, torch = dev
    print("generating 65536 shelf scenes", flush=True)
    b = sg.shelf_scenes(65536, seed=0)
    print("uploading", flush=True)
    db = scn.DeviceBatch(b)
    print("tuning", flush=True)
    sched, ms = ctx.autotune(db, scn.GenArgs(seed=1000))
    print(f"tuned 0x{sched:x}: {ms:.1f} ms", flush=True)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=321))
    status, npl, rec_i, rec_f, placed = _results(db)
    assert np.all(status != 0)
    assert np.all(npl[status == 1] == 100)
    rng = np.random.default_rng(2)
    pick = np.sort(rng.choice(b.n_scenes, size=16, replace=False))
    sub, ids = sg.subset(b, pick)
    print("oracle replay of 16 scenes", flush=True)
    ref = orc.generate(sub, seed=321, scene_id=ids, early_exit=True)
    objs = objects_of(b, pick)
    n_cmp, n_band = compare_generation(sub, ref, status[pick], rec_i[objs], rec_f[objs])
    print(f"compared {n_cmp} objects, {n_band} scenes with a banded decision", flush=True)
    assert n_cmp >= 0.9 * sub.n_objects
    aud = np.sort(rng.choice(b.n_scenes, 256, replace=False))
    asub, _ = sg.subset(b, aud)
    sidx = np.concatenate([np.arange(b.sph_off[b.obj_off[s]], b.sph_off[b.obj_off[s + 1]]) for s in aud])
    audit_placements(asub, placed[sidx], npl[aud])
