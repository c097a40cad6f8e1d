"""GPU: uneven batches, the LDS-budget launch modes, longest-first order and
the autotuner (all against the oracle or against each other)."""
import os

import numpy as np
import pytest

from gpu_util import audit_placements, compare_generation, objects_of
from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu

LDS_ALL, LDS_32K, LDS_64K, LDS_NONE = 0x000, 0x100, 0x300, 0xF00
LPT = 0x20


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


@pytest.fixture(scope="module")
def mid_uneven():
    # scenes from 5 to 40 objects of 16..256 spheres: both sides of a 32 KB budget
    return sg.uneven_batch(160, seed=21, n_obj=(5, 40), n_sph=(16, 256), n_cand=(64, 512))


@pytest.mark.parametrize("sched", [4 | LDS_ALL, 4 | LDS_32K | LPT, 8 | LDS_64K | LPT, 2 | LDS_NONE,
                                   1 | LDS_NONE | LPT])
def test_launch_modes_give_identical_results(dev, mid_uneven, sched):
    scn, ctx, torch = dev
    b = mid_uneven
    base = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, base, scn.GenArgs(seed=4, schedule=4 | LDS_ALL))
    other = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, other, scn.GenArgs(seed=4, schedule=sched))
    ref = _results(base)
    got = _results(other)
    for u, v in zip(ref, got):
        assert np.array_equal(u, v, equal_nan=True)
    assert np.all(ref[0] != 0)


def test_mid_uneven_matches_oracle_on_sampled_scenes(dev, orc, mid_uneven):
    scn, ctx, torch = dev
    b = mid_uneven
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=8, schedule=4 | LDS_32K | LPT))
    status, npl, rec_i, rec_f, placed = _results(db)
    # the oracle replays the first objects of a sample of scenes (cheap at any size)
    pick = np.random.default_rng(3).choice(b.n_scenes, size=12, replace=False)
    sub, ids = sg.subset(b, pick)
    ref = orc.generate(sub, seed=8, scene_id=ids, max_steps=6)
    objs = objects_of(b, pick)
    # device scenes ran to the end; compare the prefix the oracle placed
    compare_generation(sub, ref, status[pick], rec_i[objs], rec_f[objs], max_steps=6)


def test_autotune_picks_a_schedule_and_round_trips(dev, tmp_path, mid_uneven):
    scn, ctx, torch = dev
    b = mid_uneven
    db = scn.DeviceBatch(b)
    sched, ms = ctx.autotune(db, scn.GenArgs(seed=1))
    assert (sched & 0x1F) in (1, 2, 4, 8, 16) and ms > 0
    # schedule 0 now means the tuned one: same results as asking for it explicitly
    a = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, a, scn.GenArgs(seed=2))
    c = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, c, scn.GenArgs(seed=2, schedule=sched))
    for u, v in zip(_results(a), _results(c)):
        assert np.array_equal(u, v, equal_nan=True)
    path = os.path.join(str(tmp_path), "tune.json")
    ctx.save_tuning(path)
    ctx2 = scn.Context(0)
    ctx2.load_tuning(path)
    ctx2.save_tuning(path + ".2")
    assert open(path).read() == open(path + ".2").read()
    assert '"schedule": %d' % sched in open(path).read()
    ctx2.close()


def _extremes(b, rng, n_random):
    """Scenes that stress the launch: the largest by objects x spheres, ones
    holding 256-sphere objects and 4096-candidate objects, the smallest and
    the largest of the scenes on each side of a 32 KB LDS budget for placed
    spheres (the two halves of a split launch), and random ones."""
    nobj = b.objects_per_scene()
    sph_scene = b.spheres_per_scene()
    S = np.diff(b.sph_off)
    work = nobj * sph_scene
    obj_scene = np.repeat(np.arange(b.n_scenes), nobj)
    pick = list(np.argsort(-work)[:4])
    pick += list(rng.choice(np.unique(obj_scene[S == S.max()]), 4, replace=False))
    pick += list(rng.choice(np.unique(obj_scene[b.obj_ncand == b.obj_ncand.max()]), 4,
                            replace=False))
    small = np.nonzero(16 * sph_scene + 80 * nobj <= 32768)[0]
    large = np.nonzero(16 * sph_scene + 80 * nobj > 32768)[0]
    pick += list(rng.choice(small, 4, replace=False)) + list(rng.choice(large, 4, replace=False))
    rest = np.setdiff1d(np.arange(b.n_scenes), pick)
    pick += list(rng.choice(rest, n_random, replace=False))
    return np.unique(np.asarray(pick, np.int64))


def test_full_uneven_16384_sampled(dev, orc):
    """16384 uneven scenes in the benchmark's tuned launch; the oracle replays
    64+ sampled scenes (extremes included) through all their objects, and
    256 scenes are audited in FP64; properties checked on every scene."""
    scn, ctx, torch = dev
    b = sg.uneven_batch(16384, seed=0)
    db = scn.DeviceBatch(b)
    sched, ms = ctx.autotune(db, scn.GenArgs(seed=1000))
    print(f"tuned schedule 0x{sched:x}: {ms:.1f} ms", flush=True)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=77))
    status, npl, rec_i, rec_f, placed = _results(db)
    nobj = b.objects_per_scene()
    assert np.all(status != 0)
    assert np.all(npl[status == 1] == nobj[status == 1])
    assert np.all(npl[status == 2] < nobj[status == 2])
    rng = np.random.default_rng(5)
    pick = _extremes(b, rng, 44)
    assert len(pick) >= 64
    sub, ids = sg.subset(b, pick)
    print(f"oracle replay of {len(pick)} scenes ({sub.n_objects} objects)", flush=True)
    ref = orc.generate(sub, seed=77, scene_id=ids, early_exit=True)
    objs = objects_of(b, pick)
    n_cmp, n_band = compare_generation(sub, ref, status[pick], rec_i[objs], rec_f[objs])
    print(f"compared {n_cmp} objects, {n_band} scenes with a banded decision", flush=True)
    assert n_cmp >= 0.9 * sub.n_objects
    aud = np.sort(rng.choice(b.n_scenes, 256, replace=False))
    asub, _ = sg.subset(b, aud)
    sidx = np.concatenate([np.arange(b.sph_off[b.obj_off[s]], b.sph_off[b.obj_off[s + 1]]) for s in aud])
    audit_placements(asub, placed[sidx], npl[aud])
