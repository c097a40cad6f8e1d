"""GPU parity: the HIP path through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

from gpu_util import (BAND, CLR_TOL, MARGIN, audit_placements, compare_generation, first_banded,
                      objects_of, rot_xy, tilted)
from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_2512_16896_amd import scn
    torch.cuda.init()
    ctx = scn.Context(0)
    yield scn, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _device_results(db):
    import torch
    torch.cuda.synchronize()
    rec_f, rec_i = db.records()
    return (db.status.cpu().numpy(), db.n_placed.cpu().numpy(), rec_i, rec_f,
            db.placed.cpu().numpy())


def _poses_for(b, obj_idx, cand_off, seed):
    rng = np.random.default_rng(seed)
    tot = int(cand_off[-1])
    hx = float(np.max(b.sup[:, 12])) * 1.1
    hy = float(np.max(b.sup[:, 13])) * 1.1
    return sg.random_poses(rng, tot, hx, hy, z=(0.0, 0.3))


# ---------------------------------------------------------------------------
def test_sample_poses_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    for b, attempt in [(sg.table_scene(), 0), (sg.batched_scenes(40, seed=4), 3)]:
        db = scn.DeviceBatch(b)
        rng = np.random.default_rng(1)
        obj_idx = np.array([b.obj_off[s] + rng.integers(0, b.obj_off[s + 1] - b.obj_off[s])
                            for s in range(b.n_scenes)], np.int32)
        obj_idx[::7] = -1                      # scenes with nothing to sample
        C = rng.integers(0, 700, size=b.n_scenes)   # ragged, includes empty scenes
        cand_off = np.zeros(b.n_scenes + 1, np.int32)
        cand_off[1:] = np.cumsum(np.where(obj_idx >= 0, C, 0))
        tot = int(cand_off[-1])
        x, y, z, yaw = scn.sample_poses(ctx, db, torch.tensor(obj_idx, device="cuda"),
                                        torch.tensor(cand_off, device="cuda"), tot, int(C.max()),
                                        seed=0xDEADBEEF12345, attempt=attempt)
        ref = orc.sample_poses(b, obj_idx, cand_off, 0xDEADBEEF12345, attempt)
        got = [a.cpu().numpy().astype(np.float64) for a in (x, y, z, yaw)]
        for g, r, tol in zip(got, ref, (2e-7, 2e-7, 2e-7, 1e-6)):
            np.testing.assert_allclose(g, r, atol=tol, rtol=0)


def test_check_batch_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.batched_scenes(12, seed=5)
    # a realistic placed table: the oracle's own placements, first 4..20 objects
    gen = orc.generate(b, seed=2)
    rng = np.random.default_rng(2)
    n_placed = np.minimum(gen["n_placed"], rng.integers(0, 20, size=b.n_scenes)).astype(np.int32)
    obj_idx = np.array([b.obj_off[s] + n_placed[s] for s in range(b.n_scenes)], np.int32)
    obj_idx = np.minimum(obj_idx, b.obj_off[1:] - 1)
    C = rng.integers(1, 300, size=b.n_scenes)
    C[3] = 0
    cand_off = np.zeros(b.n_scenes + 1, np.int32)
    cand_off[1:] = np.cumsum(C)
    poses = _poses_for(b, obj_idx, cand_off, 3)
    placed = np.nan_to_num(gen["placed"], nan=0.0).astype(np.float32)
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed))
    db.n_placed.copy_(torch.tensor(n_placed))
    tp = [torch.tensor(p, device="cuda") for p in poses]
    clr, col = scn.check_batch(ctx, db, torch.tensor(obj_idx, device="cuda"),
                               torch.tensor(cand_off, device="cuda"), int(cand_off[-1]),
                               int(C.max()), tp, margin=MARGIN)
    ref = orc.check(b, obj_idx, cand_off, n_placed, placed.astype(np.float64),
                    [p.astype(np.float64) for p in poses])
    clr = clr.cpu().numpy().astype(np.float64)
    col = col.cpu().numpy()
    assert np.max(np.abs(clr - ref)) < CLR_TOL
    clear = np.abs(ref - MARGIN) >= BAND
    assert np.array_equal(col[clear].astype(bool), (ref < MARGIN)[clear])
    assert 0.05 < np.mean(ref < MARGIN) < 0.95      # both outcomes are exercised


def test_check_batch_without_obstacles_is_infinite(dev, orc):
    scn, ctx, torch = dev
    b = sg.uniform_batch(3, 2, 16, 8, 0, 0.5, 0.5, seed=1)
    db = scn.DeviceBatch(b)
    obj_idx = torch.tensor([0, 2, 4], dtype=torch.int32, device="cuda")
    cand_off = torch.tensor([0, 5, 5, 9], dtype=torch.int32, device="cuda")
    poses = [torch.tensor(p, device="cuda") for p in sg.random_poses(np.random.default_rng(0), 9, .5, .5)]
    clr, col = scn.check_batch(ctx, db, obj_idx, cand_off, 9, 5, poses)
    assert torch.isinf(clr).all() and (col == 0).all()


def test_generate_table_scene_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.table_scene(seed=0)
    for seed in range(6):
        ref = orc.generate(b, seed=seed, default_ncand=256)
        db = scn.DeviceBatch(b)
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=seed, default_ncand=256))
        status, npl, rec_i, rec_f, placed = _device_results(db)
        compare_generation(b, ref, status, rec_i, rec_f)
        audit_placements(b, placed, npl)


def test_generate_batched_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.batched_scenes(48, seed=7)
    ref = orc.generate(b, seed=123)
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=123))
    status, npl, rec_i, rec_f, placed = _device_results(db)
    n_cmp, n_band = compare_generation(b, ref, status, rec_i, rec_f)
    assert n_cmp > 0.8 * b.n_objects and n_band <= 4
    assert 0 < np.sum(status == 1) < b.n_scenes       # both valid and invalid scenes
    audit_placements(b, placed, npl)


def test_generate_full_4096_sampled_scenes(dev, orc):
    """The full 4096-scene workload on the device in the benchmark's launch
    configuration; the oracle replays a sample of scenes by their indices."""
    scn, ctx, torch = dev
    b = sg.batched_scenes(4096, seed=0)
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=2024))
    status, npl, rec_i, rec_f, placed = _device_results(db)
    pick = np.random.default_rng(0).choice(4096, size=10, replace=False)
    pick = np.concatenate([pick, [0, 4095]])
    sub, ids = sg.subset(b, pick)
    ref = orc.generate(sub, seed=2024, scene_id=ids)
    objs = objects_of(b, pick)
    compare_generation(sub, ref, status[pick], rec_i[objs], rec_f[objs])
    # every scene: valid scenes placed everything, invalid scenes stopped early
    nobj = b.objects_per_scene()
    assert np.all(npl[status == 1] == nobj[status == 1])
    assert np.all(npl[status == 2] < nobj[status == 2])
    assert np.all(status != 0)
    audit_placements(*_subset_state(b, pick, placed, npl))


def _subset_state(b, pick, placed, npl):
    sub, _ = sg.subset(b, pick)
    sidx = np.concatenate([np.arange(b.sph_off[b.obj_off[s]], b.sph_off[b.obj_off[s + 1]])
                           for s in pick])
    return sub, placed[sidx], npl[pick]


def test_place_step_sequence_equals_generate(dev, orc):
    scn, ctx, torch = dev
    b = sg.batched_scenes(64, seed=9)
    args = scn.GenArgs(seed=77)
    db1 = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db1, args)
    db2 = scn.DeviceBatch(b)
    scn.reset_scenes(ctx, db2)
    chosen_hist = []
    for step in range(21):
        chosen_hist.append(scn.place_step(ctx, db2, args).cpu().numpy())
    a = _device_results(db1)
    c = _device_results(db2)
    for u, v in zip(a[:4], c[:4]):
        assert np.array_equal(u, v, equal_nan=True)
    assert np.all(chosen_hist[-1] == -2)       # nothing left to place
    # step-by-step against the oracle limited to the same number of steps
    db3 = scn.DeviceBatch(b)
    scn.reset_scenes(ctx, db3)
    for step in range(5):
        scn.place_step(ctx, db3, args)
    status, npl, rec_i, rec_f, _ = _device_results(db3)
    ref = orc.generate(b, seed=77, max_steps=5)
    for s in range(b.n_scenes):
        assert npl[s] == ref["n_placed"][s] or ref["rec_banded"][b.obj_off[s]:b.obj_off[s] + 5].any()


@pytest.mark.parametrize("waves", [1, 2, 5, 8, 10, 16])
def test_schedules_give_identical_results(dev, waves):
    scn, ctx, torch = dev
    b = sg.batched_scenes(64, seed=10)
    base = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, base, scn.GenArgs(seed=5))
    other = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, other, scn.GenArgs(seed=5, schedule=waves))
    for u, v in zip(_device_results(base)[:4], _device_results(other)[:4]):
        assert np.array_equal(u, v, equal_nan=True)


def test_many_spheres_per_object_matches_oracle(dev, orc):
    """Objects of 65..256 spheres (two and four spheres per lane)."""
    scn, ctx, torch = dev
    for S in (100, 256):
        b = sg.uniform_batch(6, 6, S, 96, 6, 0.8, 0.5, seed=S)
        ref = orc.generate(b, seed=S, default_ncand=96)
        db = scn.DeviceBatch(b)
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=S, default_ncand=96))
        status, npl, rec_i, rec_f, placed = _device_results(db)
        compare_generation(b, ref, status, rec_i, rec_f)
        audit_placements(b, placed, npl)


def test_uneven_small_batch_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.uneven_batch(6, seed=3, n_obj=(2, 9), n_sph=(16, 200), n_cand=(64, 300))
    ref = orc.generate(b, seed=3)
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=3))
    status, npl, rec_i, rec_f, placed = _device_results(db)
    compare_generation(b, ref, status, rec_i, rec_f)
    audit_placements(b, placed, npl)


def test_infeasible_scene_and_empty_scene(dev):
    scn, ctx, torch = dev
    b = sg.uniform_batch(3, 3, 8, 16, 1, 0.5, 0.5, seed=2)
    # scene 1: one box covering the whole support -> invalid after 11 attempts
    b.box[1, 0:9] = b.sup[1, 0:9]
    b.box[1, 9:12] = b.sup[1, 9:12]
    b.box[1, 12:15] = (3.0, 3.0, 1.0)
    # scene 2: no objects at all -> valid at once
    b2 = sg.subset(b, [0, 1])[0]
    empty = sg.SceneBatch(
        obj_off=np.append(b2.obj_off, b2.obj_off[-1]).astype(np.int32), sph_off=b2.sph_off,
        tmpl=b2.tmpl, obj_sup=b2.obj_sup, obj_ncand=b2.obj_ncand, sup=b2.sup,
        box_off=np.append(b2.box_off, b2.box_off[-1]).astype(np.int32), box=b2.box)
    db = scn.DeviceBatch(empty)
    ctx.reset_counters()
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=1, retries=10, default_ncand=16))
    c = ctx.read_counters()
    status, npl, rec_i, _, _ = _device_results(db)
    assert status.tolist() == [1, 2, 1]
    assert npl.tolist() == [3, 0, 0]
    assert rec_i[3].tolist() == [-1, -1]
    assert c["candidates"] == 3 * 16 + 11 * 16 or c["candidates"] >= 11 * 16
    assert c["attempts"] >= 11 + 3


def test_invalid_arguments_are_rejected_before_launch(dev):
    scn, ctx, torch = dev
    b = sg.table_scene()
    db = scn.DeviceBatch(b)
    with pytest.raises(scn.ScnError) as e:
        scn.generate_scenes(ctx, db, scn.GenArgs(margin=-1.0))
    assert e.value.code == -1
    with pytest.raises(scn.ScnError) as e:
        scn.generate_scenes(ctx, db, scn.GenArgs(retries=-2))
    assert e.value.code == -1
    # a batch whose scenes need more spheres than the planned capacity (which
    # binds when the placed spheres are LDS-resident: 8 waves, LDS budget 0)
    db.c.max_spheres_per_scene = 10
    scn.generate_scenes(ctx, db, scn.GenArgs(schedule=8))
    with pytest.raises(scn.ScnError) as e:
        ctx.read_counters()
    assert e.value.code == -3
    ctx.reset_counters()
    assert ctx.read_counters()["error_word"] == 0


def test_repeated_runs_are_deterministic(dev):
    scn, ctx, torch = dev
    b = sg.batched_scenes(256, seed=11)
    outs = []
    for _ in range(3):
        db = scn.DeviceBatch(b)
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=9))
        outs.append(_device_results(db))
    for o in outs[1:]:
        for u, v in zip(outs[0], o):
            assert np.array_equal(u, v, equal_nan=True)


def test_general_rotations_match_oracle_and_planar_form(dev, orc):
    """Scenes tilted by a world rotation take the general kernel form; they
    match the oracle, and their records equal the planar form's on the
    untilted scenes wherever neither oracle run has a banded decision."""
    scn, ctx, torch = dev
    b = sg.batched_scenes(32, seed=21)
    bt = tilted(b, rot_xy(0.35, -0.2))
    assert scn.geometry_is_yaw(b) and not scn.geometry_is_yaw(bt)
    ref_t = orc.generate(bt, seed=77)
    dt = scn.DeviceBatch(bt)
    assert dt.c.geometry == scn.GEOM_GENERAL
    scn.generate_scenes(ctx, dt, scn.GenArgs(seed=77))
    st_t, npl_t, rec_t, recf_t, placed_t = _device_results(dt)
    n_cmp, _ = compare_generation(bt, ref_t, st_t, rec_t, recf_t)
    assert n_cmp > 0.8 * bt.n_objects
    audit_placements(bt, placed_t, npl_t)
    ref = orc.generate(b, seed=77)
    dy = scn.DeviceBatch(b)
    assert dy.c.geometry == scn.GEOM_YAW
    scn.generate_scenes(ctx, dy, scn.GenArgs(seed=77))
    st, npl, rec, _, _ = _device_results(dy)
    same = 0
    for s in range(b.n_scenes):
        nobj = b.obj_off[s + 1] - b.obj_off[s]
        if first_banded(ref, b, s) < nobj or first_banded(ref_t, bt, s) < nobj:
            continue
        o0 = b.obj_off[s]
        assert st[s] == st_t[s] and npl[s] == npl_t[s], s
        np.testing.assert_array_equal(rec[o0:o0 + nobj], rec_t[o0:o0 + nobj])
        same += 1
    assert same > 0.8 * b.n_scenes


def test_packed_scenes_near_the_margin_match_oracle(dev, orc):
    """Small supports packed with small objects: many chosen placements sit
    within half a millimetre of the collision margin, and every entry before
    each of them was rejected, most by the depth map (probes in the batch
    phase, every sphere for open candidates).  The map only proves hits with
    0.1 mm to spare; a false rejection near the margin would change the
    chosen entry against the oracle.  Planar and general (tilted) forms."""
    scn, ctx, torch = dev
    b = sg.uniform_batch(64, 24, 16, 256, 2, 0.2, 0.15, seed=31, side=(0.03, 0.06),
                         rad=(0.006, 0.02), box_half=(0.02, 0.1))
    for batch in (b, tilted(b, rot_xy(0.35, -0.25))):
        ref = orc.generate(batch, seed=77, default_ncand=256)
        clear = np.asarray(ref["rec_clear"])[np.asarray(ref["rec_idx"]) >= 0]
        assert np.sum(clear < MARGIN + 5e-4) >= 50       # the test reaches the margin
        db = scn.DeviceBatch(batch)
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=77, default_ncand=256))
        status, npl, rec_i, rec_f, placed = _device_results(db)
        n_cmp, n_band = compare_generation(batch, ref, status, rec_i, rec_f)
        assert n_cmp > 0.7 * batch.n_objects
        audit_placements(batch, placed, npl)


def test_false_yaw_declaration_marks_scenes_invalid(dev):
    """A batch that declares SCN_GEOM_YAW but holds tilted supports is not
    placed: its scenes are marked invalid and the error word says why."""
    scn, ctx, torch = dev
    bt = tilted(sg.batched_scenes(8, seed=3), rot_xy(0.3, 0.0))
    db = scn.DeviceBatch(bt)
    db.c.geometry = scn.GEOM_YAW
    ctx.reset_counters()
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=1))
    status, npl, _, _, _ = _device_results(db)
    with pytest.raises(scn.ScnError) as e:
        ctx.read_counters()
    assert e.value.code == -1 and "SCN_GEOM_YAW" in str(e.value)
    ctx.reset_counters()
    assert np.all(status == 2) and np.all(npl == 0)


@pytest.mark.parametrize("sched", [0, 0x24 | (2 << 8)])
def test_generation_graph_replays_match_eager(dev, sched):
    """use_graph: the generation's launches replay from a cached executable
    graph whose arguments are refreshed per call; every replay, with eager
    work and synchronizations between them, equals the eager run."""
    scn, ctx, torch = dev
    b = sg.uneven_batch(48, seed=2) if sched else sg.batched_scenes(64, seed=31)
    db = scn.DeviceBatch(b)
    other = scn.DeviceBatch(sg.table_scene(seed=3))
    for seed in (5, 6, 5, 7):
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=seed, schedule=sched))
        eager = _device_results(db)
        scn.generate_scenes(ctx, other, scn.GenArgs(seed=seed, default_ncand=256))
        torch.cuda.synchronize()
        scn.generate_scenes(ctx, db, scn.GenArgs(seed=seed, schedule=sched, use_graph=1))
        got = _device_results(db)
        for u, v in zip(eager, got):
            np.testing.assert_array_equal(u, v)
