"""GPU: the boundary's error behaviour through the C ABI -- non-finite input
is a collision, counted and reported as SCN_E_NONFINITE (against the FP64
oracle's reading of the same input); a workspace too small is refused before
any launch; the learned calls refuse batches outside what they compute;
scenes with more grid instances than the place kernel's masks cover."""
import ctypes

import numpy as np
import pytest

from gpu_util import BAND, CLR_TOL, MARGIN, compare_generation
from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_2512_16896_amd import scn
    torch.cuda.init()
    yield scn, torch
    torch.cuda.synchronize()


def _raw_counters(scn, ctx):
    c = scn.Counters()
    rc = scn.lib().scn_read_counters(ctx.h, ctypes.byref(c), scn._stream())
    return rc, c.as_dict()


def _results(db):
    import torch
    torch.cuda.synchronize()
    rec_f, rec_i = db.records()
    return db.status.cpu().numpy(), db.n_placed.cpu().numpy(), rec_i, rec_f


def test_nonfinite_template_and_box_fail_their_objects(dev, orc):
    scn, torch = dev
    b = sg.batched_scenes(8, seed=1)
    o_bad = int(b.obj_off[2]) + 1                     # scene 2, its second object
    b.tmpl[int(b.sph_off[o_bad]) + 5, 3] = np.nan
    b.box[int(b.box_off[4]) + 3, 10] = np.inf         # scene 4: one box centre
    o_sup = int(b.obj_off[6]) + 3                     # scene 6: a template coordinate
    b.tmpl[int(b.sph_off[o_sup]), 0] = -np.inf
    ref = orc.generate(b, seed=5)
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b)
    ctx.reset_counters()
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=5))
    status, npl, rec_i, rec_f = _results(db)
    compare_generation(b, ref, status, rec_i, rec_f)
    np.testing.assert_array_equal(npl, ref["n_placed"])
    assert status[4] == 2 and npl[4] == 0
    assert npl[2] <= 1 and npl[6] <= 3
    rc, cnt = _raw_counters(scn, ctx)
    assert rc == scn.SCN_E_NONFINITE
    want = 1 + int(ref["n_placed"][2] == 1) + int(ref["n_placed"][6] == 3)
    assert cnt["nonfinite"] == want
    # a clean batch reports nothing afterwards
    ctx.reset_counters()
    db2 = scn.DeviceBatch(sg.batched_scenes(8, seed=1))
    scn.generate_scenes(ctx, db2, scn.GenArgs(seed=5))
    rc, cnt = _raw_counters(scn, ctx)
    assert rc == 0 and cnt["nonfinite"] == 0
    ctx.close()


def test_nonfinite_placed_sphere_in_step_mode(dev, orc):
    """Three objects placed step by step; then a NaN written into a placed
    sphere of scene 1: its next object collides everywhere (the oracle,
    given the same state, agrees), the other scenes go on."""
    scn, torch = dev
    b = sg.batched_scenes(5, seed=3)
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b)
    scn.reset_scenes(ctx, db)
    for _ in range(3):
        scn.place_step(ctx, db, scn.GenArgs(seed=8))
    torch.cuda.synchronize()
    npl0 = db.n_placed.cpu().numpy().copy()
    sb = int(np.nonzero(npl0 == 3)[0][0])            # a scene with its three objects placed
    k = int(b.sph_off[int(b.obj_off[sb]) + 1]) + 2
    db.placed[k, 1] = float("nan")
    ctx.reset_counters()
    chosen = scn.place_step(ctx, db, scn.GenArgs(seed=8)).cpu().numpy()
    status, npl, rec_i, _ = _results(db)
    assert status[sb] == 2 and npl[sb] == 3 and chosen[sb] == -1
    placed = db.placed.cpu().numpy().astype(np.float64)
    o = int(b.obj_off[sb]) + 3
    obj_idx = [o if s == sb else -1 for s in range(5)]
    cand_off = [0] + [16 if s >= sb else 0 for s in range(5)]
    poses = orc.sample_poses(b, obj_idx, cand_off, 8, 0)
    clr = orc.check(b, obj_idx, cand_off, npl0, placed, poses)
    assert len(clr) == 16 and np.all(np.isnan(clr))
    for s in range(5):
        if s != sb and npl0[s] == 3:
            assert chosen[s] >= 0 or status[s] == 2
    rc, cnt = _raw_counters(scn, ctx)
    assert rc == scn.SCN_E_NONFINITE and cnt["nonfinite"] == 1
    ctx.close()


def test_nonfinite_check_batch_matches_oracle(dev, orc):
    """Dense check: NaN clearances (and collide = 1) exactly where the oracle
    has them -- a NaN pose, a NaN placed sphere of one scene, an infinite box
    half extent of another -- and the other clearances within tolerance."""
    scn, torch = dev
    b = sg.batched_scenes(6, seed=9)
    gen = orc.generate(b, seed=4)
    n_placed = np.minimum(gen["n_placed"], 6).astype(np.int32)
    placed = np.nan_to_num(gen["placed"], nan=0.0).astype(np.float32)
    placed[int(b.sph_off[int(b.obj_off[2])]) + 7, 0] = np.nan     # scene 2 (object 0 is placed)
    b.box[int(b.box_off[3]), 12] = np.inf                         # scene 3
    obj_idx = np.array([b.obj_off[s] + n_placed[s] for s in range(6)], np.int32)
    C = np.full(6, 40)
    cand_off = np.zeros(7, np.int32)
    cand_off[1:] = np.cumsum(C)
    poses = sg.random_poses(np.random.default_rng(3), 240, 1.1, 0.55)
    poses[1][5] = np.nan
    poses[3][77] = np.inf
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed))
    db.n_placed.copy_(torch.tensor(n_placed))
    ctx.reset_counters()
    clr, col = scn.check_batch(ctx, db, torch.tensor(obj_idx, device="cuda"),
                               torch.tensor(cand_off, device="cuda"), 240, 40,
                               [torch.tensor(p, device="cuda") for p in poses], margin=MARGIN)
    ref = orc.check(b, obj_idx, cand_off, n_placed, placed.astype(np.float64),
                    [p.astype(np.float64) for p in poses])
    clr = clr.cpu().numpy().astype(np.float64)
    col = col.cpu().numpy()
    bad = np.isnan(ref)
    assert bad.sum() == 2 + 40 + 40
    np.testing.assert_array_equal(np.isnan(clr), bad)
    assert np.all(col[bad] == 1)
    assert np.max(np.abs(clr[~bad] - ref[~bad])) < CLR_TOL
    clear = ~bad & (np.abs(ref - MARGIN) >= BAND)
    np.testing.assert_array_equal(col[clear].astype(bool), (ref < MARGIN)[clear])
    rc, cnt = _raw_counters(scn, ctx)
    assert rc == scn.SCN_E_NONFINITE and cnt["nonfinite"] == int(bad.sum())
    ctx.close()


def test_nonfinite_grid_node_collides_where_sampled(dev, orc):
    """A NaN node on the lower board's top of the shared bay asset: the
    samples that read it collide on both sides; the generation agrees with
    the oracle and the call reports SCN_E_NONFINITE."""
    scn, torch = dev
    b = sg.shelf_scenes(6, seed=2, n_obj=18, n_sph=16, n_cand=64)
    vals = b.grid_vals[0].copy()
    # the node layer just above the board top (z = 0 in the bay frame), which
    # the samples of spheres resting on the board read
    o = np.asarray(sg.BAY_GRID_ORIGIN)
    i, j, k = [int(round((c - o[a]) / sg.BAY_GRID_H)) for a, c in enumerate((0.0, 0.0, 0.01))]
    assert o[2] + k * sg.BAY_GRID_H > 0.0
    vals[k, j - 3:j + 4, i - 6:i + 7] = np.nan
    b.grid_vals = [vals]
    ref = orc.generate(b, seed=12, default_ncand=64)
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b)
    ctx.reset_counters()
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=12, default_ncand=64))
    status, npl, rec_i, rec_f = _results(db)
    compare_generation(b, ref, status, rec_i, rec_f)
    rc, _ = _raw_counters(scn, ctx)
    assert rc == scn.SCN_E_NONFINITE
    ctx.close()


def test_workspace_too_small_is_refused_before_any_launch(dev):
    scn, torch = dev
    ctx = scn.Context(0)
    net = scn.Network(train=False)
    net.init(ctx, 3)
    x = torch.zeros((64, scn.FEATURES), dtype=torch.bfloat16, device="cuda")
    logits = torch.full((64, scn.BINS), 7.0, device="cuda")
    need = scn.workspace_bytes(scn.WS_MLP_FORWARD, net=net, rows=64)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(small)
    rc = scn.lib().scn_mlp_forward(ctx.h, ctypes.byref(net.c), ctypes.c_void_p(x.data_ptr()), 64,
                                   ctypes.c_void_p(logits.data_ptr()), scn._stream())
    assert rc == scn.SCN_E_INVALID_ARG
    assert b"workspace" in scn.lib().scn_last_error()
    torch.cuda.synchronize()
    assert bool((logits == 7.0).all())                 # nothing was launched
    # a longest-first schedule needs the order workspace; none attached
    b = sg.batched_scenes(4, seed=0)
    db = scn.DeviceBatch(b)
    ctx.set_workspace(None)
    db.status.fill_(3)
    a = scn.GenArgs(seed=1, schedule=0xF04 | scn.SCHED_LONGEST_FIRST).c()
    rc = scn.lib().scn_generate_scenes(ctx.h, ctypes.byref(db.c), ctypes.byref(a), scn._stream())
    assert rc == scn.SCN_E_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((db.status[:4] == 3).all())
    # with exactly the bytes asked for, both run
    ctx.set_workspace(torch.empty(need, dtype=torch.uint8, device="cuda"))
    assert scn.lib().scn_mlp_forward(ctx.h, ctypes.byref(net.c), ctypes.c_void_p(x.data_ptr()),
                                     64, ctypes.c_void_p(logits.data_ptr()), scn._stream()) == 0
    ctx.set_workspace(torch.empty(scn.workspace_bytes(scn.WS_GENERATE, db), dtype=torch.uint8,
                                  device="cuda"))
    assert scn.lib().scn_generate_scenes(ctx.h, ctypes.byref(db.c), ctypes.byref(a),
                                         scn._stream()) == 0
    torch.cuda.synchronize()
    assert bool((db.status[:4] != 3).all())
    ctx.close()


def test_learned_generation_reports_a_support_shared_by_two_scenes(dev):
    """The learned path keeps one height map per support: a support that
    objects of two scenes rest on is reported by the next counter read."""
    scn, torch = dev
    ctx = scn.Context(0)
    net = scn.Network(train=False)
    net.init(ctx, 1)
    b = sg.batched_scenes(3, seed=0)
    b.obj_sup = b.obj_sup.copy()
    b.obj_sup[b.obj_off[1]] = 0                      # scene 1's first object on scene 0's support
    db = scn.DeviceBatch(b)
    ctx.reset_counters()
    scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=1, max_steps=2), net, top_k=8)
    with pytest.raises(scn.ScnError) as e:
        ctx.read_counters()
    assert e.value.code == scn.SCN_E_INVALID_ARG
    ctx.reset_counters()
    ctx.close()


def test_more_than_64_grid_instances(dev, orc):
    """70 stacked bays per scene: objects on the bays past the 64th are
    tested against their own bay's grid by the place kernel's tail loop;
    the generation matches the oracle, which tests every grid."""
    scn, torch = dev
    b = sg.shelf_scenes(2, seed=4, n_obj=140, n_sph=16, n_cand=48, n_shelves=70)
    ref = orc.generate(b, seed=21, default_ncand=48)
    ctx = scn.Context(0)
    db = scn.DeviceBatch(b)
    assert db.c.max_grids_per_scene == 70
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=21, default_ncand=48))
    status, npl, rec_i, rec_f = _results(db)
    n_cmp, _ = compare_generation(b, ref, status, rec_i, rec_f)
    assert n_cmp >= 2 * 70           # objects on the bays past the 64th were compared
    ctx.close()
