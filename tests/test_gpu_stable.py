"""GPU parity of stable-pose orientations (Sec. III "Main algorithm": an
object's orientation from its stable poses, then the turn about z) against
the FP64 oracle: the sampler's rows and poses, generation in the planar and
general forms, with spatial relations in the same batch, and the calls that
refuse them."""
import numpy as np
import pytest

from gpu_util import audit_placements, compare_generation, rot_xy, tilted
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


def _run(scn, ctx, torch, b, seed, ncand=256):
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=seed, default_ncand=ncand))
    torch.cuda.synchronize()
    ctx.read_counters()
    rec_f, rec_i = db.records()
    return (db, db.status.cpu().numpy(), db.n_placed.cpu().numpy(), rec_i, rec_f,
            db.placed.cpu().numpy(), db.rec_stable.cpu().numpy())


def test_sampled_rows_and_poses_match_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.stable_scenes(24, seed=3)
    db = scn.DeviceBatch(b)
    obj_idx = (b.obj_off[:-1] + np.arange(b.n_scenes) % 12).astype(np.int32)
    C = 500
    cand_off = (np.arange(b.n_scenes + 1) * C).astype(np.int32)
    got = scn.sample_poses(ctx, db, torch.tensor(obj_idx, device="cuda"),
                           torch.tensor(cand_off, device="cuda"), int(cand_off[-1]), C,
                           seed=4242, attempt=3, with_stable=True)
    ref = orc.sample_poses(b, obj_idx, cand_off, 4242, 3, with_stable=True)
    np.testing.assert_array_equal(got[4].cpu().numpy(), ref[4])       # rows: bit-exact
    assert np.any(ref[4] >= 0) and np.any(ref[4] < 0)
    for g, r, tol in zip(got[:4], ref[:4], (2e-7, 2e-7, 1e-6, 1e-6)):
        np.testing.assert_allclose(g.cpu().numpy().astype(np.float64), r, atol=tol, rtol=0)


@pytest.mark.parametrize("form", ["planar", "general"])
def test_stable_generation_matches_oracle(dev, orc, form):
    scn, ctx, torch = dev
    b = sg.stable_scenes(64, seed=5)
    if form == "general":
        b = tilted(b, rot_xy(0.3, -0.2))
    db, status, npl, rec_i, rec_f, placed, rows = _run(scn, ctx, torch, b, 13)
    assert db.c.geometry == (scn.GEOM_YAW if form == "planar" else scn.GEOM_GENERAL)
    ref = orc.generate(b, seed=13, default_ncand=256, early_exit=True)
    n_cmp, n_band = compare_generation(b, ref, status, rec_i, rec_f)
    print(f"{form}: compared {n_cmp} of {b.n_objects}; {n_band} scenes banded", flush=True)
    assert n_cmp >= 0.9 * b.n_objects
    # the same stable rows and (up to FP32) the same world spheres wherever
    # the decisions were compared
    n_rows = 0
    for s in range(b.n_scenes):
        for j in range(int(ref["n_placed"][s])):
            o = b.obj_off[s] + j
            if ref["rec_banded"][b.obj_off[s]:o + 1].any():
                break
            assert rows[o] == ref["rec_stable"][o]
            n_rows += rows[o] >= 0
            a0, a1 = b.sph_off[o], b.sph_off[o + 1]
            np.testing.assert_allclose(placed[a0:a1], ref["placed"][a0:a1], atol=1e-5, rtol=0)
    assert n_rows > 100
    audit_placements(b, placed, npl)


def test_relations_with_stable_poses_match_oracle(dev, orc):
    """Spatial relations and stable poses in one batch."""
    scn, ctx, torch = dev
    b = sg.relation_scenes(48, seed=31)
    rng = np.random.default_rng(2)
    tables = []
    for o in range(b.n_objects):
        tables.append(None if o % 2 == 0 else
                      sg.stable_rows(sg.haar_rotations(rng, 5), rng.uniform(0.2, 1.0, 5)))
    cnt = [0 if t is None else len(t) for t in tables]
    b.obj_pose_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    b.stable = np.concatenate([t for t in tables if t is not None]).astype(np.float32)
    db, status, npl, rec_i, rec_f, placed, rows = _run(scn, ctx, torch, b, 17)
    ref = orc.generate(b, seed=17, default_ncand=256, early_exit=True)
    n_cmp, _ = compare_generation(b, ref, status, rec_i, rec_f)
    assert n_cmp >= 0.85 * b.n_objects
    audit_placements(b, placed, npl)


def test_calls_that_refuse_stable_poses(dev):
    scn, ctx, torch = dev
    b = sg.stable_scenes(4, seed=1)
    db = scn.DeviceBatch(b)
    net = scn.Network()
    net.init(ctx, 1)
    with pytest.raises(scn.ScnError) as e:
        scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=1, default_ncand=256), net)
    assert e.value.code == scn.SCN_E_UNSUPPORTED
    one = torch.zeros(1, device="cuda")
    k = torch.zeros(1, dtype=torch.int32, device="cuda")
    oi = torch.tensor(b.obj_off[:-1], dtype=torch.int32, device="cuda")
    co = torch.tensor(np.r_[0, np.ones(b.n_scenes, np.int32)].cumsum(), dtype=torch.int32,
                      device="cuda")
    with pytest.raises(scn.ScnError) as e:
        scn.check_batch(ctx, db, oi, co, 1, 1, [one, one, one, one, k])
    assert e.value.code == scn.SCN_E_UNSUPPORTED
