"""GPU parity of placement under object-object spatial relations and
ratio_on_support (partial annulus, 'middle', face_to, support erosion)
against the FP64 oracle."""
import math

import numpy as np
import pytest

from gpu_util import audit_placements, compare_generation
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


def test_relation_generation_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.relation_scenes(64, seed=7)
    db = scn.DeviceBatch(b)
    assert db.c.geometry == scn.GEOM_YAW
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=11, default_ncand=256))
    status, npl, rec_i, rec_f, placed = _results(db)
    ctx.read_counters()
    ref = orc.generate(b, seed=11, default_ncand=256, early_exit=True)
    n_cmp, n_band = compare_generation(b, ref, status, rec_i, rec_f)
    print(f"compared {n_cmp} of {b.n_objects} objects; {n_band} scenes with a banded decision",
          flush=True)
    assert n_cmp >= 0.9 * b.n_objects
    audit_placements(b, placed, npl)
    # the relations hold on the device's own placements
    for s in range(b.n_scenes):
        o0 = b.obj_off[s]
        for j in range(int(npl[s])):
            o = o0 + j
            r = b.obj_rel[o]
            if r < 0:
                continue
            row = b.rel[r].astype(np.float64)
            anc = rec_f[o0 + row[2:2 + int(row[1])].astype(int), :2].astype(np.float64)
            x, y, yaw = float(rec_f[o, 0]), float(rec_f[o, 1]), float(rec_f[o, 3])
            if row[0] == 1:
                d = math.hypot(x - anc[0, 0], y - anc[0, 1])
                assert row[12] - 1e-5 <= d <= row[13] + 1e-5
            if int(row[15]) & 1:
                assert abs(math.cos(yaw) * (anc[0, 1] - y) - math.sin(yaw) * (anc[0, 0] - x)) < 1e-5


def test_relation_steps_match_one_launch(dev):
    """Object by object (scn_place_step, anchors read back from the records
    of earlier launches) gives the one-launch placements."""
    scn, ctx, torch = dev
    b = sg.relation_scenes(40, seed=8)
    one = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, one, scn.GenArgs(seed=3, default_ncand=256))
    step = scn.DeviceBatch(b)
    scn.reset_scenes(ctx, step)
    for _ in range(8):
        scn.place_step(ctx, step, scn.GenArgs(seed=3, default_ncand=256))
    for u, v in zip(_results(one), _results(step)):
        assert np.array_equal(u, v, equal_nan=True)


def test_eroded_sampling_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = sg.relation_scenes(20, seed=9)
    b.obj_ratio = np.linspace(0.0, 1.0, b.n_objects).astype(np.float32)
    db = scn.DeviceBatch(b)
    obj_idx = (b.obj_off[:-1] + np.arange(b.n_scenes) % 8).astype(np.int32)
    C = 300
    cand_off = (np.arange(b.n_scenes + 1) * C).astype(np.int32)
    got = scn.sample_poses(ctx, db, torch.tensor(obj_idx, device="cuda"),
                           torch.tensor(cand_off, device="cuda"), int(cand_off[-1]), C,
                           seed=12345, attempt=2)
    ref = orc.sample_poses(b, obj_idx, cand_off, 12345, 2)
    for g, r, tol in zip(got, ref, (2e-7, 2e-7, 2e-7, 1e-6)):
        np.testing.assert_allclose(g.cpu().numpy().astype(np.float64), r, atol=tol, rtol=0)


def test_learned_calls_refuse_relations(dev):
    scn, ctx, torch = dev
    b = sg.relation_scenes(4, seed=1)
    db = scn.DeviceBatch(b)
    net = scn.Network()
    net.init(ctx, 1)
    with pytest.raises(scn.ScnError) as e:
        scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=1, default_ncand=256), net)
    assert e.value.code == scn.SCN_E_UNSUPPORTED
