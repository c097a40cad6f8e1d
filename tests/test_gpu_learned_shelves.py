"""GPU parity of the learned proposal on dense multi-support scenes with
voxel furniture and uneven counts (stacked shelves): per-support height maps
and feature rows, labels harvested against the shelf grids, and learned
generation with a separated and with a random network, all against the FP64
oracle, with an FP64 audit of the placements."""
import numpy as np
import pytest

from gpu_util import audit_placements
from oracle import learned as ol
from paper_2512_16896_amd import scenegen as sg
from test_gpu_learned import _net, _separated_net, _weights

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    from paper_2512_16896_amd import scn
    ctx = scn.Context(0)
    yield scn, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _batch(n_scenes, seed):
    return sg.uneven_shelf_scenes(n_scenes, seed=seed, n_obj=(8, 18), n_sph=(16, 32),
                                  n_cand=(64, 160), chunk=4)


def _state(orc, b, seed):
    """A state of every scene: a random prefix of an oracle placement."""
    gen = orc.generate(b, seed=seed, early_exit=True)
    rng = np.random.default_rng(seed)
    nobj = np.diff(b.obj_off)
    n_state = np.minimum(gen["n_placed"], rng.integers(0, nobj + 1)).astype(np.int32)
    placed = np.nan_to_num(gen["placed"], nan=0.0).astype(np.float32)
    return n_state, placed


def test_per_support_heightmaps_and_features_match_oracle(dev, orc):
    scn, ctx, torch = dev
    b = _batch(6, 2)
    n_state, placed = _state(orc, b, 4)
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed))
    H = scn.heightmaps(ctx, db, torch.tensor(n_state, device="cuda")).cpu().numpy()
    assert H.shape[0] == b.sup.shape[0]
    n_raised = 0
    for s in range(b.n_scenes):
        for u in np.unique(b.obj_sup[b.obj_off[s]:b.obj_off[s + 1]]):
            ref = ol.heightmap(b, placed.astype(np.float64), s, int(n_state[s]), u=int(u))
            bad = np.abs(H[u] - ref.reshape(-1)) > 1e-5
            assert np.mean(bad) < 2e-3, (s, u, np.sum(bad))
            n_raised += ref.max() > 0
    assert n_raised >= 6
    desc = scn.descriptors(ctx, db)
    nobj = np.diff(b.obj_off)
    obj_idx = np.where(n_state < nobj, b.obj_off[:-1] + n_state, -1).astype(np.int32)
    X = scn.features(ctx, db, torch.tensor(H, device="cuda"), desc,
                     torch.tensor(obj_idx, device="cuda")).float().cpu().numpy()
    for s in range(b.n_scenes):
        o = obj_idx[s]
        if o < 0:
            assert np.all(X[s] == 0)
            continue
        ref = ol.heightmap(b, placed.astype(np.float64), s, int(n_state[s]))
        rx = ol.features(ref, ol.descriptor(b.tmpl[b.sph_off[o]:b.sph_off[o + 1]]))
        close = np.abs(X[s] - rx) <= 2 ** -7 * np.maximum(np.abs(rx), 1e-30)
        assert np.mean(~close) < 5e-3


def test_harvest_with_grids_matches_oracle(dev, orc):
    scn, ctx, torch = dev
    b = _batch(8, 3)
    n_state, placed = _state(orc, b, 6)
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed))
    L, seed, rnd = 48, 0x5151, 2
    bins, acc = scn.harvest_labels(ctx, db, torch.tensor(n_state, device="cuda"), L, seed, rnd)
    bins, acc = bins.cpu().numpy(), acc.cpu().numpy()
    n_cmp = n_acc = 0
    for s in range(b.n_scenes):
        sub, ids = sg.subset(b, [s])
        first = b.sph_off[b.obj_off[s]]
        own = placed[first:b.sph_off[b.obj_off[s + 1]]].astype(np.float64)

        def check(o, poses, s=s, sub=sub, ids=ids, own=own):
            j = o - b.obj_off[s]
            return orc.check(sub, [j], [0, len(poses[0])], [int(n_state[s])], own, poses,
                             scene_id=ids)

        want_bins, want_acc = ol.harvest_labels(b, placed.astype(np.float64), s, int(n_state[s]),
                                                L, seed, rnd, 0.005, check)
        np.testing.assert_array_equal(bins[s], want_bins)
        if want_bins[0] < 0:
            continue
        # labels whose clearance is within the band of the margin may differ
        o = b.obj_off[s] + int(n_state[s])
        tm = b.tmpl[b.sph_off[o]:b.sph_off[o + 1]].astype(np.float64)
        same = acc[s] == want_acc
        n_cmp += same.sum()
        n_acc += want_acc.sum()
        assert np.mean(same) > 0.97, s
    assert n_cmp > 200 and 0 < n_acc < n_cmp


@pytest.mark.parametrize("kind", ["separated", "random"])
def test_learned_generation_on_uneven_shelves_matches_oracle(dev, orc, kind):
    scn, ctx, torch = dev
    b = _batch(8, 5)
    W, bb = _separated_net(27, b) if kind == "separated" else _weights(29)
    net = _net(scn, torch, W, bb)
    db = scn.DeviceBatch(b)
    scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=41), net, top_k=64)
    torch.cuda.synchronize()
    ctx.read_counters()
    rec_f, rec_i = db.records()
    ref = ol.generate_learned(b, [w.astype(np.float64) for w in W],
                              [v.astype(np.float64) for v in bb], 41, 64, orc,
                              rank_tol=0.02 if kind == "separated" else None)
    n_cmp = n_prop = 0
    for s in range(b.n_scenes):
        for o in range(b.obj_off[s], b.obj_off[s + 1]):
            if ref["unsure"][o]:
                if tuple(rec_i[o]) != tuple(ref["rec"][o]) or ref["rec"][o][1] < 0:
                    break
                continue
            assert tuple(rec_i[o]) == tuple(ref["rec"][o]), (s, o - b.obj_off[s])
            if ref["rec"][o][1] >= 0:
                np.testing.assert_allclose(rec_f[o], ref["pose"][o], atol=2e-6, rtol=0)
                n_prop += ref["rec"][o][0] == -2
            n_cmp += 1
            if ref["rec"][o][1] < 0:
                break
    print(f"{kind}: compared {n_cmp} of {b.n_objects} objects, {n_prop} proposal picks",
          flush=True)
    assert n_prop > 0
    assert n_cmp >= (0.5 * b.n_objects if kind == "separated" else 20)
    audit_placements(b, db.placed.cpu().numpy(), db.n_placed.cpu().numpy())


def test_learned_generation_full_size_sampled(dev, orc):
    """uneven-shelves-65536 at full size, in the benchmark's launch
    configuration (learned ticks with the default launch shapes, every
    object's own candidate count): the placements of two sampled units, the
    fullest one and one drawn at random, are replayed by the oracle one by
    one (with their scene indices) and compared wherever it is sure."""
    scn, ctx, torch = dev
    b = sg.uneven_shelf_scenes(65536, seed=0)
    W, bb = _separated_net(27, sg.subset(b, list(range(16)))[0])
    net = _net(scn, torch, W, bb)
    db = scn.DeviceBatch(b)
    scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=43, default_ncand=2048), net, top_k=64)
    torch.cuda.synchronize()
    ctx.read_counters()
    rec_f, rec_i = db.records()
    nobj = np.diff(b.obj_off)
    rng = np.random.default_rng(8)
    pick = sorted({int(np.argmax(nobj)), int(rng.integers(b.n_scenes))})
    sub, ids = sg.subset(b, pick)
    ref = ol.generate_learned(sub, [w.astype(np.float64) for w in W],
                              [v.astype(np.float64) for v in bb], 43, 64, orc, rank_tol=0.02,
                              scene_id=ids)
    n_cmp = n_prop = 0
    for k, s in enumerate(pick):
        for j in range(int(nobj[s])):
            o, r = int(b.obj_off[s]) + j, int(sub.obj_off[k]) + j
            if ref["unsure"][r]:
                if tuple(rec_i[o]) != tuple(ref["rec"][r]) or ref["rec"][r][1] < 0:
                    break
                continue
            assert tuple(rec_i[o]) == tuple(ref["rec"][r]), (s, j)
            if ref["rec"][r][1] >= 0:
                np.testing.assert_allclose(rec_f[o], ref["pose"][r], atol=2e-6, rtol=0)
                n_prop += ref["rec"][r][0] == -2
            n_cmp += 1
            if ref["rec"][r][1] < 0:
                break
    print(f"full size: compared {n_cmp} of {int(nobj[pick].sum())} objects of units {pick}, "
          f"{n_prop} proposal picks", flush=True)
    assert n_prop > 0 and n_cmp >= 0.5 * int(nobj[pick].sum())
