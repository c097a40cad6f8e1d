"""GPU parity of the dense checker (scn_check_batch, distance mode) against the
FP64 oracle on the shapes its matrix-core tiling has to get right: object
sizes that are not multiples of 16 spheres (padded rows) and above 64 (several
passes over the placed spheres), placed tables of every length modulo 32
(padded columns, the second tile of a step past the end), no placed spheres,
and pairs at zero or tiny distance (where an expanded squared distance
|p|^2 - 2 p.q + |q|^2 cancels)."""
import numpy as np
import pytest

from gpu_util import BAND, CLR_TOL, MARGIN
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


def _check_both(scn, ctx, torch, orc, b, obj_idx, n_placed, placed, cand_off, poses):
    db = scn.DeviceBatch(b)
    db.placed.copy_(torch.tensor(placed.astype(np.float32)))
    db.n_placed.copy_(torch.tensor(n_placed.astype(np.int32)))
    C = np.diff(cand_off)
    tp = [torch.tensor(np.asarray(p, np.float32), device="cuda") for p in poses]
    clr, col = scn.check_batch(ctx, db, torch.tensor(obj_idx.astype(np.int32), device="cuda"),
                               torch.tensor(cand_off.astype(np.int32), device="cuda"),
                               int(cand_off[-1]), int(C.max()), tp, margin=MARGIN)
    ref = orc.check(b, obj_idx, cand_off, n_placed, placed.astype(np.float64),
                    [np.asarray(p, np.float32).astype(np.float64) for p in poses])
    return clr.cpu().numpy().astype(np.float64), col.cpu().numpy(), ref


def _assert_parity(clr, col, ref):
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(clr), fin)
    assert np.max(np.abs(clr[fin] - ref[fin]), initial=0.0) < CLR_TOL
    clear = np.abs(ref - MARGIN) >= BAND
    assert np.array_equal(col[clear].astype(bool), (ref < MARGIN)[clear])


def test_uneven_sizes_every_tile_remainder(dev, orc):
    scn, ctx, torch = dev
    # objects of 16..256 spheres; scenes of up to 12 objects
    b = sg.uneven_batch(24, seed=41, n_obj=(4, 12), n_sph=(16, 256), n_cand=(64, 128))
    gen = orc.generate(b, seed=3, default_ncand=128)
    placed = np.nan_to_num(gen["placed"], nan=0.0)
    rng = np.random.default_rng(7)
    n_placed = np.minimum(gen["n_placed"], rng.integers(0, 12, size=b.n_scenes))
    n_placed[:3] = 0                                   # nothing placed: boxes only
    obj_idx = np.minimum(b.obj_off[:-1] + n_placed, b.obj_off[1:] - 1)
    S = np.diff(b.sph_off)[obj_idx]
    P = np.array([b.sph_off[b.obj_off[s] + n_placed[s]] - b.sph_off[b.obj_off[s]]
                  for s in range(b.n_scenes)])
    # the spread of shapes this test relies on
    assert np.any(S % 16 != 0) and np.any(S > 64) and np.any(S > 192)
    assert len(set((P[P > 0] % 32).tolist())) >= 8
    C = rng.integers(1, 200, size=b.n_scenes)          # ragged candidate tiles (tile 128)
    cand_off = np.zeros(b.n_scenes + 1, np.int64)
    cand_off[1:] = np.cumsum(C)
    hx = float(np.max(b.sup[:, 12]))
    hy = float(np.max(b.sup[:, 13]))
    poses = sg.random_poses(rng, int(cand_off[-1]), hx, hy, z=(0.0, 0.3))
    clr, col, ref = _check_both(scn, ctx, torch, orc, b, obj_idx, n_placed, placed, cand_off,
                                poses)
    _assert_parity(clr, col, ref)
    assert 0.05 < np.mean(ref < MARGIN) < 0.95


@pytest.mark.parametrize("n_sph", [16, 40, 64, 100])
def test_concentric_pairs(dev, orc, n_sph):
    """The candidate is object 1 at the very pose object 0 was placed at, and
    object 1's template is object 0's: every sphere sits on a placed copy of
    itself (distance 0, clearance -2r), and the smallest clearance is
    -2 max(r).  Shifted copies probe small distances."""
    scn, ctx, torch = dev
    b = sg.uniform_batch(1, 3, n_sph, 8, 0, 0.6, 0.4, seed=11)
    s0, s1, s2 = b.sph_off[0], b.sph_off[1], b.sph_off[2]
    b.tmpl[s1:s2] = b.tmpl[s0:s1]
    gen = orc.generate(b, seed=1, default_ncand=8, max_steps=1)
    assert gen["n_placed"][0] == 1
    placed = np.nan_to_num(gen["placed"], nan=0.0)
    pose = gen["rec_pose"][0]
    # candidate 0: the placed pose; 1..5: shifted by 0.1 mm .. 3 cm in x
    shifts = np.array([0.0, 1e-4, 1e-3, 5e-3, 1e-2, 3e-2])
    poses = [pose[0] + shifts, np.full(6, pose[1]), np.full(6, pose[2]), np.full(6, pose[3])]
    cand_off = np.array([0, 6], np.int64)
    clr, col, ref = _check_both(scn, ctx, torch, orc, b, np.array([b.obj_off[0] + 1]),
                                np.array([1]), placed, cand_off, poses)
    _assert_parity(clr, col, ref)
    r = b.tmpl[s0:s1, 3].astype(np.float64)
    # the placed table holds FP32 world positions: concentric to ~1e-7 m
    assert abs(ref[0] + 2 * np.max(r)) < 1e-6
    assert np.all(col == 1)
