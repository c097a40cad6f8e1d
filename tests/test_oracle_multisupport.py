"""CPU pins of the learned path's oracle on multi-support scenes with voxel
furniture (stacked shelves): the height map covers the next object's own
support and only the objects resting on it (closed forms), and the learned
generation with a state-free ranking equals a brute force that samples the
shelf grids independently."""
import math

import numpy as np
import pytest

from gpu_util import _grid_sample_np
from oracle import bruteforce as bf
from oracle import learned as ol
from paper_2512_16896_amd import scenegen as sg

from test_oracle_pins import NTC, NXC, NYC, _bin_pose, _fixed_ranking_net


def _shelves(n_scenes=2, n_obj=6, n_sph=3, n_cand=8):
    return sg.shelf_scenes(n_scenes, seed=3, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand, chunk=2)


def _rest(b, o, x, y, yaw=0.0):
    """World spheres of object o resting on its support at (x, y, yaw)."""
    tm = b.tmpl[b.sph_off[o]:b.sph_off[o + 1]].astype(np.float64)
    sup = b.sup[b.obj_sup[o]].astype(np.float64)
    return bf.world_spheres(tm, sup, (x, y, sup[15] + float(np.max(tm[:, 3] - tm[:, 2])), yaw))


def test_state_support_is_the_next_objects():
    b = _shelves()
    for j in range(6):
        assert ol.state_support(b, 1, j) == b.obj_sup[b.obj_off[1] + j]
    assert ol.state_support(b, 1, 6) == b.obj_sup[b.obj_off[2] - 1]


def test_heightmap_covers_only_the_objects_on_its_support():
    b = _shelves()
    placed = np.full((b.n_spheres, 4), np.nan)
    # objects 0 and 1 rest on shelves 0 and 1 (round-robin), at known points
    for o, (x, y) in ((0, (0.2, -0.1)), (1, (-0.25, 0.12))):
        placed[b.sph_off[o]:b.sph_off[o + 1]] = _rest(b, o, x, y)
    for o, u in ((0, b.obj_sup[0]), (1, b.obj_sup[1])):
        H = ol.heightmap(b, placed, 0, 2, u=int(u))
        sup = b.sup[u].astype(np.float64)
        R, t, hx, hy = sup[:9].reshape(3, 3), sup[9:12], sup[12], sup[13]
        # closed form: the tops of this object's spheres above its own plane
        want = np.zeros((64, 64))
        c = -hx + (np.arange(64) + 0.5) * (2 * hx / 64), -hy + (np.arange(64) + 0.5) * (2 * hy / 64)
        X, Y = np.meshgrid(c[0], c[1], indexing="ij")
        for q in placed[b.sph_off[o]:b.sph_off[o + 1]]:
            p = R.T @ (q[:3] - t)
            d2 = (X - p[0]) ** 2 + (Y - p[1]) ** 2
            top = p[2] + np.sqrt(np.maximum(q[3] ** 2 - d2, 0.0))
            want = np.where((d2 < q[3] ** 2) & (top > 0), np.maximum(want, top), want)
        np.testing.assert_allclose(H, want, atol=1e-12)
        assert H.max() > 0 and H.max() < 0.1          # not the other shelf's object (0.4 m up)
    # a support nothing rests on yet stays flat (no boxes in shelf scenes)
    assert np.all(ol.heightmap(b, placed, 0, 2, u=int(b.obj_sup[2])) == 0)
    # the default is the next object's support
    np.testing.assert_array_equal(ol.heightmap(b, placed, 0, 2),
                                  ol.heightmap(b, placed, 0, 2, u=int(b.obj_sup[2])))


def _clearance(b, s, sph, placed):
    vals = [np.inf]
    for g in range(b.grid_off[s], b.grid_off[s + 1]):
        v = _grid_sample_np(b.grid_vals[b.grid_src[g]], b.grid[g], sph[:, :3])
        vals.append(float(np.min(v - sph[:, 3])))
    if len(placed):
        d = np.linalg.norm(sph[:, None, :3] - placed[None, :, :3], axis=2)
        vals.append(float(np.min(d - sph[:, None, 3] - placed[None, :, 3])))
    return min(vals)


def _brute_learned_grids(b, ranked, top_k, seed, margin=0.005, retries=3):
    key = (seed & 0xFFFFFFFF, seed >> 32)
    out = {}
    for s in range(b.n_scenes):
        placed = np.zeros((0, 4))
        for j, o in enumerate(range(b.obj_off[s], b.obj_off[s + 1])):
            tm = np.asarray(b.tmpl[b.sph_off[o]:b.sph_off[o + 1]], np.float64)
            sup = np.asarray(b.sup[b.obj_sup[o]], np.float64)
            ax, ay = sup[12] - sup[14], sup[13] - sup[14]
            zc = sup[15] + float(np.max(tm[:, 3] - tm[:, 2]))
            pick = pose = None
            for r in range(top_k):
                p = _bin_pose(seed, s, j, r, ranked[r], ax, ay, zc)
                if _clearance(b, s, bf.world_spheres(tm, sup, p), placed) >= margin:
                    pick, pose = (-2, r), p
                    break
            if pick is None:
                C = int(b.obj_ncand[o])
                for a in range(retries + 1):
                    u = bf.unit(bf.philox(np.stack([np.arange(C), np.full(C, a), np.full(C, j),
                                                    np.full(C, s)], 1), key))
                    for i in range(C):
                        p = (ax * (2 * u[i, 0] - 1), ay * (2 * u[i, 1] - 1), zc,
                             2 * math.pi * u[i, 2])
                        if _clearance(b, s, bf.world_spheres(tm, sup, p), placed) >= margin:
                            pick, pose = (a, i), p
                            break
                    if pick is not None:
                        break
            if pick is None:
                out[o] = (-1, -1)
                break
            out[o] = pick
            placed = np.concatenate([placed, bf.world_spheres(tm, sup, pose)])
    return out


def test_learned_generation_on_shelves_matches_bruteforce(orc):
    """Fixed ranking; the first bins sit against the bay's side wall (x cell
    0), where large objects collide with the grid, so both proposals and the
    fallback decide objects."""
    rng = np.random.default_rng(5)
    top_k, seed = 4, 0x1234_5678
    ranked = [int(0 * NYC * NTC + rng.integers(0, NYC * NTC)) for _ in range(2)] + \
             [int(rng.integers(0, 4096)) for _ in range(2)]
    ranked = list(dict.fromkeys(ranked))
    top_k = len(ranked)
    W, bias = _fixed_ranking_net(ranked)
    b = _shelves(n_scenes=2, n_obj=8, n_sph=3, n_cand=6)
    out = ol.generate_learned(b, W, bias, seed, top_k, orc, retries=3)
    want = _brute_learned_grids(b, ranked, top_k, seed, retries=3)
    assert not out["unsure"].any()
    kinds = set()
    for o, pick in want.items():
        assert tuple(int(v) for v in out["rec"][o]) == pick, o
        kinds.add(pick[0] == -2)
    assert kinds == {True, False}
