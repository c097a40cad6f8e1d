"""CPU pins of the oracle's stable-pose orientations (Sec. III "Main
algorithm": orientations from stable poses, then a random turn about z):
the row choice follows the weights (chi-square), a placed object rests its
lowest point on the support, the world spheres equal an independent
transform of the template, a face-down box stands on the chosen face (closed
form), an identity table changes nothing, and generation equals an
independent brute force on tiny scenes."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import bruteforce as bf
from paper_2512_16896_amd import scenegen as sg

from test_oracle import _random_tiny, tiny_batch


def _rz(a):
    return np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])


def _with_table(b, rows_per_obj):
    """b with stable-pose rows per object (list of [K,12] arrays or None)."""
    counts = [0 if r is None else len(r) for r in rows_per_obj]
    off = np.zeros(len(counts) + 1, np.int32)
    off[1:] = np.cumsum(counts)
    rows = [r for r in rows_per_obj if r is not None]
    b.obj_pose_off = off
    b.stable = (np.concatenate(rows) if rows else np.zeros((0, 12))).astype(np.float32)
    return b


def test_rows_follow_the_weights(orc):
    b = sg.stable_scenes(2, seed=3)
    o = 1                                        # a face-table object (6 rows)
    r0, r1 = int(b.obj_pose_off[o]), int(b.obj_pose_off[o + 1])
    cum = b.stable[r0:r1, 9].astype(np.float64)
    p = np.diff(np.concatenate([[0.0], cum]))
    n = 60000
    *_, k = orc.sample_poses(b, [o, -1], [0, n, n], seed=77, attempt=0, with_stable=True)
    assert k.min() >= r0 and k.max() < r1
    hist = np.bincount(k - r0, minlength=r1 - r0)
    assert stats.chisquare(hist, p * n).pvalue > 1e-3
    # objects without rows take none
    *_, k0 = orc.sample_poses(b, [0, -1], [0, 10, 10], seed=77, attempt=0, with_stable=True)
    assert np.all(k0 == -1)


def test_placed_objects_rest_on_the_support_and_match_an_independent_transform(orc):
    b = sg.stable_scenes(12, seed=5)
    out = orc.generate(b, seed=9, default_ncand=256, early_exit=True)
    n_chk = {0: 0, 1: 0, 2: 0}
    for s in range(b.n_scenes):
        for j in range(int(out["n_placed"][s])):
            o = b.obj_off[s] + j
            u = b.sup[b.obj_sup[o]].astype(np.float64)
            Ru, tu = u[:9].reshape(3, 3), u[9:12]
            c = b.tmpl[b.sph_off[o]:b.sph_off[o + 1]].astype(np.float64)
            k = int(out["rec_stable"][o])
            Rk = np.eye(3) if k < 0 else b.stable[k, :9].astype(np.float64).reshape(3, 3)
            x, y, z, yaw = out["rec_pose"][o]
            rest = c[:, :3] @ Rk.T
            # z = support lift + the rest lift of the turned sphere set
            assert z == pytest.approx(u[15] + np.max(c[:, 3] - rest[:, 2]), abs=1e-12)
            want = (rest @ _rz(yaw).T + [x, y, z]) @ Ru.T + tu
            got = out["placed"][b.sph_off[o]:b.sph_off[o + 1]]
            np.testing.assert_allclose(got[:, :3], want, atol=1e-12)
            np.testing.assert_array_equal(got[:, 3], c[:, 3])
            # the lowest point touches the support plane (support frame)
            local = (got[:, :3] - tu) @ Ru
            assert np.min(local[:, 2] - c[:, 3]) == pytest.approx(u[15], abs=1e-12)
            n_chk[o % 3] += 1
            assert (k < 0) == (o % 3 == 0)
    assert min(n_chk.values()) > 20


def test_face_down_box_stands_on_the_chosen_face(orc):
    # eight spheres at the corners of a 0.2 x 0.1 x 0.06 box, radius 0.01
    corners = np.array([[sx * 0.1, sy * 0.05, sz * 0.03] for sx in (-1, 1) for sy in (-1, 1)
                        for sz in (-1, 1)])
    obj = np.concatenate([corners, np.full((8, 1), 0.01)], 1)
    faces = sg.face_down_rotations()
    for f, axis in ((0, 0), (2, 1), (4, 2)):      # +x, +y, +z face down
        b = _with_table(tiny_batch([obj], hx=0.4, hy=0.3, ncand=4),
                        [sg.stable_rows(faces[f:f + 1], [1.0])])
        out = orc.generate(b, seed=3)
        assert out["status"][0] == 1 and out["rec_stable"][0] == 0
        z = out["placed"][:, 2]
        # the box's extent along the chosen axis (of the stored FP32 template)
        # is now its height, and its lowest sphere touches the plane z = 0
        height = np.ptp(b.tmpl[:, axis].astype(np.float64))
        assert np.ptp(z) == pytest.approx(height, abs=1e-12)
        r = float(np.float32(0.01))
        assert np.min(z) - r == pytest.approx(0.0, abs=1e-12)


def test_identity_table_changes_nothing(orc):
    b = sg.stable_scenes(10, seed=2)
    b.obj_pose_off = None
    b.stable = None
    ref = orc.generate(b, seed=4, default_ncand=256, early_exit=True)
    eye = sg.stable_rows(np.eye(3)[None], [1.0])
    bi = _with_table(sg.stable_scenes(10, seed=2), [eye] * b.n_objects)
    got = orc.generate(bi, seed=4, default_ncand=256, early_exit=True)
    for key in ("status", "n_placed", "rec_attempt", "rec_idx"):
        np.testing.assert_array_equal(ref[key], got[key])
    np.testing.assert_array_equal(ref["rec_pose"], got["rec_pose"])
    np.testing.assert_array_equal(ref["placed"], got["placed"])


def test_generate_with_stable_poses_matches_bruteforce(orc):
    rng = np.random.default_rng(12)
    n_ok = n_bad = 0
    for trial in range(12):
        b = _random_tiny(rng, 4, int(rng.integers(0, 6)), S=int(rng.integers(1, 5)),
                         ncand=int(rng.integers(1, 9)), box_h=(0.05, 0.3))
        tables = []
        for o in range(b.n_objects):
            K = int(rng.integers(0, 5))
            tables.append(None if K == 0 else
                          sg.stable_rows(sg.haar_rotations(rng, K), rng.uniform(0.1, 1.0, K)))
        b = _with_table(b, tables)
        seed = int(rng.integers(0, 2 ** 63))
        out = orc.generate(b, seed=seed, retries=3)
        ref = bf.generate(b, seed, retries=3)
        for s, (status, picks) in enumerate(ref):
            assert int(out["status"][s]) == status
            objs = range(b.obj_off[s], b.obj_off[s] + len(picks))
            got = [(int(out["rec_attempt"][o]), int(out["rec_idx"][o])) for o in objs]
            assert got == picks
            n_ok += status == 1
            n_bad += status == 2
    assert n_ok > 0 and n_bad > 0


def test_check_takes_the_stable_row(orc):
    """orc.check with an explicit row equals the brute-force clearance of the
    turned template."""
    rng = np.random.default_rng(8)
    b = _random_tiny(rng, 2, 3)
    R = sg.haar_rotations(rng, 3)
    b = _with_table(b, [sg.stable_rows(R, [1, 1, 1])] * b.n_objects)
    poses = list(sg.random_poses(rng, 12, 0.35, 0.25, z=(0.05, 0.2)))
    kk = np.concatenate([b.obj_pose_off[0] + rng.integers(0, 3, 6), b.obj_pose_off[2] + rng.integers(0, 3, 6)]).astype(np.int32)
    placed = np.full((b.n_spheres, 4), np.nan)
    clr = orc.check(b, [0, 2], [0, 6, 12], [0, 0], placed, poses + [kk])
    for t in range(12):
        s = t // 6
        o = b.obj_off[s]
        tm = b.tmpl[b.sph_off[o]:b.sph_off[o + 1]].astype(np.float64)
        Rk = b.stable[kk[t], :9].astype(np.float64).reshape(3, 3)
        rest = np.concatenate([tm[:, :3] @ Rk.T, tm[:, 3:]], 1)
        sph = bf.world_spheres(rest, b.sup[b.obj_sup[o]].astype(np.float64),
                               [float(a[t]) for a in poses])
        want = bf.clearance(sph, b.box[b.box_off[s]:b.box_off[s + 1]].astype(np.float64),
                            np.zeros((0, 4)))
        assert clr[t] == pytest.approx(want, abs=1e-12)
