"""Independent NumPy float64 brute force for tiny scenes (test infrastructure).

A second, differently written formulation of what oracle.c computes, used to
pin it on tiny inputs:
  * Philox4x32-10 vectorised over uint64 lanes (Salmon et al., SC'11);
  * box distance by clamping to the closest point of the box (outside) and by
    the distance to the nearest face (inside) instead of the q-vector SDF;
  * sphere distances by broadcasting over all pairs;
  * rejection sampling written as "build the whole validity vector of an
    attempt, take the first True".
It shares no code with oracle.c or with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox(ctr: np.ndarray, key) -> np.ndarray:
    """ctr: [n,4] uint32-valued, key: (k0, k1) -> [n,4] uint32."""
    c = np.asarray(ctr, np.uint64).reshape(-1, 4).copy()
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[:, 0]
        p1 = _M1 * c[:, 2]
        n0 = (p1 >> np.uint64(32)) ^ c[:, 1] ^ np.uint64(k0)
        n1 = p1 & _MASK
        n2 = (p0 >> np.uint64(32)) ^ c[:, 3] ^ np.uint64(k1)
        n3 = p0 & _MASK
        c = np.stack([n0, n1, n2, n3], 1)
    return c.astype(np.uint32)


def unit(w: np.ndarray) -> np.ndarray:
    return ((np.asarray(w, np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) / 2.0 ** 23


def box_distance(R, c, h, p) -> np.ndarray:
    """Signed distance of points p [n,3] to a box, via the closest point."""
    R = np.asarray(R, np.float64).reshape(3, 3)
    loc = (np.asarray(p, np.float64) - np.asarray(c, np.float64)) @ R   # = R^T (p - c)
    h = np.asarray(h, np.float64)
    closest = np.clip(loc, -h, h)
    out = np.linalg.norm(loc - closest, axis=1)
    inside = np.all(np.abs(loc) <= h, axis=1)
    depth = np.min(h - np.abs(loc), axis=1)
    return np.where(inside, -depth, out)


def world_spheres(tmpl, sup_row, pose) -> np.ndarray:
    x, y, z, yaw = pose
    Rz = np.array([[math.cos(yaw), -math.sin(yaw), 0], [math.sin(yaw), math.cos(yaw), 0],
                   [0, 0, 1.0]])
    R = np.asarray(sup_row[:9], np.float64).reshape(3, 3)
    t = np.asarray(sup_row[9:12], np.float64)
    loc = np.asarray(tmpl[:, :3], np.float64) @ Rz.T + np.array([x, y, z])
    return np.concatenate([loc @ R.T + t, np.asarray(tmpl[:, 3:4], np.float64)], 1)


def clearance(sph: np.ndarray, boxes: np.ndarray, placed: np.ndarray) -> float:
    vals = [np.inf]
    for B in boxes:
        vals.append(np.min(box_distance(B[:9], B[9:12], B[12:15], sph[:, :3]) - sph[:, 3]))
    if len(placed):
        d = np.linalg.norm(sph[:, None, :3] - placed[None, :, :3], axis=2)
        vals.append(np.min(d - sph[:, None, 3] - placed[None, :, 3]))
    return float(min(vals))


def generate(b, seed: int, margin=0.005, retries=10, scene_id=None):
    """Rejection sampling for every scene of a tiny batch.
    Returns per scene a list of (attempt, idx) per placed object and the status."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    results = []
    for s in range(b.n_scenes):
        sid = s if scene_id is None else int(scene_id[s])
        boxes = np.asarray(b.box[b.box_off[s]:b.box_off[s + 1]], np.float64)
        placed = np.zeros((0, 4))
        picks, status = [], 1
        for step, o in enumerate(range(b.obj_off[s], b.obj_off[s + 1])):
            tmpl = np.asarray(b.tmpl[b.sph_off[o]:b.sph_off[o + 1]], np.float64)
            sup = np.asarray(b.sup[b.obj_sup[o]], np.float64)
            C = int(b.obj_ncand[o])
            # stable poses: the template turned into each row's resting frame
            rows = None
            if getattr(b, "obj_pose_off", None) is not None:
                r0, r1 = int(b.obj_pose_off[o]), int(b.obj_pose_off[o + 1])
                if r1 > r0:
                    rows = np.asarray(b.stable[r0:r1], np.float64)
            pick = None
            for a in range(retries + 1):
                ctr = np.stack([np.arange(C), np.full(C, a), np.full(C, step), np.full(C, sid)], 1)
                w = philox(ctr, key)
                u = unit(w)
                xs = (sup[12] - sup[14]) * (2 * u[:, 0] - 1)
                ys = (sup[13] - sup[14]) * (2 * u[:, 1] - 1)
                yaws = 2 * math.pi * u[:, 2]
                if rows is None:
                    rest = [tmpl] * C
                else:
                    ks = np.minimum(np.searchsorted(rows[:, 9], u[:, 3], side="left"), len(rows) - 1)
                    rest = [np.concatenate([tmpl[:, :3] @ rows[k, :9].reshape(3, 3).T, tmpl[:, 3:]], 1)
                            for k in ks]
                lifts = [float(np.max(t[:, 3] - t[:, 2])) for t in rest]
                ok = np.array([clearance(world_spheres(rest[i], sup, (xs[i], ys[i], sup[15] + lifts[i],
                                                                        yaws[i])), boxes, placed)
                               >= margin for i in range(C)])
                if ok.any():
                    i = int(np.argmax(ok))
                    pick = (a, i)
                    placed = np.concatenate(
                        [placed, world_spheres(rest[i], sup, (xs[i], ys[i], sup[15] + lifts[i], yaws[i]))])
                    break
            if pick is None:
                status = 2
                picks.append((-1, -1))
                break
            picks.append(pick)
        results.append((status, picks))
    return results
