"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the FP64 oracle under the parity rule.

Parity rule (FP32 device vs FP64 oracle on identical FP32 inputs):
  * clearance within CLR_TOL metres;
  * collision flags identical unless the oracle's clearance lies within BAND
    of the margin (such candidates are counted, not compared);
  * per (scene, object) the chosen (attempt, index) is identical for every
    object before the first one whose decision involved a banded candidate
    (oracle flag); scene status identical for scenes without a banded step.
"""
import numpy as np

CLR_TOL = 1e-5
BAND = 1e-5
MARGIN = 0.005


def first_banded(out, b, s):
    o0, o1 = b.obj_off[s], b.obj_off[s + 1]
    idx = np.nonzero(out["rec_banded"][o0:o1])[0]
    return int(idx[0]) if len(idx) else o1 - o0


def compare_generation(b, ref, status, rec_i, rec_f, max_steps=None):
    """ref: oracle.generate output on batch b; status [n], rec_i [n_obj,2]
    (attempt, idx) and rec_f [n_obj,4] (x, y, z, yaw): device results for the
    same scenes and objects.  With max_steps the oracle placed only the first
    max_steps objects of each scene: only those are compared (the device may
    have gone on).  Returns (objects compared, scenes with a banded decision)."""
    n_cmp = n_band = 0
    for s in range(b.n_scenes):
        fb = first_banded(ref, b, s)
        o0, nobj = b.obj_off[s], b.obj_off[s + 1] - b.obj_off[s]
        if fb < nobj:
            n_band += 1
        if max_steps is not None:
            if int(ref["status"][s]) == 0:       # oracle stopped early on purpose
                fb = min(fb, max_steps)
                nobj = -1                        # no final status to compare
        for j in range(fb):
            o = o0 + j
            want = (int(ref["rec_attempt"][o]), int(ref["rec_idx"][o]))
            got = (int(rec_i[o, 0]), int(rec_i[o, 1]))
            assert got == want, f"scene {s} object {j}: device {got} oracle {want}"
            if want[1] >= 0:
                np.testing.assert_allclose(rec_f[o], ref["rec_pose"][o], atol=2e-6, rtol=0,
                                           err_msg=f"scene {s} object {j} pose")
            n_cmp += 1
        if fb == nobj:
            assert int(status[s]) == int(ref["status"][s]), f"scene {s} status"
    return n_cmp, n_band


def objects_of(b, scenes):
    """Object indices of the given scenes of batch b, in subset order."""
    return np.concatenate([np.arange(b.obj_off[s], b.obj_off[s + 1]) for s in scenes])


def box_distance(B, p):
    R = B[:9].reshape(3, 3).astype(np.float64)
    loc = (p - B[9:12].astype(np.float64)) @ R
    h = B[12:15].astype(np.float64)
    closest = np.clip(loc, -h, h)
    out = np.linalg.norm(loc - closest, axis=1)
    inside = np.all(np.abs(loc) <= h, axis=1)
    return np.where(inside, -np.min(h - np.abs(loc), axis=1), out)


def _grid_sample_np(vals, G, pts):
    """Trilinear samples of a node-centred grid instance at world points
    (FP64; +inf outside the node box; NaN where a node read is not finite)."""
    G = np.asarray(G, np.float64)
    pg = pts @ G[:9].reshape(3, 3).T + G[9:12]
    f = (pg - G[12:15]) / G[15]
    n = np.array([vals.shape[2], vals.shape[1], vals.shape[0]])
    inside = np.all((f >= 0) & (f <= n - 1), axis=1)
    out = np.full(len(pts), np.inf)
    if not np.any(inside):
        return out
    fi = f[inside]
    i0 = np.minimum(np.floor(fi).astype(np.int64), n - 2)
    t = fi - i0
    v = vals.astype(np.float64)
    acc = np.zeros(len(fi))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (t[:, 0] if dx else 1 - t[:, 0]) * (t[:, 1] if dy else 1 - t[:, 1]) * \
                    (t[:, 2] if dz else 1 - t[:, 2])
                acc += w * v[i0[:, 2] + dz, i0[:, 1] + dy, i0[:, 0] + dx]
    out[inside] = acc
    return out


def audit_placements(b, placed, n_placed, margin=MARGIN, tol=CLR_TOL):
    """Property of the output, in FP64: every placed object of every scene is
    at least margin - tol away from the scene's boxes and grids and from every
    other placed object of the scene (pairs found with a k-d tree; objects
    overlap only within 2 r_max + margin).  Returns the smallest clearance."""
    from scipy.spatial import cKDTree
    worst = np.inf
    placed = np.asarray(placed)
    for s in range(b.n_scenes):
        o0, npl = int(b.obj_off[s]), int(n_placed[s])
        if npl == 0:
            continue
        a0, a1 = int(b.sph_off[o0]), int(b.sph_off[o0 + npl])
        sp = placed[a0:a1].astype(np.float64)
        assert np.all(np.isfinite(sp)), f"scene {s}: non-finite placed sphere"
        owner = np.repeat(np.arange(npl), np.diff(b.sph_off[o0:o0 + npl + 1]))
        for B in b.box[b.box_off[s]:b.box_off[s + 1]]:
            worst = min(worst, float(np.min(box_distance(B, sp[:, :3]) - sp[:, 3])))
        if b.grid_off is not None:
            for g in range(b.grid_off[s], b.grid_off[s + 1]):
                v = _grid_sample_np(b.grid_vals[b.grid_src[g]], b.grid[g], sp[:, :3])
                assert not np.any(np.isnan(v))
                worst = min(worst, float(np.min(v - sp[:, 3])))
        rmax = float(np.max(sp[:, 3]))
        pairs = cKDTree(sp[:, :3]).query_pairs(2 * rmax + margin + tol, output_type="ndarray")
        if len(pairs):
            pairs = pairs[owner[pairs[:, 0]] != owner[pairs[:, 1]]]
        if len(pairs):
            d = np.linalg.norm(sp[pairs[:, 0], :3] - sp[pairs[:, 1], :3], axis=1)
            worst = min(worst, float(np.min(d - sp[pairs[:, 0], 3] - sp[pairs[:, 1], 3])))
    assert worst >= margin - tol, worst
    return worst


def rot_xy(ax: float, ay: float) -> np.ndarray:
    """Rotation about x by ax, then about y by ay (a tilt: not a turn about z)."""
    cx, sx, cy, sy = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    return Ry @ Rx


def tilted(b, Q):
    """The same scenes moved by the world rotation Q: supports and boxes turn
    with the world, so every candidate's clearance is unchanged (up to
    rounding) while no rotation is a turn about z any more."""
    import dataclasses
    sup = np.array(b.sup, np.float64).reshape(-1, 16)
    sup[:, :9] = (Q @ sup[:, :9].reshape(-1, 3, 3)).reshape(-1, 9)
    sup[:, 9:12] = sup[:, 9:12] @ Q.T
    box = np.array(b.box, np.float64).reshape(-1, 16)
    box[:, :9] = (Q @ box[:, :9].reshape(-1, 3, 3)).reshape(-1, 9)
    box[:, 9:12] = box[:, 9:12] @ Q.T
    return dataclasses.replace(b, sup=sup.astype(np.float32),
                               box=box.astype(np.float32).reshape(np.shape(b.box)))
