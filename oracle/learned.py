"""FP64 oracle of the learned pose proposal (test infrastructure only).

Plain NumPy definitions of what the learned path computes: the object
descriptor, the support height map of a state, the network input rows, the
4-layer perceptron (forward and exact backward in FP64 on BF16-rounded
weights, inputs and activations, the rounding points of the device path),
binary cross-entropy on labelled bins, one AdamW step, the top-k bin ranking,
and the pose drawn inside a proposed bin.  Random bits come from the
oracle's own Philox (oracle.philox4x32_10 / bruteforce.philox).

Not imported by the product path; shares no code with it.
"""
from __future__ import annotations

import math

import numpy as np

from . import bruteforce as bf

HMAP = 64
NX, NY, NYAW = 32, 16, 8          # pose bins: x cells, y cells, yaw cells
N_BINS = NX * NY * NYAW


# ---------------------------------------------------------------------------
# BF16 rounding (round to nearest even), applied to FP32 values
def bf16(a) -> np.ndarray:
    f = np.asarray(a, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
def descriptor(tmpl: np.ndarray) -> np.ndarray:
    """32 sphere-set moments of one object template [S,4] (object frame)."""
    t = np.asarray(tmpl, np.float64)
    c, r = t[:, :3], t[:, 3]
    S = len(r)
    d = np.zeros(32)
    if S == 0:
        return d
    r3 = r ** 3
    mean_c = c.mean(0)
    cov = (c - mean_c).T @ (c - mean_c) / S
    lo, hi = (c - r[:, None]).min(0), (c + r[:, None]).max(0)
    lift = np.max(r - c[:, 2])
    d[0] = S / 256.0
    d[1:5] = 10 * np.array([r.mean(), r.min(), r.max(), r.std()])
    d[5] = 1e3 * r3.sum()
    d[6:9] = 10 * (r3[:, None] * c).sum(0) / r3.sum()
    d[9:15] = 100 * np.array([cov[0, 0], cov[1, 1], cov[2, 2], cov[0, 1], cov[0, 2], cov[1, 2]])
    d[15:18] = 10 * 0.5 * (hi - lo)
    d[18] = 10 * lift
    d[19] = 10 * (np.max(c[:, 2] + r) + lift)
    d[20] = 10 * np.max(np.hypot(c[:, 0], c[:, 1]) + r)
    return d


def state_support(b, s: int, n_state: int) -> int:
    """The support a state's height map covers: that of the scene's next
    object (object n_state), or of its last one when every object is placed."""
    o0, o1 = int(b.obj_off[s]), int(b.obj_off[s + 1])
    o = min(o0 + n_state, o1 - 1) if o1 > o0 else o0
    return int(b.obj_sup[o])


def heightmap(b, placed: np.ndarray, s: int, n_state: int, u: int = None) -> np.ndarray:
    """Height map [64,64] (metres above the support plane) over support u
    (default: the state's, see state_support) of scene s with its first
    n_state objects placed (world spheres in `placed`, parallel to the
    templates): the scene's boxes, and the placed objects that rest on u.
    Cell (ix, iy) centre (-hx + (ix+1/2) 2hx/64, -hy + ...)."""
    if u is None:
        u = state_support(b, s, n_state)
    row = np.asarray(b.sup[int(u)], np.float64)
    R, t, hx, hy = row[:9].reshape(3, 3), row[9:12], row[12], row[13]
    ix = np.arange(HMAP)
    cx = -hx + (ix + 0.5) * (2 * hx / HMAP)
    cy = -hy + (ix + 0.5) * (2 * hy / HMAP)
    X, Y = np.meshgrid(cx, cy, indexing="ij")
    H = np.zeros((HMAP, HMAP))
    for bx in range(int(b.box_off[s]), int(b.box_off[s + 1])):
        B = np.asarray(b.box[bx], np.float64)
        Rb, cb, h = B[:9].reshape(3, 3), B[9:12], B[12:15]
        Rl = R.T @ Rb                    # box axes in the support frame (columns)
        cl = R.T @ (cb - t)
        dx, dy = X - cl[0], Y - cl[1]    # cell centres at the box centre's height
        qx = Rl[0, 0] * dx + Rl[1, 0] * dy
        qy = Rl[0, 1] * dx + Rl[1, 1] * dy
        top = cl[2] + np.abs(Rl[2, :]) @ h
        H = np.where((np.abs(qx) <= h[0]) & (np.abs(qy) <= h[1]), np.maximum(H, top), H)
    o0 = int(b.obj_off[s])
    on_u = [o for o in range(o0, o0 + n_state) if int(b.obj_sup[o]) == int(u)]
    rows = [np.asarray(placed[int(b.sph_off[o]):int(b.sph_off[o + 1])], np.float64) for o in on_u]
    for q in (np.concatenate(rows) if rows else np.zeros((0, 4))):
        p = R.T @ (q[:3] - t)
        d2 = (X - p[0]) ** 2 + (Y - p[1]) ** 2
        inside = d2 < q[3] ** 2
        top = p[2] + np.sqrt(np.where(inside, q[3] ** 2 - d2, 0.0))
        H = np.where(inside & (top > 0), np.maximum(H, top), H)
    return H


def features(hmap: np.ndarray, desc: np.ndarray) -> np.ndarray:
    """Network input row (BF16 values): [10 * height map (ix-major), descriptor]."""
    return bf16(np.concatenate([10.0 * np.asarray(hmap, np.float64).reshape(-1),
                                np.asarray(desc, np.float64)]))


# ---------------------------------------------------------------------------
# The network.  W[l] is [out, in] (FP32 master values); the device multiplies
# BF16(W[l]) with BF16 activations and accumulates in FP32; hidden outputs are
# rounded to BF16 after the ReLU.
def forward(x, W, b, round_bf16=True):
    """Returns (logits, [inputs of each layer])."""
    q = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    h = q(x)
    ins = []
    for l in range(len(W)):
        ins.append(h)
        z = h @ q(W[l]).T + np.asarray(b[l], np.float64)
        if l < len(W) - 1:
            h = q(np.maximum(z, 0.0))
        else:
            return z, ins


def bce_loss(z, bins, tgt):
    """Mean over the M*L label slots of softplus(z) - t z at the labelled bins
    (slots with bin < 0 count as zero)."""
    M, L = bins.shape
    total = 0.0
    g = np.zeros_like(z)
    for m in range(M):
        for i in range(L):
            bn = int(bins[m, i])
            if bn < 0:
                continue
            zz, t = float(z[m, bn]), float(tgt[m, i])
            total += max(zz, 0.0) - zz * t + math.log1p(math.exp(-abs(zz)))
            g[m, bn] += (1.0 / (1.0 + math.exp(-zz)) - t) / (M * L)
    return total / (M * L), g


def backward(x, W, b, bins, tgt, round_bf16=True):
    """Exact FP64 gradients of bce_loss(forward(x)) w.r.t. W and b (the BF16
    rounding of weights and activations is treated as part of the inputs:
    gradients flow through it unchanged)."""
    q = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    z, ins = forward(x, W, b, round_bf16)
    loss, dz = bce_loss(z, bins, tgt)
    gW, gb = [None] * len(W), [None] * len(W)
    d = dz
    for l in range(len(W) - 1, -1, -1):
        gW[l] = d.T @ ins[l]
        gb[l] = d.sum(0)
        if l == 0:
            break
        d = (d @ q(W[l])) * (ins[l] > 0)
    return loss, gW, gb


def adamw_step(w, g, m, v, step, lr, b1, b2, eps, wd):
    """One AdamW step (decoupled decay, bias-corrected); returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    t = step + 1
    mh, vh = m / (1 - b1 ** t), v / (1 - b2 ** t)
    return w - lr * (mh / (np.sqrt(vh) + eps) + wd * w), m, v


# ---------------------------------------------------------------------------
def topk(logits: np.ndarray, k: int) -> np.ndarray:
    """Rank order of bins: logit descending, ties to the lower bin."""
    z = np.asarray(logits, np.float64)
    order = np.lexsort((np.arange(len(z)), -z))
    return order[:k]


def bin_of(u0, u1, u2) -> int:
    """Pose bin of a candidate drawn from uniforms (u0 -> x, u1 -> y, u2 -> yaw)."""
    return (min(int(u0 * NX), NX - 1) * NY + min(int(u1 * NY), NY - 1)) * NYAW + \
        min(int(u2 * NYAW), NYAW - 1)


def proposal_pose(seed: int, s: int, j: int, rank: int, bin_: int, ax: float, ay: float,
                  z: float):
    """Pose drawn inside pose bin `bin_` for the proposal of rank `rank`:
    Philox counter (rank, 0x10000, j, s); x = ax (2 u0 - 1) with
    u0 = (x cell + unit) / 32, and likewise y (16 cells) and yaw (8 cells)."""
    w = bf.philox(np.array([[rank, 0x10000, j, s]]), (seed & 0xFFFFFFFF, seed >> 32))[0]
    u = bf.unit(w)
    ix, iy, it = bin_ // (NY * NYAW), (bin_ // NYAW) % NY, bin_ % NYAW
    u0, u1, u2 = (ix + u[0]) / NX, (iy + u[1]) / NY, (it + u[2]) / NYAW
    return ax * (2 * u0 - 1), ay * (2 * u1 - 1), z, 2 * math.pi * u2


def generate_learned(b, W, bias, seed: int, top_k: int, orc, margin=0.005, retries=10,
                     band=1e-5, rank_tol=None, scene_id=None):
    """Learned-proposal placement of every scene of batch b (independent per
    scene): for object j the state's height map and the object's descriptor
    go through the network; the top_k bins are tried in rank order (one pose
    drawn inside each), then the uniform attempts 0..retries as in the plain
    method.  `orc` is the FP64 oracle module (its checker and sampler).
    Returns per-object (attempt, idx) (attempt -2 = proposal of rank idx),
    status per scene, and for each object whether its decision involved a
    banded clearance or a near-tie of the ranking (then the decision is not
    compared)."""
    n = b.n_scenes
    rec = -np.ones((b.n_objects, 2), np.int64)
    pose = np.full((b.n_objects, 4), np.nan)
    unsure = np.zeros(b.n_objects, bool)
    status = np.zeros(n, np.int8)
    placed = np.zeros((b.n_spheres, 4))
    import paper_2512_16896_amd.scenegen as sg
    for s in range(n):
        sid = s if scene_id is None else int(scene_id[s])
        one, _ = sg.subset(b, [s])
        o0 = int(b.obj_off[s])
        ok = True
        for j in range(int(b.obj_off[s + 1]) - o0):
            o = o0 + j
            tm = np.asarray(b.tmpl[int(b.sph_off[o]):int(b.sph_off[o + 1])], np.float64)
            sup = np.asarray(b.sup[int(b.obj_sup[o])], np.float64)
            ax, ay = sup[12] - sup[14], sup[13] - sup[14]
            zc = sup[15] + np.max(tm[:, 3] - tm[:, 2])
            H = heightmap(b, placed, s, j)
            x = features(H, descriptor(tm))
            z, _ = forward(x[None], W, bias)
            z = z[0]
            ranks = topk(z, top_k + 1)
            tol = rank_tol if rank_tol is not None else 5e-3 * float(np.max(np.abs(z))) + 1e-4
            poses = np.array([proposal_pose(seed, sid, j, r, int(ranks[r]), ax, ay, zc)
                              for r in range(top_k)])
            oj = np.array([j], np.int32)
            one_placed = placed[int(b.sph_off[o0]):int(b.sph_off[int(b.obj_off[s + 1])])]
            clr = orc.check(one, oj, [0, top_k], [j], one_placed, poses.T, scene_id=[sid])
            hit = np.nonzero(clr >= margin)[0]
            checked = int(hit[0]) + 1 if len(hit) else top_k
            zs = z[ranks]
            if np.any(zs[:checked] - zs[1:checked + 1] < tol):
                unsure[o] = True
            if np.any(np.abs(clr[:checked] - margin) < band):
                unsure[o] = True
            if len(hit):
                r = int(hit[0])
                rec[o] = (-2, r)
                pose[o] = poses[r]
            else:
                C = int(b.obj_ncand[o])
                for a in range(retries + 1):
                    ps = orc.sample_poses(one, oj, [0, C], seed, a, scene_id=[sid])
                    cl = orc.check(one, oj, [0, C], [j], one_placed, ps, scene_id=[sid])
                    hh = np.nonzero(cl >= margin)[0]
                    last = int(hh[0]) + 1 if len(hh) else C
                    if np.any(np.abs(cl[:last] - margin) < band):
                        unsure[o] = True
                    if len(hh):
                        i = int(hh[0])
                        rec[o] = (a, i)
                        pose[o] = [ps[0][i], ps[1][i], ps[2][i], ps[3][i]]
                        break
            if rec[o, 1] < 0:
                ok = False
                break
            placed[int(b.sph_off[o]):int(b.sph_off[o + 1])] = bf.world_spheres(tm, sup, pose[o])
        status[s] = 1 if ok else 2
    return dict(rec=rec, pose=pose, unsure=unsure, status=status, placed=placed)


def harvest_labels(b, placed, s: int, n_state: int, L: int, seed: int, round_: int,
                   margin: float, check):
    """Labels of a state: L uniform candidates of the next object (counter
    (i, 0x20000 | round, n_state, s)); returns (bins, accept).  `check`
    evaluates clearances of poses (the FP64 oracle checker)."""
    o = int(b.obj_off[s]) + n_state
    if o >= int(b.obj_off[s + 1]):
        return -np.ones(L, np.int64), np.zeros(L)
    ctr = np.stack([np.arange(L), np.full(L, 0x20000 | round_), np.full(L, n_state),
                    np.full(L, s)], 1)
    w = bf.philox(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    u = bf.unit(w)
    sup = np.asarray(b.sup[int(b.obj_sup[o])], np.float64)
    tm = np.asarray(b.tmpl[int(b.sph_off[o]):int(b.sph_off[o + 1])], np.float64)
    lift = sup[15] + np.max(tm[:, 3] - tm[:, 2])
    x = (sup[12] - sup[14]) * (2 * u[:, 0] - 1)
    y = (sup[13] - sup[14]) * (2 * u[:, 1] - 1)
    yaw = 2 * np.pi * u[:, 2]
    clr = check(o, (x, y, np.full(L, lift), yaw))
    bins = np.array([bin_of(*u[i, :3]) for i in range(L)])
    return bins, (clr >= margin).astype(np.float64)
