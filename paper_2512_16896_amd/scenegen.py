"""Seeded synthetic scene batches (inputs only).

This module draws the *inputs* of a placement run: object sphere templates,
support surfaces and their world poses, static boxes and voxel-grid furniture.
It holds none of the placement method's arithmetic (no pose sampling, no
collision test, no selection); both the HIP path and the CPU oracle read the
arrays it returns.

Layouts (row-major, FP32 unless noted):
  obj_off   int32 [n+1]        objects of scene s: obj_off[s] .. obj_off[s+1]-1,
                               in placement order
  sph_off   int32 [n_obj+1]    template spheres of object o
  tmpl      float32 [n_sph,4]  sphere (x, y, z, r) in the object frame
  obj_sup   int32 [n_obj]      support surface index of object o
  obj_ncand int32 [n_obj]      candidates drawn per attempt for object o
  sup       float32 [n_sup,16] R[9] (row-major, support->world), t[3],
                               half-x, half-y, inset, z lift
  box_off   int32 [n+1]        static boxes of scene s
  box       float32 [n_box,16] R[9] (box->world), centre[3], half extents[3], 0
  grid_*    voxel-grid furniture (optional, multi-shelf workload only)

The workloads follow the five synthetic configurations of the project (one
table scene; 4096 batched scenes; 16384 uneven scenes; the learned-proposal
workload on 4096-scene shapes; dense shelves with voxel grids).  Sizes that
the paper does not give are the readings recorded in the design notes.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import math
import os
from typing import Optional

import numpy as np

# Clutter knob: static box centres are drawn over the support rectangle grown
# by this many metres on each side (calibrated so that the plain method leaves
# a non-degenerate fraction of scenes valid on the 4096-scene workload).
BOX_SPREAD_DEFAULT = 1.0


@dataclasses.dataclass
class SceneBatch:
    obj_off: np.ndarray
    sph_off: np.ndarray
    tmpl: np.ndarray
    obj_sup: np.ndarray
    obj_ncand: np.ndarray
    sup: np.ndarray
    box_off: np.ndarray
    box: np.ndarray
    # voxel-grid furniture (None when absent)
    grid_off: Optional[np.ndarray] = None     # int32 [n+1]
    grid: Optional[np.ndarray] = None         # float32 [n_grid,24] see grid_instance()
    grid_src: Optional[np.ndarray] = None     # int32 [n_grid] asset index
    grid_vals: Optional[list] = None          # list of float32 [nz,ny,nx] assets
    # object-object spatial relations and support erosion (None when absent)
    obj_rel: Optional[np.ndarray] = None      # int32 [n_obj] relation row, -1 none
    rel: Optional[np.ndarray] = None          # float32 [n_rel,16] relation rows
    obj_ratio: Optional[np.ndarray] = None    # float32 [n_obj] ratio_on_support
    # reachability (None when absent)
    robot: Optional[np.ndarray] = None        # float32 [n,12] robot base pose per scene
    obj_reach: Optional[np.ndarray] = None    # float32 [n_obj] approach angle, < 0 no check
    reach_map: Optional[np.ndarray] = None    # uint8 [nz, ntheta, nx, ny], 1 = reachable
    reach_geom: Optional[np.ndarray] = None   # float32 [12] lo[4], h[4], dims[4]
    # stable poses (None when absent): rows [obj_pose_off[o], obj_pose_off[o+1])
    obj_pose_off: Optional[np.ndarray] = None  # int32 [n_obj+1]
    stable: Optional[np.ndarray] = None        # float32 [n_rows,12] R[9], cumulative weight, 0, 0
    name: str = ""
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_scenes(self) -> int:
        return int(self.obj_off.shape[0] - 1)

    @property
    def n_objects(self) -> int:
        return int(self.sph_off.shape[0] - 1)

    @property
    def n_spheres(self) -> int:
        return int(self.tmpl.shape[0])

    @property
    def n_boxes(self) -> int:
        return int(self.box.shape[0])

    def objects_per_scene(self) -> np.ndarray:
        return np.diff(self.obj_off)

    def spheres_per_object(self) -> np.ndarray:
        return np.diff(self.sph_off)

    def spheres_per_scene(self) -> np.ndarray:
        return self.sph_off[self.obj_off[1:]] - self.sph_off[self.obj_off[:-1]]

    def boxes_per_scene(self) -> np.ndarray:
        return np.diff(self.box_off)


def rotz(a: np.ndarray) -> np.ndarray:
    """Rotation matrices about z for an array of angles -> [..., 3, 3]."""
    c, s = np.cos(a), np.sin(a)
    z, o = np.zeros_like(a), np.ones_like(a)
    return np.stack([np.stack([c, -s, z], -1), np.stack([s, c, z], -1),
                     np.stack([z, z, o], -1)], -2)


def _support_rows(R: np.ndarray, t: np.ndarray, hx, hy, inset, lift) -> np.ndarray:
    n = R.shape[0]
    out = np.zeros((n, 16), np.float64)
    out[:, 0:9] = R.reshape(n, 9)
    out[:, 9:12] = t
    out[:, 12] = hx
    out[:, 13] = hy
    out[:, 14] = inset
    out[:, 15] = lift
    return out.astype(np.float32)


def _templates(rng, n_obj, S, side=(0.05, 0.25), rad=(0.01, 0.05)):
    """Sphere sets: per object a cube side L ~ U(side); centres uniform in the
    cube [-L/2, L/2]^3, radii ~ U(rad).  S may be an int or a per-object array."""
    S = np.broadcast_to(np.asarray(S, np.int64), (n_obj,))
    sph_off = np.zeros(n_obj + 1, np.int64)
    sph_off[1:] = np.cumsum(S)
    tot = int(sph_off[-1])
    L = rng.uniform(side[0], side[1], size=n_obj)
    Lrep = np.repeat(L, S)
    c = (rng.random((tot, 3)) - 0.5) * Lrep[:, None]
    r = rng.uniform(rad[0], rad[1], size=tot)
    tmpl = np.concatenate([c, r[:, None]], 1)
    return sph_off, tmpl


def _footprint_order(obj_off, sph_off, tmpl):
    """Placement order inside each scene: descending footprint radius
    (largest objects first).  Returns a permutation of the objects."""
    n_obj = sph_off.shape[0] - 1
    rho = np.hypot(tmpl[:, 0], tmpl[:, 1]) + tmpl[:, 3]
    fp = np.maximum.reduceat(rho, sph_off[:-1]) if n_obj else np.zeros(0)
    scene_of = np.repeat(np.arange(obj_off.shape[0] - 1), np.diff(obj_off))
    return np.lexsort((-fp, scene_of))


def _ranges(starts, lengths):
    """Concatenation of arange(starts[i], starts[i] + lengths[i])."""
    lengths = np.asarray(lengths, np.int64)
    tot = int(lengths.sum())
    if tot == 0:
        return np.zeros(0, np.int64)
    first = np.zeros(len(lengths), np.int64)
    first[1:] = np.cumsum(lengths)[:-1]
    return np.repeat(np.asarray(starts, np.int64) - first, lengths) + np.arange(tot)


def _reorder_objects(perm, sph_off, tmpl, *per_obj):
    S = np.diff(sph_off)[perm]
    new_off = np.zeros_like(sph_off)
    new_off[1:] = np.cumsum(S)
    idx = _ranges(sph_off[perm], S)
    return (new_off, tmpl[idx]) + tuple(a[perm] for a in per_obj)


def _boxes(rng, n, B, hx, hy, spread, sup_R, sup_t, half=(0.05, 0.5)):
    """Static cuboids resting on each scene's support: half extents ~ U(half)^3,
    yaw ~ U[0, 2pi), centre uniform over the support grown by `spread`."""
    B = np.broadcast_to(np.asarray(B, np.int64), (n,))
    hx = np.broadcast_to(np.asarray(hx, np.float64), (n,))
    hy = np.broadcast_to(np.asarray(hy, np.float64), (n,))
    box_off = np.zeros(n + 1, np.int64)
    box_off[1:] = np.cumsum(B)
    tot = int(box_off[-1])
    scene = np.repeat(np.arange(n), B)
    h = rng.uniform(half[0], half[1], size=(tot, 3))
    yaw = rng.uniform(0, 2 * np.pi, size=tot)
    ex, ey = hx[scene] + spread, hy[scene] + spread
    cx = rng.uniform(-1, 1, size=tot) * ex
    cy = rng.uniform(-1, 1, size=tot) * ey
    cl = np.stack([cx, cy, h[:, 2]], 1)
    Rl = rotz(yaw)
    Rw = np.einsum('nij,njk->nik', sup_R[scene], Rl)
    cw = np.einsum('nij,nj->ni', sup_R[scene], cl) + sup_t[scene]
    box = np.zeros((tot, 16), np.float64)
    box[:, 0:9] = Rw.reshape(tot, 9)
    box[:, 9:12] = cw
    box[:, 12:15] = h
    return box_off, box.astype(np.float32)


def _support_poses(rng, n):
    """Per-scene world pose of the support: yaw about z, translation
    (U[-1,1], U[-1,1], U[0.4, 1.0])."""
    R = rotz(rng.uniform(0, 2 * np.pi, size=n))
    t = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(0.4, 1.0, n)], 1)
    return R, t


def uniform_batch(n_scenes: int, n_obj: int, n_sph: int, n_cand: int, n_box: int,
                  hx: float, hy: float, seed: int = 0, spread: float = BOX_SPREAD_DEFAULT,
                  side=(0.05, 0.25), rad=(0.01, 0.05), box_half=(0.05, 0.5),
                  inset: float = 0.0, lift: float = 0.0, name: str = "") -> SceneBatch:
    """Every scene: one rectangular support (half extents hx, hy) at a random
    world pose, n_box static cuboids, n_obj objects of n_sph spheres each."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5CE2]))
    sup_R, sup_t = _support_poses(rng, n_scenes)
    sup = _support_rows(sup_R, sup_t, hx, hy, inset, lift)
    obj_off = np.arange(n_scenes + 1, dtype=np.int64) * n_obj
    sph_off, tmpl = _templates(rng, n_scenes * n_obj, n_sph, side, rad)
    perm = _footprint_order(obj_off, sph_off, tmpl)
    sph_off, tmpl = _reorder_objects(perm, sph_off, tmpl)
    obj_sup = np.repeat(np.arange(n_scenes), n_obj)
    box_off, box = _boxes(rng, n_scenes, n_box, hx, hy, spread, sup_R, sup_t, box_half)
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=obj_sup.astype(np.int32),
        obj_ncand=np.full(n_scenes * n_obj, n_cand, np.int32), sup=sup,
        box_off=box_off.astype(np.int32), box=box, name=name,
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand,
                    n_box=n_box, hx=hx, hy=hy, seed=seed, spread=spread))


def uneven_batch(n_scenes: int, seed: int = 0, spread: float = BOX_SPREAD_DEFAULT,
                 n_obj=(5, 60), n_sph=(16, 256), n_cand=(512, 4096), n_box=(4, 32),
                 name: str = "") -> SceneBatch:
    """Uneven workload: per scene N ~ U{5..60} objects, B ~ U{4..32} boxes;
    per object S ~ U{16..256} spheres and C ~ U{512..4096} candidates per
    attempt; the 2.0 x 1.0 m support is scaled by sqrt(N / 20)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x0E7E]))
    N = rng.integers(n_obj[0], n_obj[1] + 1, size=n_scenes)
    B = rng.integers(n_box[0], n_box[1] + 1, size=n_scenes)
    scale = np.sqrt(N / 20.0)
    hx, hy = 1.0 * scale, 0.5 * scale
    sup_R, sup_t = _support_poses(rng, n_scenes)
    sup = _support_rows(sup_R, sup_t, hx, hy, 0.0, 0.0)
    obj_off = np.zeros(n_scenes + 1, np.int64)
    obj_off[1:] = np.cumsum(N)
    n_tot = int(obj_off[-1])
    S = rng.integers(n_sph[0], n_sph[1] + 1, size=n_tot)
    C = rng.integers(n_cand[0], n_cand[1] + 1, size=n_tot)
    sph_off, tmpl = _templates(rng, n_tot, S)
    perm = _footprint_order(obj_off, sph_off, tmpl)
    sph_off, tmpl, C = _reorder_objects(perm, sph_off, tmpl, C)
    obj_sup = np.repeat(np.arange(n_scenes), N)
    box_off, box = _boxes(rng, n_scenes, B, hx, hy, spread, sup_R, sup_t)
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=obj_sup.astype(np.int32),
        obj_ncand=C.astype(np.int32), sup=sup, box_off=box_off.astype(np.int32),
        box=box, name=name, params=dict(n_scenes=n_scenes, seed=seed, spread=spread))


def table_scene(seed: int = 0, spread: float = BOX_SPREAD_DEFAULT) -> SceneBatch:
    """One 1.2 x 0.8 m table; 8 objects x 32 spheres; 256 candidates; 4 boxes."""
    return uniform_batch(1, 8, 32, 256, 4, 0.6, 0.4, seed=seed, spread=spread, name="table-1")


def batched_scenes(n_scenes: int = 4096, seed: int = 0,
                   spread: float = BOX_SPREAD_DEFAULT) -> SceneBatch:
    """4096 scenes on a 2.0 x 1.0 m support; 20 objects x 64 spheres; 1024
    candidates per attempt; 16 static oriented cuboids."""
    return uniform_batch(n_scenes, 20, 64, 1024, 16, 1.0, 0.5, seed=seed, spread=spread,
                         name=f"batched-{n_scenes}")


# ---------------------------------------------------------------------------
# Dense multi-shelf scenes with voxel signed-distance furniture
BAY_GRID_N = 64
BAY_GRID_H = 0.96 / 63             # node spacing (m): 64 nodes span 0.96 m
BAY_GRID_ORIGIN = (-0.48, -0.48, -0.16)
BAY_HALF = (0.4, 0.2)              # shelf surface 0.8 x 0.4 m
BAY_PITCH = 0.40                   # vertical distance between shelf surfaces
# solids of one bay in its own frame (origin at the centre of the board top,
# z up, open towards -y): two boards, two side walls, a back wall
BAY_SOLIDS = [((0.0, 0.0, -0.016), (0.43, 0.23, 0.016)),
              ((0.0, 0.0, 0.316), (0.43, 0.23, 0.016)),
              ((-0.416, 0.0, 0.15), (0.016, 0.23, 0.182)),
              ((0.416, 0.0, 0.15), (0.016, 0.23, 0.182)),
              ((0.0, 0.216, 0.15), (0.43, 0.016, 0.182))]


def bay_sdf_asset() -> np.ndarray:
    """Node values [nz, ny, nx] (x fastest) of the bay's signed distance:
    the minimum over its solids of the axis-aligned box distance, at nodes
    origin + h (i, j, k).  Boards are 2.1 node spacings thick."""
    n, h = BAY_GRID_N, BAY_GRID_H
    o = np.asarray(BAY_GRID_ORIGIN)
    z, y, x = np.meshgrid(o[2] + h * np.arange(n), o[1] + h * np.arange(n),
                          o[0] + h * np.arange(n), indexing="ij")
    p = np.stack([x, y, z], -1)
    best = np.full(x.shape, np.inf)
    for c, hh in BAY_SOLIDS:
        q = np.abs(p - np.asarray(c)) - np.asarray(hh)
        d = np.linalg.norm(np.maximum(q, 0), axis=-1) + np.minimum(q.max(-1), 0)
        best = np.minimum(best, d)
    return best.astype(np.float32)


def shelf_scenes(n_scenes: int = 65536, seed: int = 0, n_obj: int = 100, n_sph: int = 128,
                 n_cand: int = 2048, n_shelves: int = 6, side=(0.03, 0.08),
                 rad=(0.005, 0.02), margin: float = 0.005, chunk: int = 2048) -> SceneBatch:
    """Every scene: a shelf unit of n_shelves stacked 0.8 x 0.4 m surfaces at a
    random world pose (yaw, translation); its furniture is one voxel-SDF grid
    instance per bay (one shared 64^3 asset); n_obj objects of n_sph spheres
    (cube side ~ U(side), radii ~ U(rad)) assigned round-robin to the shelves
    in placement order; objects rest margin + 1 mm above the board (the board
    is part of the field)."""
    lift = margin + 0.001
    n_tot_obj = n_scenes * n_obj
    tmpl = np.empty((n_tot_obj * n_sph, 4), np.float32)
    sph_off = (np.arange(n_tot_obj + 1, dtype=np.int64) * n_sph)
    sup = np.zeros((n_scenes * n_shelves, 16), np.float32)
    grid = np.zeros((n_scenes * n_shelves, 24), np.float32)
    def fill(c0):
        # chunks draw from their own seeded streams and write disjoint rows,
        # so they run on a thread pool with the same result in any order
        c1 = min(n_scenes, c0 + chunk)
        m = c1 - c0
        rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5E1F, c0 // chunk]))
        yaw = rng.uniform(0, 2 * np.pi, m)
        base = np.stack([rng.uniform(-1, 1, m), rng.uniform(-1, 1, m), rng.uniform(0.0, 0.3, m)], 1)
        R = rotz(yaw)
        for k in range(n_shelves):
            t = base + np.einsum('nij,j->ni', R, np.array([0.0, 0.0, BAY_PITCH * k]))
            rows = np.arange(c0, c1) * n_shelves + k
            sup[rows] = _support_rows(R, t, BAY_HALF[0], BAY_HALF[1], 0.0, lift)
            Rt = np.transpose(R, (0, 2, 1))
            grid[rows, 0:9] = Rt.reshape(m, 9)
            grid[rows, 9:12] = -np.einsum('nij,nj->ni', Rt, t)
            grid[rows, 12:15] = BAY_GRID_ORIGIN
            grid[rows, 15] = BAY_GRID_H
            grid[rows, 16:19] = BAY_GRID_N
        so, tm = _templates(rng, m * n_obj, n_sph, side, rad)
        oo = np.arange(m + 1, dtype=np.int64) * n_obj
        perm = _footprint_order(oo, so, tm)
        so, tm = _reorder_objects(perm, so, tm)
        tmpl[c0 * n_obj * n_sph:c1 * n_obj * n_sph] = tm

    starts = range(0, n_scenes, chunk)
    workers = max(1, min(len(starts), 8, os.cpu_count() or 1))
    if workers == 1:
        for c0 in starts:
            fill(c0)
    else:
        with concurrent.futures.ThreadPoolExecutor(workers) as ex:
            list(ex.map(fill, starts))
    obj_sup = (np.repeat(np.arange(n_scenes), n_obj) * n_shelves +
               np.tile(np.arange(n_obj) % n_shelves, n_scenes)).astype(np.int32)
    return SceneBatch(
        obj_off=(np.arange(n_scenes + 1) * n_obj).astype(np.int32),
        sph_off=sph_off.astype(np.int32), tmpl=tmpl, obj_sup=obj_sup,
        obj_ncand=np.full(n_tot_obj, n_cand, np.int32), sup=sup,
        box_off=np.zeros(n_scenes + 1, np.int32), box=np.zeros((0, 16), np.float32),
        grid_off=(np.arange(n_scenes + 1) * n_shelves).astype(np.int32), grid=grid,
        grid_src=np.zeros(n_scenes * n_shelves, np.int32), grid_vals=[bay_sdf_asset()],
        name=f"shelves-{n_scenes}",
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand,
                    n_shelves=n_shelves, seed=seed))


def uneven_shelf_scenes(n_scenes: int = 65536, seed: int = 0, n_obj=(40, 100),
                        n_sph=(64, 128), n_cand=(1024, 2048), chunk: int = 2048) -> SceneBatch:
    """Shelf units as in shelf_scenes with uneven counts: per scene N ~
    U{n_obj} objects (the first N of its round-robin order), per object S ~
    U{n_sph} spheres (the first S of its template) and C ~ U{n_cand}
    candidates per attempt."""
    full = shelf_scenes(n_scenes, seed=seed, n_obj=n_obj[1], n_sph=n_sph[1], n_cand=n_cand[1],
                        chunk=chunk)
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x0E5F]))
    N = rng.integers(n_obj[0], n_obj[1] + 1, size=n_scenes)
    keep = (np.arange(n_obj[1])[None, :] < N[:, None]).ravel()
    objs = np.nonzero(keep)[0]
    S = rng.integers(n_sph[0], n_sph[1] + 1, size=len(objs))
    sidx = _ranges(full.sph_off[objs].astype(np.int64), S)
    sph_off = np.zeros(len(objs) + 1, np.int64)
    sph_off[1:] = np.cumsum(S)
    obj_off = np.zeros(n_scenes + 1, np.int64)
    obj_off[1:] = np.cumsum(N)
    b = dataclasses.replace(
        full, obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=full.tmpl[sidx], obj_sup=full.obj_sup[objs].copy(),
        obj_ncand=rng.integers(n_cand[0], n_cand[1] + 1, size=len(objs)).astype(np.int32),
        name=f"uneven-shelves-{n_scenes}",
        params=dict(full.params, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand))
    return b


# Drawer cabinet (base link frame: x out of the front, z up; metres).  Static
# boards as (centre, half extents); each drawer is a prismatic joint along +x
# at height z_d with its bottom as a support surface and four walls as boxes,
# given in the drawer link frame.
CABINET_BOARDS = (((0.0, 0.31, 0.42), (0.25, 0.01, 0.42)),     # left side
                  ((0.0, -0.31, 0.42), (0.25, 0.01, 0.42)),    # right side
                  ((-0.26, 0.0, 0.42), (0.01, 0.30, 0.42)),    # back
                  ((0.0, 0.0, 0.83), (0.25, 0.30, 0.01)),      # top
                  ((0.0, 0.0, 0.42), (0.25, 0.30, 0.01)),      # middle board
                  ((0.0, 0.0, 0.01), (0.25, 0.30, 0.01)))      # bottom board
DRAWER_Z = (0.05, 0.46)
DRAWER_TRAVEL = (0.0, 0.35)
DRAWER_HALF = (0.21, 0.26)           # support half sizes of a drawer bottom
DRAWER_WALLS = (((0.23, 0.0, 0.09), (0.01, 0.29, 0.09)),      # front panel
                ((-0.22, 0.0, 0.07), (0.01, 0.27, 0.07)),     # back
                ((0.0, 0.27, 0.07), (0.22, 0.01, 0.07)),      # left
                ((0.0, -0.27, 0.07), (0.22, 0.01, 0.07)))     # right


def drawer_scenes(n_scenes: int = 4096, seed: int = 0, n_obj_per_drawer: int = 4,
                  n_sph: int = 32, n_cand: int = 256, side=(0.04, 0.12),
                  rad=(0.01, 0.03)) -> SceneBatch:
    """Every scene: a two-drawer cabinet at a random world pose (yaw about z,
    translation); the drawers are prismatic joints along the cabinet's +x with
    a travel drawn per scene by the forward kinematics; n_obj_per_drawer
    objects of n_sph spheres (cube side ~ U(side), radii ~ U(rad)) go into
    each drawer, resting on its bottom.  The batch's box and support rows of
    the drawers are left zero: they are the forward kinematics' output.
    b.params["art"] holds the articulation: joint_off, joint [n_j][24], base
    [n][12], box_link / box_local, sup_link / sup_local (scenegen layout of
    the scn_joints arrays)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xD2A3]))
    nd = len(DRAWER_Z)
    n_obj = nd * n_obj_per_drawer
    yaw = rng.uniform(0, 2 * np.pi, n_scenes)
    R = rotz(yaw)
    t = np.stack([rng.uniform(-1, 1, n_scenes), rng.uniform(-1, 1, n_scenes),
                  np.zeros(n_scenes)], 1)
    base = np.concatenate([R.reshape(n_scenes, 9), t], 1)
    nb_static, nb_drawer = len(CABINET_BOARDS), len(DRAWER_WALLS)
    B = nb_static + nd * nb_drawer
    box = np.zeros((n_scenes * B, 16), np.float64)
    box_link = -np.ones(n_scenes * B, np.int32)
    box_local = np.zeros((n_scenes * B, 12), np.float64)
    for k, (c, h) in enumerate(CABINET_BOARDS):
        rows = np.arange(n_scenes) * B + k
        box[rows, 0:9] = R.reshape(n_scenes, 9)
        box[rows, 9:12] = np.einsum('nij,j->ni', R, np.asarray(c)) + t
        box[rows, 12:15] = h
    eye = np.eye(3).ravel()
    for d in range(nd):
        for w, (c, h) in enumerate(DRAWER_WALLS):
            rows = np.arange(n_scenes) * B + nb_static + d * nb_drawer + w
            box[rows, 12:15] = h
            box_link[rows] = np.arange(n_scenes) * nd + d
            box_local[rows, 0:9] = eye
            box_local[rows, 9:12] = c
    joint = np.zeros((n_scenes * nd, 24), np.float64)
    for d in range(nd):
        rows = np.arange(n_scenes) * nd + d
        joint[rows, 0] = 0           # prismatic
        joint[rows, 1] = -1          # hangs from the base
        joint[rows, 2:4] = DRAWER_TRAVEL
        joint[rows, 4:7] = (1.0, 0.0, 0.0)
        joint[rows, 8:17] = eye
        joint[rows, 17:20] = (0.0, 0.0, DRAWER_Z[d])
    sup = np.zeros((n_scenes * nd, 16), np.float64)
    sup[:, 12] = DRAWER_HALF[0]
    sup[:, 13] = DRAWER_HALF[1]
    sup_link = np.arange(n_scenes * nd, dtype=np.int32)
    sup_local = np.zeros((n_scenes * nd, 12), np.float64)
    sup_local[:, 0:9] = eye
    sph_off, tmpl = _templates(rng, n_scenes * n_obj, n_sph, side, rad)
    obj_off = np.arange(n_scenes + 1, dtype=np.int64) * n_obj
    perm = _footprint_order(obj_off, sph_off, tmpl)
    sph_off, tmpl = _reorder_objects(perm, sph_off, tmpl)
    obj_sup = (np.repeat(np.arange(n_scenes), n_obj) * nd +
               np.tile(np.arange(n_obj) % nd, n_scenes)).astype(np.int32)
    art = dict(joint_off=(np.arange(n_scenes + 1) * nd).astype(np.int32),
               joint=joint.astype(np.float32), base=base.astype(np.float32),
               box_link=box_link, box_local=box_local.astype(np.float32),
               sup_link=sup_link, sup_local=sup_local.astype(np.float32))
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=obj_sup,
        obj_ncand=np.full(n_scenes * n_obj, n_cand, np.int32), sup=sup.astype(np.float32),
        box_off=(np.arange(n_scenes + 1) * B).astype(np.int32), box=box.astype(np.float32),
        name=f"drawers-{n_scenes}",
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand, seed=seed,
                    art=art))


def relation_scenes(n_scenes: int = 4096, seed: int = 0, n_sph: int = 32, n_cand: int = 256,
                    n_box: int = 4, side=(0.05, 0.15), rad=(0.01, 0.03)) -> SceneBatch:
    """Object-object spatial relations (Sec. IV-F) on a 2.0 x 1.0 m support at
    a random world pose with n_box cuboids; 8 objects per scene, in this
    order (anchors are always earlier objects):
      0  free, ratio_on_support 1 (the projection stays on the support)
      1  'less' than 0.45 m from object 0, within pi/4 of a random direction,
         face_to object 0
      2  'greater' than 0.5 m from object 0, any direction
      3  'equal' to 0.35 +- 0.03 m from object 1, within pi/2 of a random
         direction
      4  'middle' of objects 0, 1 and 2
      5  'less' than 0.3 m from object 4, face_to
      6, 7 free, ratio_on_support 0.5
    Relation rows follow the oracle's layout: kind, anchor count, anchor
    positions, direction, min_r, max_r, angle threshold, flags."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x2E1A]))
    n_obj, hx, hy = 8, 1.0, 0.5
    sup_R, sup_t = _support_poses(rng, n_scenes)
    sup = _support_rows(sup_R, sup_t, hx, hy, 0.0, 0.0)
    obj_off = np.arange(n_scenes + 1, dtype=np.int64) * n_obj
    sph_off, tmpl = _templates(rng, n_scenes * n_obj, n_sph, side, rad)
    box_off, box = _boxes(rng, n_scenes, n_box, hx, hy, 0.5, sup_R, sup_t, half=(0.05, 0.2))
    rel = np.zeros((n_scenes, 5, 16), np.float64)
    ang = rng.uniform(0, 2 * np.pi, size=(n_scenes, 2))
    inf = np.inf
    spec = [  # (object, kind, anchors, direction index or -1, min_r, max_r, theta, face_to)
        (1, 1, [0], 0, 0.0, 0.45, np.pi / 4, 1),
        (2, 1, [0], -1, 0.5, inf, np.pi, 0),
        (3, 1, [1], 1, 0.32, 0.38, np.pi / 2, 0),
        (4, 2, [0, 1, 2], -1, 0.0, 0.0, np.pi, 0),
        (5, 1, [4], -1, 0.0, 0.3, np.pi, 1),
    ]
    obj_rel = -np.ones(n_scenes * n_obj, np.int32)
    for k, (o, kind, anc, di, r0, r1, th, ft) in enumerate(spec):
        rel[:, k, 0] = kind
        rel[:, k, 1] = len(anc)
        rel[:, k, 2:2 + len(anc)] = anc
        if di >= 0:
            rel[:, k, 10] = np.cos(ang[:, di])
            rel[:, k, 11] = np.sin(ang[:, di])
        rel[:, k, 12], rel[:, k, 13], rel[:, k, 14], rel[:, k, 15] = r0, r1, th, ft
        obj_rel[np.arange(n_scenes) * n_obj + o] = np.arange(n_scenes) * 5 + k
    ratio = np.zeros(n_scenes * n_obj, np.float32)
    ratio[np.arange(n_scenes) * n_obj] = 1.0
    ratio[np.arange(n_scenes) * n_obj + 6] = 0.5
    ratio[np.arange(n_scenes) * n_obj + 7] = 0.5
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=np.repeat(np.arange(n_scenes), n_obj).astype(np.int32),
        obj_ncand=np.full(n_scenes * n_obj, n_cand, np.int32), sup=sup,
        box_off=box_off.astype(np.int32), box=box, obj_rel=obj_rel,
        rel=rel.reshape(-1, 16).astype(np.float32), obj_ratio=ratio,
        name=f"relations-{n_scenes}",
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand, seed=seed))


# Synthetic reachability map of a 6-axis arm (no robot model is available):
# axes (z*, theta, x*, y*) of the base-symmetric parametrization, with the
# reachable shell of a shoulder 0.35 m above the base (0.25 .. 0.80 m, the
# outer radius shrinking by 0.15 m towards side approaches), a floor 0.25 m
# below the base and a wrist limit x* >= -0.15 m (the object's x axis may not
# point back at the base by much).  Values at the cell centres.
REACH_LO = (-0.3, -np.pi / 32, -1.0, -1.0)     # approach angles 0, pi/16, ... at cell centres
REACH_H = (0.05, np.pi / 16, 1.0 / 32, 1.0 / 32)
REACH_DIMS = (24, 9, 64, 64)


def reach_map():
    c = [REACH_LO[a] + REACH_H[a] * (np.arange(REACH_DIMS[a]) + 0.5) for a in range(4)]
    z, th, x, y = np.meshgrid(*c, indexing="ij")
    rho = np.sqrt(x * x + y * y + (z - 0.35) ** 2)
    ok = (rho >= 0.25) & (rho <= 0.80 - 0.15 * th / (np.pi / 2)) & (z >= -0.25) & (x >= -0.15)
    geom = np.array(list(REACH_LO) + list(REACH_H) + list(REACH_DIMS), np.float32)
    return ok.astype(np.uint8), geom


def reach_scenes(n_scenes: int = 4096, seed: int = 0, n_obj: int = 8, n_sph: int = 32,
                 n_cand: int = 256, n_box: int = 4, side=(0.05, 0.15),
                 rad=(0.01, 0.03)) -> SceneBatch:
    """Robot-manipulation tables (Sec. IV-E): a 1.2 x 0.8 m support at a
    random world pose with n_box cuboids and a robot base 0.15 m off the
    middle of its near long edge, 0.2 m below the top, facing across the
    table; every object must be reachable, objects 0..5 from above
    (approach angle 0), the rest at 45 degrees."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x2EAC]))
    hx, hy = 0.6, 0.4
    sup_R, sup_t = _support_poses(rng, n_scenes)
    sup = _support_rows(sup_R, sup_t, hx, hy, 0.0, 0.0)
    obj_off = np.arange(n_scenes + 1, dtype=np.int64) * n_obj
    sph_off, tmpl = _templates(rng, n_scenes * n_obj, n_sph, side, rad)
    perm = _footprint_order(obj_off, sph_off, tmpl)
    sph_off, tmpl = _reorder_objects(perm, sph_off, tmpl)
    box_off, box = _boxes(rng, n_scenes, n_box, hx, hy, 0.5, sup_R, sup_t, half=(0.05, 0.2))
    Rb = np.einsum('nij,jk->nik', sup_R, rotz(np.array(np.pi / 2)))
    tb = np.einsum('nij,j->ni', sup_R, np.array([0.0, -hy - 0.15, -0.2])) + sup_t
    robot = np.concatenate([Rb.reshape(n_scenes, 9), tb], 1).astype(np.float32)
    reach = np.tile(np.array([0.0] * 6 + [np.pi / 4] * (n_obj - 6), np.float32), n_scenes)
    m, geom = reach_map()
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=np.repeat(np.arange(n_scenes), n_obj).astype(np.int32),
        obj_ncand=np.full(n_scenes * n_obj, n_cand, np.int32), sup=sup,
        box_off=box_off.astype(np.int32), box=box, robot=robot, obj_reach=reach, reach_map=m,
        reach_geom=geom, name=f"reach-{n_scenes}",
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand, seed=seed))


def face_down_rotations() -> np.ndarray:
    """The 6 rotations (object frame -> resting frame) that turn the outward
    normal of one face of an axis-aligned box (+x, -x, +y, -y, +z, -z, in
    this order) to -z: the box resting on that face."""
    def rx(a):
        c, s = np.cos(a), np.sin(a)
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])

    def ry(a):
        c, s = np.cos(a), np.sin(a)
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    R = np.stack([ry(np.pi / 2), ry(-np.pi / 2), rx(-np.pi / 2), rx(np.pi / 2), rx(np.pi),
                  np.eye(3)])
    return np.round(R, 15)


def haar_rotations(rng, n: int) -> np.ndarray:
    """n rotations uniform on SO(3) (normalised Gaussian quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def stable_rows(R: np.ndarray, weights) -> np.ndarray:
    """Stable-pose table rows [K,12]: R[9], cumulative weight (last 1), 0, 0."""
    w = np.asarray(weights, np.float64)
    cum = np.cumsum(w / w.sum())
    cum[-1] = 1.0
    rows = np.zeros((len(w), 12), np.float32)
    rows[:, :9] = np.asarray(R).reshape(-1, 9)
    rows[:, 9] = cum
    return rows


def stable_scenes(n_scenes: int = 4096, seed: int = 0, n_obj: int = 12, n_sph: int = 32,
                  n_cand: int = 256, n_box: int = 6, n_free: int = 12,
                  side=(0.05, 0.20), rad=(0.01, 0.04)) -> SceneBatch:
    """Objects with stable poses (Sec. III "Main algorithm": orientations from
    rules or from stable poses): a 1.6 x 1.0 m support at a random world pose
    with n_box cuboids; of every three objects one turns about z only, one
    rests on a face of its sphere set's bounding box (6 rows, weight = the
    face's area), one takes one of n_free rotations uniform on SO(3) (equal
    weights), each followed by the random rotation about z."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x57AB]))
    hx, hy = 0.8, 0.5
    sup_R, sup_t = _support_poses(rng, n_scenes)
    sup = _support_rows(sup_R, sup_t, hx, hy, 0.0, 0.0)
    obj_off = np.arange(n_scenes + 1, dtype=np.int64) * n_obj
    sph_off, tmpl = _templates(rng, n_scenes * n_obj, n_sph, side, rad)
    perm = _footprint_order(obj_off, sph_off, tmpl)
    sph_off, tmpl = _reorder_objects(perm, sph_off, tmpl)
    box_off, box = _boxes(rng, n_scenes, n_box, hx, hy, 0.5, sup_R, sup_t, half=(0.05, 0.25))
    n_o = n_scenes * n_obj
    kind = np.arange(n_o) % 3
    t = tmpl.astype(np.float64)
    starts = sph_off[:-1].astype(np.int64)
    ext = (np.maximum.reduceat(t[:, :3] + t[:, 3:4], starts, axis=0)
           - np.minimum.reduceat(t[:, :3] - t[:, 3:4], starts, axis=0))
    counts = np.where(kind == 0, 0, np.where(kind == 1, 6, n_free)).astype(np.int64)
    pose_off = np.zeros(n_o + 1, np.int64)
    pose_off[1:] = np.cumsum(counts)
    rows = np.zeros((int(pose_off[-1]), 12), np.float32)
    # face rows: weights are the face areas, cumulative per object
    f = np.nonzero(kind == 1)[0]
    e = ext[f]
    area = np.stack([e[:, 1] * e[:, 2]] * 2 + [e[:, 0] * e[:, 2]] * 2 + [e[:, 0] * e[:, 1]] * 2, 1)
    cum = np.cumsum(area / area.sum(1, keepdims=True), 1)
    cum[:, -1] = 1.0
    fr = pose_off[f][:, None] + np.arange(6)
    rows[fr, :9] = face_down_rotations().reshape(6, 9)
    rows[fr, 9] = cum
    # free rows: uniform on SO(3), equal weights
    g = np.nonzero(kind == 2)[0]
    gr = (pose_off[g][:, None] + np.arange(n_free)).ravel()
    rows[gr, :9] = haar_rotations(rng, len(gr)).reshape(-1, 9)
    cg = np.arange(1, n_free + 1) / n_free
    cg[-1] = 1.0
    rows[gr, 9] = np.tile(cg, len(g))
    return SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=tmpl.astype(np.float32), obj_sup=np.repeat(np.arange(n_scenes), n_obj).astype(np.int32),
        obj_ncand=np.full(n_o, n_cand, np.int32), sup=sup,
        box_off=box_off.astype(np.int32), box=box, obj_pose_off=pose_off.astype(np.int32),
        stable=rows, name=f"stable-{n_scenes}",
        params=dict(n_scenes=n_scenes, n_obj=n_obj, n_sph=n_sph, n_cand=n_cand, seed=seed))


def subset(b: SceneBatch, scenes) -> tuple[SceneBatch, np.ndarray]:
    """The scenes `scenes` of a batch as a batch of their own, plus the
    original scene indices (which the random-number counters must keep)."""
    scenes = np.asarray(scenes, np.int64)
    objs = _ranges(b.obj_off[scenes], b.obj_off[scenes + 1] - b.obj_off[scenes])
    boxes = _ranges(b.box_off[scenes], b.box_off[scenes + 1] - b.box_off[scenes])
    obj_off = np.zeros(len(scenes) + 1, np.int64)
    obj_off[1:] = np.cumsum(b.obj_off[scenes + 1] - b.obj_off[scenes])
    box_off = np.zeros(len(scenes) + 1, np.int64)
    box_off[1:] = np.cumsum(b.box_off[scenes + 1] - b.box_off[scenes])
    S = (b.sph_off[objs + 1] - b.sph_off[objs]).astype(np.int64)
    sph_off = np.zeros(len(objs) + 1, np.int64)
    sph_off[1:] = np.cumsum(S)
    sidx = _ranges(b.sph_off[objs], S)
    sups = np.unique(b.obj_sup[objs])
    remap = -np.ones(b.sup.shape[0], np.int64)
    remap[sups] = np.arange(len(sups))
    out = SceneBatch(
        obj_off=obj_off.astype(np.int32), sph_off=sph_off.astype(np.int32),
        tmpl=b.tmpl[sidx].copy(), obj_sup=remap[b.obj_sup[objs]].astype(np.int32),
        obj_ncand=b.obj_ncand[objs].copy(), sup=b.sup[sups].copy(),
        box_off=box_off.astype(np.int32), box=b.box[boxes].copy(),
        name=b.name + "-subset", params=dict(b.params))
    if b.obj_rel is not None:
        out.obj_rel = b.obj_rel[objs].copy()
        out.rel = b.rel
    if b.obj_ratio is not None:
        out.obj_ratio = b.obj_ratio[objs].copy()
    if b.robot is not None:
        out.robot = b.robot[scenes].copy()
        out.obj_reach = b.obj_reach[objs].copy()
        out.reach_map, out.reach_geom = b.reach_map, b.reach_geom
    if b.obj_pose_off is not None:
        cnt = (b.obj_pose_off[objs + 1] - b.obj_pose_off[objs]).astype(np.int64)
        poff = np.zeros(len(objs) + 1, np.int64)
        poff[1:] = np.cumsum(cnt)
        out.obj_pose_off = poff.astype(np.int32)
        out.stable = b.stable[_ranges(b.obj_pose_off[objs], cnt)].copy()
    if b.grid_off is not None:
        grids = _ranges(b.grid_off[scenes], b.grid_off[scenes + 1] - b.grid_off[scenes])
        goff = np.zeros(len(scenes) + 1, np.int64)
        goff[1:] = np.cumsum(b.grid_off[scenes + 1] - b.grid_off[scenes])
        out.grid_off = goff.astype(np.int32)
        out.grid = b.grid[grids].copy()
        out.grid_src = b.grid_src[grids].copy()
        out.grid_vals = b.grid_vals
    return out, scenes.astype(np.int32)


def random_poses(rng, n: int, hx: float, hy: float, z=(0.0, 0.3)):
    """Arbitrary candidate poses (support frame) for checker tests."""
    x = rng.uniform(-hx, hx, n)
    y = rng.uniform(-hy, hy, n)
    zz = rng.uniform(z[0], z[1], n)
    yaw = rng.uniform(0, 2 * math.pi, n)
    return [a.astype(np.float32) for a in (x, y, zz, yaw)]
