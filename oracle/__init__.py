"""FP64 CPU oracle for batched rejection-sampling placement (test infrastructure).

Only tests/, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg
may import this package.  The product path (the HIP library and its binding)
never does.  The C part (oracle.c) is compiled with gcc into liboracle.so; it
shares no code with the GPU path.

Parity notes for each function are in the C source and in the tests that pin
them (Philox known-answer vectors, box-SDF and sphere-distance closed forms,
rigid-motion invariance, brute force on tiny scenes).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "fk.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c -> liboracle.so (plain -O2, IEEE FP64, OpenMP over scenes)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, *_SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Batch(C.Structure):
    _fields_ = [("n_scenes", C.c_int),
                ("obj_off", C.c_void_p), ("sph_off", C.c_void_p), ("tmpl", C.c_void_p),
                ("obj_sup", C.c_void_p), ("obj_ncand", C.c_void_p), ("sup", C.c_void_p),
                ("box_off", C.c_void_p), ("box", C.c_void_p),
                ("grid_off", C.c_void_p), ("grid", C.c_void_p), ("grid_src", C.c_void_p),
                ("grid_val", C.c_void_p), ("scene_id", C.c_void_p),
                ("obj_rel", C.c_void_p), ("rel", C.c_void_p), ("obj_ratio", C.c_void_p),
                ("robot", C.c_void_p), ("obj_reach", C.c_void_p), ("reach_map", C.c_void_p),
                ("reach_geom", C.c_void_p), ("obj_pose_off", C.c_void_p), ("stable", C.c_void_p)]


class _GenArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("margin", C.c_double), ("retries", C.c_int),
                ("default_ncand", C.c_int), ("band", C.c_double), ("max_steps", C.c_int),
                ("early_exit", C.c_int), ("band_region", C.c_double)]


class _GenOut(C.Structure):
    _fields_ = [("status", C.c_void_p), ("n_placed", C.c_void_p),
                ("rec_attempt", C.c_void_p), ("rec_idx", C.c_void_p),
                ("rec_pose", C.c_void_p), ("rec_stable", C.c_void_p), ("rec_banded", C.c_void_p),
                ("rec_clear", C.c_void_p), ("placed", C.c_void_p), ("n_cand", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_u01.argtypes = [C.c_uint32]
        L.orc_u01.restype = C.c_double
        L.orc_box_sdf.argtypes = [C.c_void_p] * 4
        L.orc_box_sdf.restype = C.c_double
        L.orc_grid_sample.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.orc_grid_sample.restype = C.c_double
        L.orc_sample_poses.argtypes = [C.POINTER(_Batch), C.c_void_p, C.c_void_p, C.c_uint64,
                                       C.c_int] + [C.c_void_p] * 5
        L.orc_check.argtypes = [C.POINTER(_Batch)] + [C.c_void_p] * 10
        L.orc_generate.argtypes = [C.POINTER(_Batch), C.POINTER(_GenArgs), C.POINTER(_GenOut)]
        L.orc_fk_links.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_uint64, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_fk_rows.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_reach_query.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_sample_relation.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                          C.c_void_p, C.c_double, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data if a is not None else None


class _Keep:
    """Holds the FP64 / int32 copies a ctypes batch points into."""

    def __init__(self, b, scene_id=None):
        self.obj_off = np.ascontiguousarray(b.obj_off, np.int32)
        self.sph_off = np.ascontiguousarray(b.sph_off, np.int32)
        self.tmpl = np.ascontiguousarray(b.tmpl, np.float64)
        self.obj_sup = np.ascontiguousarray(b.obj_sup, np.int32)
        self.obj_ncand = np.ascontiguousarray(b.obj_ncand, np.int32)
        self.sup = np.ascontiguousarray(b.sup, np.float64)
        self.box_off = np.ascontiguousarray(b.box_off, np.int32)
        self.box = np.ascontiguousarray(b.box, np.float64).reshape(-1, 16)
        self.scene_id = None if scene_id is None else np.ascontiguousarray(scene_id, np.int32)
        self.grid_off = self.grid = self.grid_src = self.grid_ptrs = None
        self._vals = None
        if getattr(b, "grid_off", None) is not None:
            self.grid_off = np.ascontiguousarray(b.grid_off, np.int32)
            self.grid = np.ascontiguousarray(b.grid, np.float64).reshape(-1, 24)
            self.grid_src = np.ascontiguousarray(b.grid_src, np.int32)
            self._vals = [np.ascontiguousarray(v, np.float32) for v in b.grid_vals]
            self.grid_ptrs = (C.c_void_p * len(self._vals))(*[v.ctypes.data for v in self._vals])
        rel = getattr(b, "obj_rel", None)
        self.obj_rel = None if rel is None else np.ascontiguousarray(rel, np.int32)
        self.rel = None if rel is None else np.ascontiguousarray(b.rel, np.float64).reshape(-1, 16)
        ratio = getattr(b, "obj_ratio", None)
        self.obj_ratio = None if ratio is None else np.ascontiguousarray(ratio, np.float64)
        self.robot = self.obj_reach = self.reach_map = self.reach_geom = None
        if getattr(b, "robot", None) is not None:
            self.robot = np.ascontiguousarray(b.robot, np.float64).reshape(-1, 12)
            self.obj_reach = np.ascontiguousarray(b.obj_reach, np.float64)
            self.reach_map = np.ascontiguousarray(b.reach_map, np.uint8)
            self.reach_geom = np.ascontiguousarray(b.reach_geom, np.float64)
        self.obj_pose_off = self.stable = None
        if getattr(b, "obj_pose_off", None) is not None:
            self.obj_pose_off = np.ascontiguousarray(b.obj_pose_off, np.int32)
            self.stable = np.ascontiguousarray(b.stable, np.float64).reshape(-1, 12)
        self.cb = _Batch(int(len(self.obj_off) - 1), _p(self.obj_off), _p(self.sph_off),
                         _p(self.tmpl), _p(self.obj_sup), _p(self.obj_ncand), _p(self.sup),
                         _p(self.box_off), _p(self.box), _p(self.grid_off), _p(self.grid),
                         _p(self.grid_src),
                         C.cast(self.grid_ptrs, C.c_void_p) if self.grid_ptrs is not None else None,
                         _p(self.scene_id), _p(self.obj_rel), _p(self.rel), _p(self.obj_ratio),
                         _p(self.robot), _p(self.obj_reach), _p(self.reach_map),
                         _p(self.reach_geom), _p(self.obj_pose_off), _p(self.stable))


# ---------------------------------------------------------------------------
def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def u01(w: int) -> float:
    return float(lib().orc_u01(int(w) & 0xFFFFFFFF))


def box_sdf(R, c, h, p) -> float:
    R = np.ascontiguousarray(R, np.float64).reshape(9)
    c = np.ascontiguousarray(c, np.float64)
    h = np.ascontiguousarray(h, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    return float(lib().orc_box_sdf(_p(R), _p(c), _p(h), _p(p)))


def grid_sample(vals, origin, h, pg) -> float:
    v = np.ascontiguousarray(vals, np.float32)
    dims = np.array([v.shape[2], v.shape[1], v.shape[0]], np.int32)
    o = np.ascontiguousarray(origin, np.float64)
    pg = np.ascontiguousarray(pg, np.float64)
    return float(lib().orc_grid_sample(_p(v), _p(dims), _p(o), float(h), _p(pg)))


def sample_poses(b, obj_idx, cand_off, seed: int, attempt: int, scene_id=None,
                 with_stable: bool = False):
    """Candidate poses (x, y, z, yaw) in the support frame; with_stable also
    returns each candidate's stable-pose row (-1: none)."""
    K = _Keep(b, scene_id)
    oi = np.ascontiguousarray(obj_idx, np.int32)
    co = np.ascontiguousarray(cand_off, np.int32)
    tot = int(co[-1])
    out = [np.zeros(tot, np.float64) for _ in range(4)]
    kk = np.zeros(tot, np.int32)
    lib().orc_sample_poses(C.byref(K.cb), _p(oi), _p(co), C.c_uint64(seed), int(attempt),
                           *[_p(a) for a in out], _p(kk))
    return out + [kk] if with_stable else out


def check(b, obj_idx, cand_off, n_placed, placed, poses, scene_id=None) -> np.ndarray:
    """Clearance of each candidate pose (support frame) of object obj_idx[s]
    against scene s's boxes/grids and its first n_placed[s] objects.  poses:
    (x, y, z, yaw) or (x, y, z, yaw, stable row)."""
    K = _Keep(b, scene_id)
    oi = np.ascontiguousarray(obj_idx, np.int32)
    co = np.ascontiguousarray(cand_off, np.int32)
    npl = np.ascontiguousarray(n_placed, np.int32)
    pl = np.ascontiguousarray(placed, np.float64).reshape(-1, 4)
    ps = [np.ascontiguousarray(a, np.float64) for a in poses[:4]]
    kk = np.ascontiguousarray(poses[4], np.int32) if len(poses) > 4 else None
    clr = np.zeros(int(co[-1]), np.float64)
    lib().orc_check(C.byref(K.cb), _p(oi), _p(co), _p(npl), _p(pl), *[_p(a) for a in ps],
                    _p(kk), _p(clr))
    return clr


def generate(b, seed: int, margin: float = 0.005, retries: int = 10, default_ncand: int = 1024,
             band: float = 1e-5, max_steps: int = 0, scene_id=None, threads=None,
             early_exit: bool = False, band_region: float = 1e-6) -> dict:
    """Batched rejection-sampling placement; returns per-scene status
    (1 valid, 2 invalid), per-object chosen (attempt, idx), poses, band flags,
    and the world spheres of the placed objects.  early_exit: stop each
    candidate's clearance at its first term below margin - band (same
    results; for replaying large scenes in tests)."""
    if threads is not None:
        set_threads(threads)
    K = _Keep(b, scene_id)
    n, n_obj, n_sph = K.cb.n_scenes, len(K.sph_off) - 1, K.tmpl.shape[0]
    out = dict(status=np.zeros(n, np.int8), n_placed=np.zeros(n, np.int32),
               rec_attempt=np.zeros(n_obj, np.int32), rec_idx=np.zeros(n_obj, np.int32),
               rec_pose=np.zeros((n_obj, 4), np.float64), rec_stable=np.zeros(n_obj, np.int32),
               rec_banded=np.zeros(n_obj, np.int8),
               rec_clear=np.zeros(n_obj, np.float64),
               placed=np.full((n_sph, 4), np.nan, np.float64), n_cand=np.zeros(n, np.int64))
    go = _GenOut(*[_p(out[k]) for k in ("status", "n_placed", "rec_attempt", "rec_idx",
                                         "rec_pose", "rec_stable", "rec_banded", "rec_clear",
                                         "placed",
                                         "n_cand")])
    ga = _GenArgs(int(seed), float(margin), int(retries), int(default_ncand), float(band),
                  int(max_steps), int(bool(early_exit)), float(band_region))
    lib().orc_generate(C.byref(K.cb), C.byref(ga), C.byref(go))
    return out


# ---------------------------------------------------------------------------
def forward_kinematics(joint_off, joint, base, seed: int = 0, q=None, scene_id=None,
                       rows=()):
    """Batched forward kinematics (fk.c): joint values (sampled from seed when
    q is None), world link poses [n_joints][12], and for every (rows [n][16],
    row_link [n], local [n][12]) in `rows` the rows with their linked entries
    moved (FP64 copies).  Returns (q, link, [moved rows...])."""
    jo = np.ascontiguousarray(joint_off, np.int32)
    J = np.ascontiguousarray(joint, np.float64).reshape(-1, 24)
    B = np.ascontiguousarray(base, np.float64).reshape(-1, 12)
    n = int(len(jo) - 1)
    nj = int(J.shape[0])
    sid = None if scene_id is None else np.ascontiguousarray(scene_id, np.int32)
    qq = np.zeros(nj, np.float64) if q is None else np.array(q, np.float64)
    link = np.zeros((max(nj, 1), 12), np.float64)
    lib().orc_fk_links(n, _p(jo), _p(J), _p(B), _p(sid), C.c_uint64(seed), int(q is None),
                       _p(qq), _p(link))
    moved = []
    for table, row_link, local in rows:
        R = np.array(table, np.float64).reshape(-1, 16).copy()
        rl = np.ascontiguousarray(row_link, np.int32)
        Lc = np.ascontiguousarray(local, np.float64).reshape(-1, 12)
        lib().orc_fk_rows(int(R.shape[0]), _p(rl), _p(Lc), _p(link), _p(R))
        moved.append(R)
    return qq, link[:nj], moved


def sample_relation(rel, anchors, ax: float, ay: float, words, band: float = 1e-6):
    """One sample of a spatial relation (oracle.c sample_relation): returns
    (x, y, yaw, inside, banded) for the four Philox words of a candidate."""
    r = np.ascontiguousarray(rel, np.float64)
    a = np.ascontiguousarray(anchors, np.float64).reshape(-1, 2)
    w = np.ascontiguousarray(words, np.uint32)
    out = np.zeros(5, np.float64)
    lib().orc_sample_relation(_p(r), _p(a), float(ax), float(ay), _p(w), float(band), _p(out))
    return out[0], out[1], out[2], bool(out[3]), bool(out[4])


def relation_row(kind: int, anchors, v=(0.0, 0.0), min_r=0.0, max_r=np.inf, theta=np.pi,
                 face_to=False) -> np.ndarray:
    """A relation row in the layout sample_relation reads (16 floats)."""
    row = np.zeros(16, np.float64)
    row[0], row[1] = kind, len(anchors)
    row[2:2 + len(anchors)] = anchors
    row[10:12] = v
    row[12], row[13], row[14] = min_r, max_r, theta
    row[15] = 1.0 if face_to else 0.0
    return row


def reach_query(reach_map, geom, robot, pose, theta, band: float = 1e-6):
    """Batched reachability queries (oracle.c reachable): object-frame world
    poses [n][12], robot base poses [n][12], approach angles [n] ->
    (reachable [n] bool, banded [n] bool)."""
    m = np.ascontiguousarray(reach_map, np.uint8)
    g = np.ascontiguousarray(geom, np.float64)
    r = np.ascontiguousarray(robot, np.float64).reshape(-1, 12)
    P = np.ascontiguousarray(pose, np.float64).reshape(-1, 12)
    th = np.ascontiguousarray(theta, np.float64)
    n = int(P.shape[0])
    out = np.zeros(n, np.int8)
    bd = np.zeros(n, np.int8)
    lib().orc_reach_query(n, _p(m), _p(g), _p(r), _p(P), _p(th), float(band), _p(out), _p(bd))
    return out.astype(bool), bd.astype(bool)
