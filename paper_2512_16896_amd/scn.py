"""ctypes binding of libscn.so (include/scn.h).  Argument marshalling only.

Every step of the hot path runs in the HIP kernels of libscn.so; this module
turns torch tensors (device memory) and Python scalars into the C structs of
the ABI.  If the library is missing the import fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libscn.so")

SCN_OK = 0
SCN_E_INVALID_ARG, SCN_E_HIP, SCN_E_CAPACITY, SCN_E_NO_DEVICE, SCN_E_UNSUPPORTED, \
    SCN_E_NONFINITE = -1, -2, -3, -4, -5, -6
ACTIVE, VALID, INVALID = 0, 1, 2
# workspace kinds (scn_workspace_bytes)
WS_GENERATE, WS_MLP_FORWARD, WS_MLP_BACKWARD, WS_MLP_TRAIN, WS_GENERATE_LEARNED = 0, 1, 2, 3, 4


class ScnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libscn error {code}: {msg}")
        self.code = code


class PoseRec(C.Structure):
    _fields_ = [("x", C.c_float), ("y", C.c_float), ("z", C.c_float), ("yaw", C.c_float),
                ("attempt", C.c_int32), ("idx", C.c_int32)]


class _ReachMap(C.Structure):
    _fields_ = [("map", C.c_void_p), ("lo", C.c_float * 4), ("h", C.c_float * 4),
                ("dims", C.c_int32 * 4)]


class _Batch(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "n_scenes", "n_objects", "n_spheres", "n_supports", "n_boxes", "n_grids", "n_grid_assets",
        "max_objects_per_scene", "max_spheres_per_object", "max_spheres_per_scene",
        "max_boxes_per_scene", "max_grids_per_scene", "max_cand_per_object", "geometry")] + \
        [(n, C.c_void_p) for n in (
            "obj_off", "sph_off", "tmpl", "obj_sup", "obj_ncand", "sup", "box_off", "box",
            "grid_off", "grid", "grid_src", "grid_val_off", "grid_val",
            "placed", "n_placed", "status", "rec", "obj_rel", "rel", "obj_ratio", "robot",
            "obj_reach")] + [("reach", _ReachMap)] + \
        [(n, C.c_void_p) for n in ("obj_pose_off", "stable", "rec_stable")]


class _Joints(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("n_joints", C.c_int32), ("joint_off", C.c_void_p),
                ("joint", C.c_void_p), ("base", C.c_void_p)]


class _Poses(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("yaw", C.c_void_p),
                ("stable", C.c_void_p)]


class _GenArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("margin", C.c_float), ("retries", C.c_int32),
                ("default_ncand", C.c_int32), ("max_steps", C.c_int32),
                ("schedule", C.c_int32), ("use_graph", C.c_int32),
                ("fallback_chunk", C.c_int32), ("wide_schedule", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class Counters(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "candidates", "sphere_pairs", "box_pairs", "grid_samples", "attempts", "placed",
        "error_word", "transforms", "box_culls", "object_culls", "valid_scenes",
        "invalid_scenes", "sphere_culls", "nonfinite", "check_refined")] + \
        [("reserved", C.c_int64 * 1)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_ if n != "reserved"}


N_LAYERS = 4
FEATURES, BINS, DESC, HMAP_CELLS = 4128, 4096, 32, 4096


class Mlp(C.Structure):
    _fields_ = [("dims", C.c_int32 * (N_LAYERS + 1))] + \
        [(n, C.c_void_p * N_LAYERS) for n in ("w", "b", "wb", "wt", "m_w", "v_w", "m_b", "v_b")] + \
        [("step", C.c_int64)]


class AdamW(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2512_16896_amd.build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, u64, f32 = C.c_void_p, C.c_int32, C.c_uint64, C.c_float
    sigs = {
        "scn_ctx_create": [C.POINTER(vp), C.c_int],
        "scn_ctx_destroy": [vp],
        "scn_workspace_bytes": [C.c_int, vp, vp, i32, i32, C.POINTER(C.c_size_t)],
        "scn_set_workspace": [vp, vp, C.c_size_t],
        "scn_reset_counters": [vp, vp],
        "scn_read_counters": [vp, C.POINTER(Counters), vp],
        "scn_sample_poses": [vp, C.POINTER(_Batch), vp, vp, i32, i32, u64, i32, _Poses, vp],
        "scn_check_batch": [vp, C.POINTER(_Batch), vp, vp, i32, i32, _Poses, f32, vp, vp, vp],
        "scn_reset_scenes": [vp, C.POINTER(_Batch), vp],
        "scn_place_step": [vp, C.POINTER(_Batch), C.POINTER(_GenArgs), vp, vp],
        "scn_generate_scenes": [vp, C.POINTER(_Batch), C.POINTER(_GenArgs), vp],
        "scn_generate_scenes_noalloc": [vp, C.POINTER(_Batch), C.POINTER(_GenArgs), vp],
        "scn_forward_kinematics": [vp, C.POINTER(_Joints), u64, i32, vp, vp, i32, vp, vp, vp,
                                   i32, vp, vp, vp, vp],
        "scn_reach_query": [vp, C.POINTER(_ReachMap), i32, vp, vp, vp, vp, vp],
        "scn_autotune": [vp, C.POINTER(_Batch), C.POINTER(_GenArgs), C.POINTER(C.c_int32),
                         C.POINTER(C.c_float), vp],
        "scn_autotune_save": [vp, C.c_char_p],
        "scn_autotune_load": [vp, C.c_char_p],
        "scn_mlp_init": [vp, C.POINTER(Mlp), u64, vp],
        "scn_mlp_forward": [vp, C.POINTER(Mlp), vp, i32, vp, vp],
        "scn_mlp_backward": [vp, C.POINTER(Mlp), vp, i32, vp, vp, i32, vp, vp, vp, vp],
        "scn_mlp_train_step": [vp, C.POINTER(Mlp), vp, i32, vp, vp, i32, C.POINTER(AdamW), vp, vp],
        "scn_descriptors": [vp, C.POINTER(_Batch), vp, vp],
        "scn_heightmaps": [vp, C.POINTER(_Batch), vp, vp, vp],
        "scn_features": [vp, C.POINTER(_Batch), i32, vp, vp, vp, vp, vp],
        "scn_proposal_topk": [vp, vp, i32, i32, vp, vp, vp],
        "scn_harvest_labels": [vp, C.POINTER(_Batch), vp, i32, u64, i32, f32, vp, vp, vp],
        "scn_generate_scenes_learned": [vp, C.POINTER(_Batch), C.POINTER(_GenArgs),
                                        C.POINTER(Mlp), i32, vp],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.scn_last_error.restype = C.c_char_p
    L.scn_status_string.restype = C.c_char_p
    L.scn_status_string.argtypes = [C.c_int]
    return L


_lib = _load()

# names of the C ABI entry points (what include/scn.h declares)
EXPORTS = ("scn_ctx_create", "scn_ctx_destroy", "scn_status_string", "scn_last_error",
           "scn_workspace_bytes", "scn_set_workspace", "scn_reset_counters",
           "scn_read_counters", "scn_sample_poses", "scn_check_batch",
           "scn_reset_scenes", "scn_place_step", "scn_generate_scenes",
           "scn_generate_scenes_noalloc", "scn_forward_kinematics", "scn_reach_query",
           "scn_autotune",
           "scn_autotune_save", "scn_autotune_load", "scn_mlp_init", "scn_mlp_forward",
           "scn_mlp_backward", "scn_mlp_train_step", "scn_descriptors", "scn_heightmaps",
           "scn_features", "scn_proposal_topk", "scn_harvest_labels",
           "scn_generate_scenes_learned")

SCHED_LONGEST_FIRST = 0x20
# the library's schedule when none is given and none is tuned (scn.h):
# 4 waves, batch order, placed spheres from global memory
DEFAULT_SCHEDULE = 0xF04


def lib():
    return _lib


def _ok(code: int):
    if code != SCN_OK:
        raise ScnError(code, (_lib.scn_last_error() or b"").decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def workspace_bytes(kind: int, db=None, net=None, rows: int = 0, top_k: int = 0) -> int:
    n = C.c_size_t()
    _ok(_lib.scn_workspace_bytes(int(kind), None if db is None else C.byref(db.c),
                                 None if net is None else C.byref(net.c), int(rows), int(top_k),
                                 C.byref(n)))
    return int(n.value)


class Context:
    """An scn_ctx on one device, with the caller-owned workspace (a torch
    uint8 tensor) the library's calls take their scratch memory from."""

    def __init__(self, device: int = 0):
        self.device = device
        h = C.c_void_p()
        _ok(_lib.scn_ctx_create(C.byref(h), int(device)))
        self.h = h
        self.ws = None

    def ensure_workspace(self, nbytes: int):
        """Attach a workspace of at least nbytes (grown, never shrunk)."""
        if nbytes <= 0 or (self.ws is not None and self.ws.numel() >= nbytes):
            return
        size = max(int(nbytes), 2 * (0 if self.ws is None else self.ws.numel()))
        ws = torch.empty(size, dtype=torch.uint8, device=torch.device("cuda", self.device))
        _ok(_lib.scn_set_workspace(self.h, C.c_void_p(ws.data_ptr()), size))
        self.ws = ws

    def set_workspace(self, ws: Optional[torch.Tensor]):
        """Attach exactly this uint8 tensor (None detaches)."""
        if ws is None:
            _ok(_lib.scn_set_workspace(self.h, None, 0))
        else:
            _ok(_lib.scn_set_workspace(self.h, C.c_void_p(ws.data_ptr()), int(ws.numel())))
        self.ws = ws

    def close(self):
        if self.h:
            _lib.scn_ctx_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset_counters(self, stream=None):
        _ok(_lib.scn_reset_counters(self.h, _stream(stream)))

    def read_counters(self, stream=None) -> dict:
        c = Counters()
        _ok(_lib.scn_read_counters(self.h, C.byref(c), _stream(stream)))
        return c.as_dict()

    def autotune(self, db: "DeviceBatch", args: "GenArgs", stream=None):
        """Time every schedule on this batch; returns (schedule, ms)."""
        sched, ms = C.c_int32(), C.c_float()
        self.ensure_workspace(workspace_bytes(WS_GENERATE, db))
        a = args.c()
        _ok(_lib.scn_autotune(self.h, C.byref(db.c), C.byref(a), C.byref(sched), C.byref(ms),
                              _stream(stream)))
        return int(sched.value), float(ms.value)

    def save_tuning(self, path: str):
        _ok(_lib.scn_autotune_save(self.h, path.encode()))

    def load_tuning(self, path: str):
        _ok(_lib.scn_autotune_load(self.h, path.encode()))


@dataclass
class GenArgs:
    seed: int = 0
    margin: float = 0.005
    retries: int = 10
    default_ncand: int = 1024
    max_steps: int = 0
    schedule: int = 0
    use_graph: int = 0
    fallback_chunk: int = 0
    wide_schedule: int = 0

    def c(self) -> _GenArgs:
        a = _GenArgs()
        a.seed, a.margin, a.retries = int(self.seed) & (2 ** 64 - 1), float(self.margin), int(self.retries)
        a.default_ncand, a.max_steps = int(self.default_ncand), int(self.max_steps)
        a.schedule, a.use_graph = int(self.schedule), int(self.use_graph)
        a.fallback_chunk = int(self.fallback_chunk)
        a.wide_schedule = int(self.wide_schedule)
        return a


GEOM_GENERAL, GEOM_YAW = 0, 1


def geometry_is_yaw(b) -> bool:
    """Whether every support rotation of the (host) batch is a turn about z,
    [[a, -b, 0], [b, a, 0], [0, 0, 1]] exactly in FP32, and every box rotation
    keeps the z axis: the class the library's SCN_GEOM_YAW declares."""
    sup = np.asarray(b.sup, np.float32).reshape(-1, 16)
    box = np.asarray(b.box, np.float32).reshape(-1, 16) if b.n_boxes else np.zeros((0, 16), np.float32)
    zero = lambda a, cols: bool(np.all(a[:, cols] == 0))
    sup_ok = (zero(sup, [2, 5, 6, 7]) and bool(np.all(sup[:, 8] == 1)) and
              bool(np.all(sup[:, 0] == sup[:, 4])) and bool(np.all(sup[:, 1] == -sup[:, 3])))
    box_ok = zero(box, [2, 5, 6, 7]) and bool(np.all(box[:, 8] == 1))
    return sup_ok and box_ok


class DeviceBatch:
    """Device copies of a SceneBatch plus the mutable placement state."""

    def __init__(self, b, device: str = "cuda"):
        dev = torch.device(device)
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
        self.host = b
        self.obj_off = t(b.obj_off, torch.int32)
        self.sph_off = t(b.sph_off, torch.int32)
        self.tmpl = t(b.tmpl, torch.float32)
        self.obj_sup = t(b.obj_sup, torch.int32)
        self.obj_ncand = t(b.obj_ncand, torch.int32)
        self.sup = t(b.sup, torch.float32)
        self.box_off = t(b.box_off, torch.int32)
        self.box = t(b.box.reshape(-1, 16), torch.float32) if b.n_boxes else \
            torch.zeros((1, 16), dtype=torch.float32, device=dev)
        self.grid_off = self.grid = self.grid_src = self.grid_val_off = self.grid_val = None
        n_assets = 0
        if b.grid_off is not None:
            self.grid_off = t(b.grid_off, torch.int32)
            self.grid = t(b.grid.reshape(-1, 24), torch.float32)
            self.grid_src = t(b.grid_src, torch.int32)
            vals = [np.ascontiguousarray(v, np.float32).ravel() for v in b.grid_vals]
            off = np.zeros(len(vals) + 1, np.int64)
            off[1:] = np.cumsum([v.size for v in vals])
            self.grid_val_off = t(off, torch.int64)
            self.grid_val = t(np.concatenate(vals), torch.float32)
            n_assets = len(vals)
        self.obj_rel = self.rel = self.obj_ratio = None
        if getattr(b, "obj_rel", None) is not None:
            self.obj_rel = t(b.obj_rel, torch.int32)
            self.rel = t(np.asarray(b.rel, np.float32).reshape(-1, 16), torch.float32)
        if getattr(b, "obj_ratio", None) is not None:
            self.obj_ratio = t(b.obj_ratio, torch.float32)
        self.robot = self.obj_reach = self.reach_map = None
        if getattr(b, "robot", None) is not None:
            self.robot = t(np.asarray(b.robot, np.float32).reshape(-1, 12), torch.float32)
            self.obj_reach = t(b.obj_reach, torch.float32)
            self.reach_map = t(np.asarray(b.reach_map, np.uint8).ravel(), torch.uint8)
        self.obj_pose_off = self.stable = self.rec_stable = None
        if getattr(b, "obj_pose_off", None) is not None:
            self.obj_pose_off = t(b.obj_pose_off, torch.int32)
            st = np.asarray(b.stable, np.float32).reshape(-1, 12)
            self.stable = t(st if len(st) else np.zeros((1, 12), np.float32), torch.float32)
            self.rec_stable = torch.full((max(b.n_objects, 1),), -1, dtype=torch.int32, device=dev)
        n, n_obj, n_sph = b.n_scenes, b.n_objects, b.n_spheres
        self.placed = torch.full((max(n_sph, 1), 4), float("nan"), dtype=torch.float32, device=dev)
        self.n_placed = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
        self.status = torch.zeros(max(n, 1), dtype=torch.int8, device=dev)
        self.rec = torch.zeros((max(n_obj, 1), 6), dtype=torch.int32, device=dev)  # 24 B records
        nobj = b.objects_per_scene()
        self.c = _Batch()
        c = self.c
        c.n_scenes, c.n_objects, c.n_spheres = n, n_obj, n_sph
        c.n_supports, c.n_boxes = int(b.sup.shape[0]), b.n_boxes
        c.n_grids = 0 if b.grid is None else int(b.grid.shape[0])
        c.n_grid_assets = n_assets
        c.max_objects_per_scene = int(nobj.max()) if n else 0
        c.max_spheres_per_object = int(b.spheres_per_object().max()) if n_obj else 0
        c.max_spheres_per_scene = int(b.spheres_per_scene().max()) if n else 0
        c.max_boxes_per_scene = int(b.boxes_per_scene().max()) if n else 0
        c.max_grids_per_scene = int(np.diff(b.grid_off).max()) if b.grid_off is not None and n else 0
        c.max_cand_per_object = int(b.obj_ncand.max()) if n_obj else 0
        c.geometry = GEOM_YAW if geometry_is_yaw(b) else GEOM_GENERAL
        for name in ("obj_off", "sph_off", "tmpl", "obj_sup", "obj_ncand", "sup", "box_off", "box",
                     "grid_off", "grid", "grid_src", "grid_val_off", "grid_val",
                     "placed", "n_placed", "status", "rec", "obj_rel", "rel", "obj_ratio",
                     "robot", "obj_reach", "obj_pose_off", "stable", "rec_stable"):
            setattr(c, name, None if getattr(self, name) is None else getattr(self, name).data_ptr())
        if self.reach_map is not None:
            c.reach = reach_map_struct(self.reach_map, b.reach_geom)

    def refresh_geometry(self):
        """Re-derive the declared geometry class from the device's support and
        box rows (after a call that rewrote them, e.g. forward kinematics)."""
        import dataclasses
        h = dataclasses.replace(self.host, sup=self.sup.cpu().numpy(),
                                box=self.box.cpu().numpy()[:self.host.n_boxes])
        self.c.geometry = GEOM_YAW if geometry_is_yaw(h) else GEOM_GENERAL

    # -- views of the state ------------------------------------------------
    def records(self):
        r = self.rec.cpu()
        f = r.view(torch.float32)[:, :4].numpy().copy()
        i = r[:, 4:6].numpy().copy()
        return f, i

    @property
    def max_cand(self) -> int:
        return int(self.c.max_cand_per_object)


# ---------------------------------------------------------------------------
def sample_poses(ctx: Context, db: DeviceBatch, obj_idx: torch.Tensor, cand_off: torch.Tensor,
                 total: int, max_cand: int, seed: int, attempt: int, stream=None,
                 with_stable: bool = False):
    """scn_sample_poses: (x, y, z, yaw) per candidate, and with with_stable
    the stable-pose row of each (-1: none)."""
    out = [torch.empty(max(total, 1), dtype=torch.float32, device=obj_idx.device) for _ in range(4)]
    k = torch.empty(max(total, 1), dtype=torch.int32, device=obj_idx.device) if with_stable else None
    p = _Poses(*[o.data_ptr() for o in out], _ptr(k))
    _ok(_lib.scn_sample_poses(ctx.h, C.byref(db.c), _ptr(obj_idx), _ptr(cand_off), int(total),
                              int(max_cand), int(seed) & (2 ** 64 - 1), int(attempt), p,
                              _stream(stream)))
    res = [o[:total] for o in out]
    return res + [k[:total]] if with_stable else res


def check_batch(ctx: Context, db: DeviceBatch, obj_idx: torch.Tensor, cand_off: torch.Tensor,
                total: int, max_cand: int, poses, margin: float = 0.005, want_clearance=True,
                want_collide=True, stream=None):
    dev = obj_idx.device
    clr = torch.empty(max(total, 1), dtype=torch.float32, device=dev) if want_clearance else None
    col = torch.empty(max(total, 1), dtype=torch.uint8, device=dev) if want_collide else None
    p = _Poses(*[q.data_ptr() for q in poses[:4]], _ptr(poses[4]) if len(poses) > 4 else None)
    _ok(_lib.scn_check_batch(ctx.h, C.byref(db.c), _ptr(obj_idx), _ptr(cand_off), int(total),
                             int(max_cand), p, float(margin), _ptr(clr), _ptr(col),
                             _stream(stream)))
    return (None if clr is None else clr[:total]), (None if col is None else col[:total])


def reset_scenes(ctx: Context, db: DeviceBatch, stream=None):
    _ok(_lib.scn_reset_scenes(ctx.h, C.byref(db.c), _stream(stream)))


def place_step(ctx: Context, db: DeviceBatch, args: GenArgs, stream=None) -> torch.Tensor:
    chosen = torch.empty(max(db.c.n_scenes, 1), dtype=torch.int32, device=db.n_placed.device)
    ctx.ensure_workspace(workspace_bytes(WS_GENERATE, db))
    a = args.c()
    _ok(_lib.scn_place_step(ctx.h, C.byref(db.c), C.byref(a), _ptr(chosen), _stream(stream)))
    return chosen[:db.c.n_scenes]


def generate_scenes(ctx: Context, db: DeviceBatch, args: GenArgs, stream=None):
    ctx.ensure_workspace(workspace_bytes(WS_GENERATE, db))
    a = args.c()
    _ok(_lib.scn_generate_scenes(ctx.h, C.byref(db.c), C.byref(a), _stream(stream)))


class Joints:
    """Device copies of a batch's articulation (scn_joints) and of the rows the
    links carry, plus the joint values and link poses FK writes."""

    def __init__(self, art: dict, device: str = "cuda"):
        dev = torch.device(device)
        t = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(dev)
        self.joint_off = t(art["joint_off"], torch.int32)
        self.joint = t(np.asarray(art["joint"]).reshape(-1, 24), torch.float32)
        self.base = t(np.asarray(art["base"]).reshape(-1, 12), torch.float32)
        self.box_link = t(art.get("box_link"), torch.int32)
        self.box_local = t(art.get("box_local"), torch.float32)
        self.sup_link = t(art.get("sup_link"), torch.int32)
        self.sup_local = t(art.get("sup_local"), torch.float32)
        n, nj = int(self.joint_off.numel() - 1), int(self.joint.shape[0])
        self.q = torch.zeros(max(nj, 1), dtype=torch.float32, device=dev)
        self.link = torch.zeros((max(nj, 1), 12), dtype=torch.float32, device=dev)
        self.c = _Joints(n, nj, self.joint_off.data_ptr(), self.joint.data_ptr(),
                         self.base.data_ptr())


def forward_kinematics(ctx: Context, joints: Joints, db: Optional["DeviceBatch"] = None,
                       seed: int = 0, sample: bool = True, stream=None):
    """scn_forward_kinematics: joint values (drawn from seed, or joints.q as
    set), link poses, and the box / support rows of db that links carry."""
    nb = 0 if db is None or joints.box_link is None else int(joints.box_link.numel())
    ns = 0 if db is None or joints.sup_link is None else int(joints.sup_link.numel())
    _ok(_lib.scn_forward_kinematics(
        ctx.h, C.byref(joints.c), int(seed) & (2 ** 64 - 1), int(bool(sample)), _ptr(joints.q),
        _ptr(joints.link), nb, _ptr(joints.box_link) if nb else None,
        _ptr(joints.box_local) if nb else None, _ptr(db.box) if nb else None, ns,
        _ptr(joints.sup_link) if ns else None, _ptr(joints.sup_local) if ns else None,
        _ptr(db.sup) if ns else None, _stream(stream)))


def reach_map_struct(dev_map: torch.Tensor, geom) -> _ReachMap:
    """scn_reach_map over a device uint8 map; geom = lo[4], h[4], dims[4]."""
    g = np.asarray(geom, np.float64)
    m = _ReachMap()
    m.map = dev_map.data_ptr()
    for a in range(4):
        m.lo[a], m.h[a], m.dims[a] = float(g[a]), float(g[4 + a]), int(g[8 + a])
    return m


def reach_query(ctx: Context, dev_map: torch.Tensor, geom, robot: torch.Tensor,
                pose: torch.Tensor, theta: torch.Tensor, stream=None) -> torch.Tensor:
    """scn_reach_query: reachable flags (uint8) of n object-frame world poses."""
    n = int(pose.shape[0])
    out = torch.empty(max(n, 1), dtype=torch.uint8, device=pose.device)
    m = reach_map_struct(dev_map, geom)
    _ok(_lib.scn_reach_query(ctx.h, C.byref(m), n, _ptr(robot), _ptr(pose), _ptr(theta),
                             _ptr(out), _stream(stream)))
    return out[:n]


NOALLOC_MAX_SCENES = 1 << 20


def generate_scenes_noalloc(ctx: Context, db: DeviceBatch, args: GenArgs, stream=None):
    """scn_generate_scenes with the scene-order scratch in the library's fixed
    device array: attaches no workspace and allocates nothing."""
    a = args.c()
    _ok(_lib.scn_generate_scenes_noalloc(ctx.h, C.byref(db.c), C.byref(a), _stream(stream)))


# ---------------------------------------------------------------------------
# Learned pose proposal
class Network:
    """Device tensors of the proposal network (scn_mlp) -- FP32 master weights
    and biases, BF16 copies (W and W^T, as int16 storage) and AdamW moments."""

    def __init__(self, dims=(FEATURES, 512, 512, 512, BINS), device="cuda", train=True):
        dev = torch.device(device)
        self.dims = tuple(int(d) for d in dims)
        L = len(self.dims) - 1
        assert L == N_LAYERS
        f32 = lambda *s: torch.zeros(*s, dtype=torch.float32, device=dev)
        b16 = lambda *s: torch.zeros(*s, dtype=torch.bfloat16, device=dev)
        self.w = [f32(self.dims[l + 1], self.dims[l]) for l in range(L)]
        self.b = [f32(self.dims[l + 1]) for l in range(L)]
        self.wb = [b16(self.dims[l + 1], self.dims[l]) for l in range(L)]
        self.wt = [b16(self.dims[l], self.dims[l + 1]) for l in range(L)]
        self.mw = [f32(self.dims[l + 1], self.dims[l]) for l in range(L)] if train else None
        self.vw = [f32(self.dims[l + 1], self.dims[l]) for l in range(L)] if train else None
        self.mb = [f32(self.dims[l + 1]) for l in range(L)] if train else None
        self.vb = [f32(self.dims[l + 1]) for l in range(L)] if train else None
        self.c = Mlp()
        for l, d in enumerate(self.dims):
            self.c.dims[l] = d
        for l in range(L):
            self.c.w[l], self.c.b[l] = self.w[l].data_ptr(), self.b[l].data_ptr()
            self.c.wb[l], self.c.wt[l] = self.wb[l].data_ptr(), self.wt[l].data_ptr()
            if train:
                self.c.m_w[l], self.c.v_w[l] = self.mw[l].data_ptr(), self.vw[l].data_ptr()
                self.c.m_b[l], self.c.v_b[l] = self.mb[l].data_ptr(), self.vb[l].data_ptr()
        self.c.step = 0

    def init(self, ctx: Context, seed: int, stream=None):
        _ok(_lib.scn_mlp_init(ctx.h, C.byref(self.c), int(seed) & (2 ** 64 - 1), _stream(stream)))

    def load(self, ws, bs):
        """Set FP32 weights/biases (host arrays) and refresh the BF16 copies
        (the copies are conversions of the given values)."""
        for l in range(N_LAYERS):
            self.w[l].copy_(torch.as_tensor(np.asarray(ws[l], np.float32)))
            self.b[l].copy_(torch.as_tensor(np.asarray(bs[l], np.float32)))
            self.wb[l].copy_(self.w[l].to(torch.bfloat16))
            self.wt[l].copy_(self.w[l].t().contiguous().to(torch.bfloat16))
        if self.mw is not None:
            for t in self.mw + self.vw + self.mb + self.vb:
                t.zero_()
        self.c.step = 0

    def state(self):
        return {"dims": self.dims, "step": int(self.c.step),
                "w": [t.cpu() for t in self.w], "b": [t.cpu() for t in self.b]}


def mlp_forward(ctx: Context, net: Network, x: torch.Tensor, stream=None) -> torch.Tensor:
    M = int(x.shape[0])
    out = torch.empty((max(M, 1), net.dims[-1]), dtype=torch.float32, device=x.device)
    ctx.ensure_workspace(workspace_bytes(WS_MLP_FORWARD, net=net, rows=M))
    _ok(_lib.scn_mlp_forward(ctx.h, C.byref(net.c), _ptr(x), M, _ptr(out), _stream(stream)))
    return out[:M]


def mlp_backward(ctx: Context, net: Network, x, bins, tgt, stream=None):
    M, L = int(bins.shape[0]), int(bins.shape[1])
    gw = [torch.empty_like(w) for w in net.w]
    gb = [torch.empty_like(b) for b in net.b]
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    pw = (C.c_void_p * N_LAYERS)(*[g.data_ptr() for g in gw])
    pb = (C.c_void_p * N_LAYERS)(*[g.data_ptr() for g in gb])
    ctx.ensure_workspace(workspace_bytes(WS_MLP_BACKWARD, net=net, rows=M))
    _ok(_lib.scn_mlp_backward(ctx.h, C.byref(net.c), _ptr(x), M, _ptr(bins), _ptr(tgt), L,
                              C.cast(pw, C.c_void_p), C.cast(pb, C.c_void_p), _ptr(loss),
                              _stream(stream)))
    return loss, gw, gb


def mlp_train_step(ctx: Context, net: Network, x, bins, tgt, lr=1e-3, betas=(0.9, 0.999),
                   eps=1e-8, weight_decay=1e-4, loss=None, stream=None):
    M, L = int(bins.shape[0]), int(bins.shape[1])
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    opt = AdamW(float(lr), float(betas[0]), float(betas[1]), float(eps), float(weight_decay))
    ctx.ensure_workspace(workspace_bytes(WS_MLP_TRAIN, net=net, rows=M))
    _ok(_lib.scn_mlp_train_step(ctx.h, C.byref(net.c), _ptr(x), M, _ptr(bins), _ptr(tgt), L,
                                C.byref(opt), _ptr(loss), _stream(stream)))
    return loss


def descriptors(ctx: Context, db: DeviceBatch, stream=None) -> torch.Tensor:
    out = torch.empty((max(db.c.n_objects, 1), DESC), dtype=torch.float32, device=db.tmpl.device)
    _ok(_lib.scn_descriptors(ctx.h, C.byref(db.c), _ptr(out), _stream(stream)))
    return out[:db.c.n_objects]


def heightmaps(ctx: Context, db: DeviceBatch, n_state: Optional[torch.Tensor] = None,
               stream=None) -> torch.Tensor:
    """scn_heightmaps: one [4096] map per support (zeros where no object rests)."""
    out = torch.zeros((max(db.c.n_supports, 1), HMAP_CELLS), dtype=torch.float32,
                      device=db.tmpl.device)
    _ok(_lib.scn_heightmaps(ctx.h, C.byref(db.c), _ptr(n_state), _ptr(out), _stream(stream)))
    return out[:db.c.n_supports]


def features(ctx: Context, db: DeviceBatch, hmap, desc, obj_idx, stream=None) -> torch.Tensor:
    """scn_features: row r = [10 x the map of obj_idx[r]'s support, its descriptor]."""
    n = int(obj_idx.shape[0])
    out = torch.empty((max(n, 1), FEATURES), dtype=torch.bfloat16, device=obj_idx.device)
    _ok(_lib.scn_features(ctx.h, C.byref(db.c), n, _ptr(hmap), _ptr(desc), _ptr(obj_idx),
                          _ptr(out), _stream(stream)))
    return out[:n]


def proposal_topk(ctx: Context, logits, k: int, active=None, stream=None) -> torch.Tensor:
    M = int(logits.shape[0])
    out = torch.full((max(M, 1), k), -1, dtype=torch.int32, device=logits.device)
    _ok(_lib.scn_proposal_topk(ctx.h, _ptr(logits), M, int(k), _ptr(active), _ptr(out),
                               _stream(stream)))
    return out[:M]


def harvest_labels(ctx: Context, db: DeviceBatch, n_state, L: int, seed: int, round_: int = 0,
                   margin: float = 0.005, stream=None):
    n = db.c.n_scenes
    bins = torch.empty((max(n, 1), L), dtype=torch.int32, device=db.tmpl.device)
    acc = torch.empty((max(n, 1), L), dtype=torch.float32, device=db.tmpl.device)
    _ok(_lib.scn_harvest_labels(ctx.h, C.byref(db.c), _ptr(n_state), int(L),
                                int(seed) & (2 ** 64 - 1), int(round_), float(margin), _ptr(bins),
                                _ptr(acc), _stream(stream)))
    return bins[:n], acc[:n]


def generate_scenes_learned(ctx: Context, db: DeviceBatch, args: GenArgs, net: Network,
                            top_k: int = 64, stream=None):
    ctx.ensure_workspace(workspace_bytes(WS_GENERATE_LEARNED, db, net, top_k=top_k))
    a = args.c()
    _ok(_lib.scn_generate_scenes_learned(ctx.h, C.byref(db.c), C.byref(a), C.byref(net.c),
                                         int(top_k), _stream(stream)))
