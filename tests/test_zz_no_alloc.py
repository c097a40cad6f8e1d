"""GPU: scn_generate_scenes_noalloc (scene-order scratch in the library's fixed
device array) against scn_generate_scenes (scratch in the caller's workspace),
through the C ABI, on two calls in a row with the second batch smaller."""
import ctypes as C

import numpy as np
import pytest

from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu

LPT_GLOBAL = 0xF24     # 4 waves, longest-first order, placed spheres from global memory
LPT_LDS32 = 0x124      # 4 waves, longest-first order, 32 KB LDS budget (split launch)


def _state(db):
    import torch
    torch.cuda.synchronize()
    rec_f, rec_i = db.records()
    return (db.status.cpu().numpy(), db.n_placed.cpu().numpy(), rec_i, rec_f,
            db.placed.cpu().numpy())


@pytest.mark.parametrize("sched", [LPT_GLOBAL, LPT_LDS32])
def test_noalloc_matches_workspace_generation(sched):
    import torch
    from paper_2512_16896_amd import scn
    ctx = scn.Context(0)
    try:
        big = sg.uneven_batch(96, seed=31, n_obj=(5, 30), n_sph=(16, 256), n_cand=(64, 512))
        small = sg.uneven_batch(40, seed=32, n_obj=(5, 30), n_sph=(16, 256), n_cand=(64, 512))
        for k, b in enumerate((big, small)):
            print(f"noalloc call {k}: {b.n_scenes} scenes, schedule 0x{sched:x}", flush=True)
            args = scn.GenArgs(seed=40 + k, schedule=sched)
            ref = scn.DeviceBatch(b)
            scn.generate_scenes(ctx, ref, args)
            want = _state(ref)
            got_db = scn.DeviceBatch(b)
            scn.generate_scenes_noalloc(ctx, got_db, args)
            got = _state(got_db)
            for u, v in zip(want, got):
                assert np.array_equal(u, v, equal_nan=True)
            assert np.all(want[0] != scn.ACTIVE)
            ctx.read_counters()          # no device-side error either
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_noalloc_rejects_graphs_and_too_many_scenes():
    import torch
    from paper_2512_16896_amd import scn
    ctx = scn.Context(0)
    try:
        b = sg.uneven_batch(8, seed=33, n_obj=(5, 10), n_sph=(16, 64), n_cand=(64, 128))
        db = scn.DeviceBatch(b)
        with pytest.raises(scn.ScnError) as e:
            scn.generate_scenes_noalloc(ctx, db, scn.GenArgs(seed=1, schedule=LPT_GLOBAL,
                                                             use_graph=1))
        assert e.value.code == scn.SCN_E_UNSUPPORTED
        # A valid batch of empty scenes, one more than the fixed scratch holds:
        # every array is sized for it, and the call refuses it on the host.
        n = scn.NOALLOC_MAX_SCENES + 1
        dev = torch.device("cuda", 0)
        zeros = torch.zeros(n + 1, dtype=torch.int32, device=dev)
        n_placed = torch.zeros(n, dtype=torch.int32, device=dev)
        status = torch.zeros(n, dtype=torch.int8, device=dev)
        one = torch.zeros(16, dtype=torch.float32, device=dev)
        rec = torch.zeros(6, dtype=torch.int32, device=dev)
        c = scn._Batch()
        c.n_scenes, c.n_supports = n, 1
        for name in ("obj_off", "box_off"):
            setattr(c, name, zeros.data_ptr())
        c.sph_off, c.obj_sup, c.obj_ncand = zeros.data_ptr(), zeros.data_ptr(), zeros.data_ptr()
        c.sup = c.tmpl = c.box = c.placed = one.data_ptr()
        c.n_placed, c.status, c.rec = n_placed.data_ptr(), status.data_ptr(), rec.data_ptr()
        a = scn.GenArgs(seed=1, schedule=LPT_GLOBAL, default_ncand=64).c()
        rc = scn.lib().scn_generate_scenes_noalloc(ctx.h, C.byref(c), C.byref(a),
                                                   scn._stream(None))
        assert rc == scn.SCN_E_INVALID_ARG
        assert b"fixed scratch" in scn.lib().scn_last_error()
        torch.cuda.synchronize()
        # nothing was launched: the state arrays are untouched
        assert int(status.abs().sum()) == 0 and int(n_placed.abs().sum()) == 0
    finally:
        torch.cuda.synchronize()
        ctx.close()
