"""GPU: what the trained proposal network gains over uniform sampling.

A network is trained on the device (library forward / backward / AdamW
kernels) on accept / reject labels harvested from plain runs, then used on
held-out scenes of the same shape.  The gain is measured against the plain
method on the same scenes: how often the first candidate tried is accepted,
and how many candidates (in try order) precede the accepted one.  Every
learned placement is audited in FP64 for the margin.  The size of the gain is
an empirical property of the trained network, not fixed by the method, so
the thresholds are loose lower bounds.
"""
import numpy as np
import pytest

from gpu_util import audit_placements
from paper_2512_16896_amd import scenegen as sg

pytestmark = pytest.mark.gpu


def _tries_before(rec_i, ncand, top_k, learned):
    """Candidates tried before the accepted one, per placed object, in the
    order each method tries them (proposals first for the learned method)."""
    a, i = rec_i[:, 0].astype(np.int64), rec_i[:, 1].astype(np.int64)
    placed = i >= 0
    off = top_k if learned else 0
    tries = np.where(a == -2, i, off + a * ncand + i)
    return tries[placed]


def test_trained_network_beats_uniform_sampling():
    import torch
    from paper_2512_16896_amd import learned as L
    from paper_2512_16896_amd import scn
    ctx = scn.Context(0)
    parts = []
    for k in range(4):
        tb = sg.batched_scenes(1024, seed=300 + k)
        tdb = scn.DeviceBatch(tb)
        scn.generate_scenes(ctx, tdb, scn.GenArgs(seed=40 + k))
        parts.append(L.harvest(ctx, tdb, seed=60 + k, labels_per_state=64))
    data = L.merge(parts)
    uniform_rate = data.positive_rate()
    net = scn.Network()
    net.init(ctx, 5)
    log = L.train(ctx, net, data, steps=4000, batch=256, log_every=3999)
    assert log[-1][1] < 0.8 * log[0][1]

    b = sg.batched_scenes(512, seed=999)         # held out
    db = scn.DeviceBatch(b)
    scn.generate_scenes(ctx, db, scn.GenArgs(seed=7))
    torch.cuda.synchronize()
    _, plain_rec = db.records()
    plain_valid = int((db.status == 1).sum().item())
    scn.generate_scenes_learned(ctx, db, scn.GenArgs(seed=7), net, top_k=64)
    torch.cuda.synchronize()
    _, rec = db.records()
    valid = int((db.status == 1).sum().item())

    first_plain = float(np.mean(_tries_before(plain_rec, 1024, 64, False) == 0))
    first_learned = float(np.mean(_tries_before(rec, 1024, 64, True) == 0))
    within_plain = float(np.mean(_tries_before(plain_rec, 1024, 64, False) < 4))
    within_learned = float(np.mean(_tries_before(rec, 1024, 64, True) < 4))
    print(f"labels {len(data) * 64}, uniform accept rate {uniform_rate:.3f}; first candidate "
          f"accepted: plain {first_plain:.3f}, learned {first_learned:.3f}; accepted within 4 "
          f"tries: plain {within_plain:.3f}, learned {within_learned:.3f}; valid scenes: "
          f"plain {plain_valid}, learned {valid} of {b.n_scenes}")
    # the top-ranked bin is accepted far more often than a uniform candidate
    assert first_learned > 2.0 * max(first_plain, uniform_rate)
    assert within_learned > 1.3 * within_plain
    # no loss of validity from the proposal (the exact checker decides)
    assert valid >= 0.95 * plain_valid
    pick = np.arange(0, b.n_scenes, 64)
    sub, _ = sg.subset(b, pick)
    placed = db.placed.cpu().numpy()
    npl = db.n_placed.cpu().numpy()
    rows = np.concatenate([np.arange(b.sph_off[b.obj_off[s]], b.sph_off[b.obj_off[s + 1]])
                           for s in pick])
    audit_placements(sub, placed[rows], npl[pick])
    ctx.close()
