"""Learned pose proposal: label harvesting and training on the GPU.

Labels come from the exact checker: for every state of a plain generation run
(scene s with its first j objects placed, about to place object j) the
library's harvest kernel draws uniform candidates of object j, records their
pose bins and whether they are collision-free.  The state's features (the
height map of object j's support + its descriptor) are built by the
library's kernels too.  Training runs the
library's BF16 matrix-core forward / backward kernels and its AdamW kernel;
PyTorch here only holds the tensors and shuffles rows into minibatches.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import scn


@dataclass
class Dataset:
    x: torch.Tensor       # [N, FEATURES] bfloat16 state features
    bins: torch.Tensor    # [N, L] int32 pose bins of the label candidates
    accept: torch.Tensor  # [N, L] float32 1 = collision-free, 0 = collides

    def __len__(self):
        return int(self.x.shape[0])

    def positive_rate(self) -> float:
        return float(self.accept.mean().item())


def harvest(ctx: scn.Context, db: scn.DeviceBatch, seed: int, labels_per_state: int = 64,
            margin: float = 0.005, round_: int = 0) -> Dataset:
    """States of the batch's current placement (run a generation first): for
    every scene and j = 0 .. n_placed[s] (the object that failed included),
    the state with the first j objects placed."""
    dev = db.tmpl.device
    n = db.c.n_scenes
    nobj = (db.obj_off[1:] - db.obj_off[:-1]).to(torch.int32)
    desc = scn.descriptors(ctx, db)
    xs, bs, acs = [], [], []
    for j in range(int(nobj.max().item())):
        use = (db.n_placed[:n] >= j) & (nobj > j)
        if not bool(use.any()):
            continue
        n_state = torch.where(use, torch.full_like(nobj, j), nobj)   # no next object when unused
        obj_idx = torch.where(use, db.obj_off[:n] + j, torch.full_like(nobj, -1)).to(torch.int32)
        hmap = scn.heightmaps(ctx, db, n_state)
        x = scn.features(ctx, db, hmap, desc, obj_idx)
        bins, acc = scn.harvest_labels(ctx, db, n_state, labels_per_state, seed, round_, margin)
        keep = use.nonzero().squeeze(1)
        xs.append(x.index_select(0, keep))
        bs.append(bins.index_select(0, keep))
        acs.append(acc.index_select(0, keep))
    return Dataset(torch.cat(xs), torch.cat(bs), torch.cat(acs))


def merge(parts) -> Dataset:
    return Dataset(torch.cat([p.x for p in parts]), torch.cat([p.bins for p in parts]),
                   torch.cat([p.accept for p in parts]))


def train(ctx: scn.Context, net: scn.Network, data: Dataset, steps: int, batch: int = 256,
          lr: float = 1e-3, weight_decay: float = 1e-4, seed: int = 0, log_every: int = 0):
    """AdamW on minibatches of `batch` states (the library's kernels); returns
    the list of (step, loss) logged."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = len(data)
    perm = torch.randperm(N, generator=g).to(data.x.device)
    loss = torch.zeros(1, dtype=torch.float32, device=data.x.device)
    logged = []
    pos = 0
    for t in range(steps):
        if pos + batch > N:
            perm = torch.randperm(N, generator=g).to(data.x.device)
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        scn.mlp_train_step(ctx, net, data.x.index_select(0, idx), data.bins.index_select(0, idx),
                           data.accept.index_select(0, idx), lr=lr, weight_decay=weight_decay,
                           loss=loss)
        if log_every and (t % log_every == 0 or t == steps - 1):
            logged.append((t, float(loss.item())))
    return logged
