"""Training data and training of the learned interpolation (argument
marshalling around the C ABI; every step runs in the library's kernels).

collect(): one setup of a chain in the least-squares form with
options.collect, then for every non-coarsest level the first-pass features
(n x 24) of its F points and, as the target, how far the final interpolation
weights (after the recomputation pass) are from the first pass's fit, in slot
order (n x 4): the correction the network should predict from what the first
pass knows.
train(): Adam through bamg_mlp_train on the collected pairs.
"""
from __future__ import annotations

import torch

from . import bamg as B


# Training pairs are limited to ordinary points: all features within
# +-FEATURE_CAP and all target corrections within +-TARGET_CAP.  A tiny share
# of degenerate points (vanishing test-vector values, near-singular Gram) has
# features and corrections orders of magnitude larger, and would otherwise own
# the squared loss; at setup time the judge still screens every point.
FEATURE_CAP = 16.0
TARGET_CAP = 1.0


def collect(chain, r=12, levels=6, precision=None, seed=0, filtered=True):
    """(features, targets) of the chain's F points on every non-coarsest level,
    as device FP32 tensors (ordinary points only when filtered)."""
    opts = B.default_options(levels=levels, collect=1, seed=seed,
                             precision=B.FP64 if precision is None else precision)
    h = B.Hierarchy.from_chain(chain, r, opts)
    fs, ts = [], []
    for l in range(h.stats().n_levels - 1):
        n = h.level_info(l).n
        F = torch.from_numpy(h.export(l, B.X_FEATURES).reshape(n, 24))
        T = torch.from_numpy(h.export(l, B.X_SLOTW).reshape(n, 4) - h.export(l, B.X_SLOTW0).reshape(n, 4))
        f = F[:, :4].sum(1) > 0                      # F points: at least one slot
        if filtered:
            f &= (F.abs().amax(1) <= FEATURE_CAP) & (T.abs().amax(1) <= TARGET_CAP)
        fs.append(F[f])
        ts.append(T[f])
    h.close()
    return torch.cat(fs).cuda(), torch.cat(ts).cuda()


def dataset(chains, r=12, levels=6):
    feats, tgts = [], []
    for ch in chains:
        f, t = collect(ch, r, levels)
        feats.append(f)
        tgts.append(t)
    return torch.cat(feats), torch.cat(tgts)


def train(chains, r=12, levels=6, n_val=4, epochs=8, batch=4096, lr=1e-3, seed=6, init_seed=5):
    """Train on all but the last n_val chains, validate on those; returns
    (params (device FP32), MlpTrainInfo, sizes)."""
    ftr, ttr = dataset(chains[:-n_val] if n_val else chains, r, levels)
    fva, tva = dataset(chains[-n_val:], r, levels) if n_val else (None, None)
    params = B.mlp_init(init_seed)
    info = B.mlp_train(ftr, ttr, params, fva, tva, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return params, info, (ftr.shape[0], 0 if fva is None else fva.shape[0])
