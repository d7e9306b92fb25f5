"""Training data and training of the learned interpolation (argument
marshalling around the C ABI; every step runs in the library).

collect(): one setup of a chain in the least-squares form with
options.collect, then bamg_mlp_collect: for every non-coarsest level the
first-pass features of its F points and, as the target, the correction of
their fitted weights (final minus first pass), ordinary points only.
train(): bamg_mlp_train_spec, which builds the training chains (jittered
tandem queues), collects their pairs and trains the network.
"""
from __future__ import annotations

from . import bamg as B


def collect(chain, r=12, levels=6, precision=None, seed=0):
    """(features, targets) of the chain's ordinary F points on every
    non-coarsest level, as device FP32 tensors."""
    opts = B.default_options(levels=levels, collect=1, seed=seed,
                             precision=B.FP64 if precision is None else precision)
    h = B.Hierarchy.from_chain(chain, r, opts)
    try:
        return B.mlp_collect(h)
    finally:
        h.close()


def train(n_chains=32, n_val=4, side_min=256, side_max=1024, r=12, levels=6, epochs=8, batch=4096, lr=1e-3,
          seed=0, shuffle_seed=6, init_seed=5, out_path=None):
    """Train on all but the last n_val chains of the library-built training
    set, validate on those; returns (params (device FP32), MlpTrainInfo)."""
    sp = B.train_spec(n_chains=n_chains, n_val=n_val, side_min=side_min, side_max=side_max, r=r, levels=levels,
                      epochs=epochs, batch=batch, lr=lr, seed=seed, shuffle_seed=shuffle_seed, init_seed=init_seed)
    return B.mlp_train_spec(sp, out_path)
