"""Seeded synthetic Markov chains shaped like the paper's test problems (Section 5).

This module only builds inputs: the column-stochastic transition matrix ``A`` in
CSR form (row = destination state, column = source state, so every column sums
to one, Section 2) plus the grid geometry the full coarsening needs.  It holds
none of the multilevel method's arithmetic, so both the GPU path and the CPU
oracle may use it.

State numbering is row-major on an ``nx x ny`` grid: state ``s = a*ny + b``.
A chain without a grid (``nx = ny = 0``) is coarsened by compatible relaxation.

Randomness is counter-based: ``uniform(seed, stream, idx)`` is the SplitMix64
finaliser (Steele, Lea and Flood, OOPSLA 2014) applied to
``(seed XOR stream*GAMMA) + idx + GAMMA`` and mapped to [0, 1) with 53 bits.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream identifiers.  STREAM_TV is drawn by the method itself (initial test
# vectors); the others only by the generators in this module.
STREAM_TV = 1
STREAM_LATTICE_W = 2
STREAM_JITTER = 3
STREAM_BATCH = 4
STREAM_MLP_INIT = 5
STREAM_MLP_SHUFFLE = 6
STREAM_TRAIN_SIZES = 8   # (stream 7 is the coarsest Arnoldi start vector)
STREAM_UPG = 9           # point coordinates of the unstructured planar graph
# (streams 16 + l are the compatible-relaxation start vectors of level l)


def splitmix64(key: np.ndarray) -> np.ndarray:
    """SplitMix64 output for state ``key`` (one increment by GAMMA, then mix)."""
    z = np.asarray(key, dtype=np.uint64) + GAMMA
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, idx) -> np.ndarray:
    """Counter-based uniform numbers in [0, 1): one per entry of ``idx``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) ^ (np.uint64(stream) * GAMMA)) + idx
    h = splitmix64(key)
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


@dataclass
class Chain:
    """A transition matrix in CSR (row = destination, column = source)."""
    n: int
    row_ptr: np.ndarray   # int32, n+1
    col_idx: np.ndarray   # int32, nnz, ascending within each row
    val: np.ndarray       # float64, nnz
    nx: int
    ny: int
    periodic: bool
    name: str = ""
    exact: np.ndarray | None = None   # closed-form stationary vector, if known

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _csr_from_triplets(n, dst, src, p):
    """Sum duplicates and sort columns within each row."""
    order = np.lexsort((src, dst))
    dst, src, p = dst[order], src[order], p[order]
    key = dst.astype(np.int64) * n + src
    uniq, start = np.unique(key, return_index=True)
    sums = np.add.reduceat(p, start) if len(p) else p
    rows = (uniq // n).astype(np.int64)
    cols = (uniq % n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols, sums.astype(np.float64)


def tandem_queue(N: int, rates=(11 / 31, 10 / 31, 10 / 31), jitter: float = 0.0,
                 seed: int = 0, chain_id: int = 0) -> Chain:
    """Two queues in tandem with capacities ``N`` (Section 5, Table 2).

    State (a, b): ``a`` customers in queue 1 and ``b`` in queue 2, 0 <= a, b <= N.
    Moves: arrival (a,b)->(a+1,b) at rate ``rates[0]``; service
    (a,b)->(a-1,b+1) at ``rates[1]``; departure (a,b)->(a,b-1) at ``rates[2]``.
    The chain is uniformised by the total rate; a move that is blocked at the
    boundary becomes a self-loop, so every column of ``A`` sums to one.
    ``jitter`` multiplies each rate by ``1 + jitter*(2u-1)`` with ``u`` drawn
    from (seed, STREAM_JITTER, 3*chain_id + k).
    """
    lam, mu1, mu2 = (float(r) for r in rates)
    if jitter:
        u = uniform(seed, STREAM_JITTER, np.arange(3) + 3 * chain_id)
        lam, mu1, mu2 = (r * (1.0 + jitter * (2.0 * ui - 1.0)) for r, ui in zip((lam, mu1, mu2), u))
    tot = lam + mu1 + mu2
    pa, ps, pd = lam / tot, mu1 / tot, mu2 / tot
    side = N + 1
    a, b = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    a = a.ravel(); b = b.ravel()
    s = a * side + b
    dst, src, p = [], [], []
    # arrival
    ok = a < N
    dst.append(s[ok] + side); src.append(s[ok]); p.append(np.full(ok.sum(), pa))
    # service 1 -> 2
    ok = (a > 0) & (b < N)
    dst.append(s[ok] - side + 1); src.append(s[ok]); p.append(np.full(ok.sum(), ps))
    # departure from queue 2
    ok = b > 0
    dst.append(s[ok] - 1); src.append(s[ok]); p.append(np.full(ok.sum(), pd))
    # self-loops carry the blocked probability
    blocked = pa * (a >= N) + ps * ((a == 0) | (b >= N)) + pd * (b == 0)
    ok = blocked > 0
    dst.append(s[ok]); src.append(s[ok]); p.append(blocked[ok])
    dst = np.concatenate(dst); src = np.concatenate(src); p = np.concatenate(p)
    row_ptr, col, val = _csr_from_triplets(side * side, dst, src, p)
    return Chain(side * side, row_ptr, col, val, side, side, False, name=f"tandem{N}")


def weighted_lattice(m: int, seed: int = 0, periodic: bool = True, my: int | None = None,
                     chain_id: int = 0, wlo: float = 0.1, whi: float = 1.0,
                     uniform_weights: bool = False) -> Chain:
    """Random walk on an ``m x my`` lattice with symmetric edge weights.

    Edge ids: ``2s`` joins s=(a,b) to (a,b+1) and ``2s+1`` joins s to (a+1,b)
    (wrapping when periodic, absent at the border otherwise).  Each weight is
    ``wlo + (whi-wlo)*u`` with ``u`` from (seed, STREAM_LATTICE_W, id + chain
    offset); ``uniform_weights`` sets every weight to one (the paper's uniform
    network, Section 5, Table 1).  ``p(i->j) = w_ij / d_i`` with
    ``d_i = sum_k w_ik``; the walk is reversible, so the stationary vector is
    proportional to the weighted degree ``d``.
    """
    my = m if my is None else my
    n = m * my
    a, b = np.meshgrid(np.arange(m), np.arange(my), indexing="ij")
    a = a.ravel(); b = b.ravel()
    s = a * my + b
    off = np.uint64(chain_id) << np.uint64(40)
    ends_i, ends_j, w = [], [], []
    for d, (da, db) in enumerate(((0, 1), (1, 0))):
        na, nb = a + da, b + db
        if periodic:
            ok = np.ones(n, dtype=bool)
            na %= m; nb %= my
        else:
            ok = (na < m) & (nb < my)
        ids = (2 * s + d).astype(np.uint64)[ok] + off
        if uniform_weights:
            ww = np.ones(ok.sum())
        else:
            ww = wlo + (whi - wlo) * uniform(seed, STREAM_LATTICE_W, ids)
        ends_i.append(s[ok]); ends_j.append((na * my + nb)[ok]); w.append(ww)
    ei = np.concatenate(ends_i); ej = np.concatenate(ends_j); w = np.concatenate(w)
    deg = np.zeros(n)
    np.add.at(deg, ei, w)
    np.add.at(deg, ej, w)
    # A[j, i] = w_ij / d_i for both directions of every edge
    dst = np.concatenate([ej, ei]); src = np.concatenate([ei, ej])
    p = np.concatenate([w / deg[ei], w / deg[ej]])
    row_ptr, col, val = _csr_from_triplets(n, dst, src, p)
    exact = deg / deg.sum()
    name = ("uniform" if uniform_weights else "lattice") + f"{m}" + ("p" if periodic else "")
    return Chain(n, row_ptr, col, val, m, my, periodic, name=name, exact=exact)


def upg(N: int, seed: int = 0) -> Chain:
    """Unstructured planar graph (Section 5, Table 4): the Delaunay
    triangulation of ``N`` points in the unit square, point ``i`` at
    ``(u(2i), u(2i+1))`` drawn from (seed, STREAM_UPG); from state ``j`` the walk
    moves to each of its ``d_j`` triangulation neighbours with probability
    ``1/d_j``.  It is reversible with stationary vector proportional to ``d``.
    The points are numbered in the order drawn, so the numbering carries no
    geometry; the chain has no grid (``nx = ny = 0``)."""
    from scipy.spatial import Delaunay
    xy = uniform(seed, STREAM_UPG, np.arange(2 * N)).reshape(N, 2)
    tri = Delaunay(xy).simplices.astype(np.int64)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]])
    e = np.sort(e, axis=1)
    e = np.unique(e[:, 0] * N + e[:, 1])
    ei, ej = e // N, e % N
    deg = np.zeros(N)
    np.add.at(deg, ei, 1.0)
    np.add.at(deg, ej, 1.0)
    dst = np.concatenate([ej, ei]); src = np.concatenate([ei, ej])
    p = 1.0 / deg[src]
    row_ptr, col, val = _csr_from_triplets(N, dst, src, p)
    return Chain(N, row_ptr, col, val, 0, 0, False, name=f"upg{N}", exact=deg / deg.sum())


def batch_mix(n_chains: int = 64, seed: int = 0):
    """The batched workload: each chain is a jittered tandem queue (probability
    1/2, N uniform in [31, 511]) or a weighted periodic lattice (side uniform in
    [32, 512], rounded down to a multiple of 16 so that it coarsens evenly)."""
    chains = []
    for c in range(n_chains):
        u = uniform(seed, STREAM_BATCH, np.arange(3) + 3 * c)
        if u[0] < 0.5:
            N = 31 + int(u[1] * 481)
            chains.append(tandem_queue(N, jitter=0.2, seed=seed, chain_id=c))
        else:
            side = 32 + int(u[2] * 481)
            side = max(32, side - side % 16)
            chains.append(weighted_lattice(side, seed=seed, chain_id=c))
    return chains


def training_chains(n_chains: int = 32, seed: int = 0, n_min: int = 255, n_max: int = 1023):
    """Training set of the learned form: jittered tandem queues (rates times
    1 +- 0.2) with N = n_min + floor((n_max - n_min + 1) u), u drawn from
    (seed, STREAM_TRAIN_SIZES, chain)."""
    u = uniform(seed, STREAM_TRAIN_SIZES, np.arange(n_chains))
    return [tandem_queue(n_min + int(u[c] * (n_max - n_min + 1)), jitter=0.2, seed=seed, chain_id=1000 + c)
            for c in range(n_chains)]


def config_chain(cfg: int, seed: int = 0) -> Chain:
    """The single-chain workloads: 0 = tandem N=32, 1 = periodic lattice 1024,
    2 = tandem N=2047."""
    if cfg == 0:
        return tandem_queue(32, seed=seed)
    if cfg == 1:
        return weighted_lattice(1024, seed=seed + 1)
    if cfg == 2:
        return tandem_queue(2047, seed=seed)
    raise ValueError(cfg)
