"""Test oracle of the learned-interpolation form (plain FP64 on the CPU).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's cpu_baseline leg, never by the product path.

The paper's method fits each interpolation row by least squares (Section 3.2,
Algorithm 2).  The learned form corrects the first-pass fit with a small
network that predicts, from features of the same local least-squares problem,
how far the weights the method settles on after its recomputation pass are
from the first-pass fit; the fit stays as judge and fallback.  None of this is
in the paper: the features, network and training follow the project's own
specification (24 features, 24-64-64-4 ReLU network, masked mean-squared
loss, Adam).

Everything here is written out plainly:
  * features(): 24 scale-free numbers per fine point from the weighted Gram
    G (4 x 4 over the slots), right-hand side b, sigma and the operator row;
  * forward()/loss_and_grad(): the network and its gradient by the chain rule,
    optionally with the operands of every matrix product rounded to bfloat16
    (round to nearest even), which is what the GPU's matrix cores see;
  * adam_step(): Kingma and Ba (2015), bias-corrected;
  * init_params(): He-uniform weights, U(-sqrt(6/fan_in), sqrt(6/fan_in)),
    drawn from the shared counter-based generator; zero biases;
  * ls_functional(): the least-squares functional of eq. LSfuncrowi at given
    weights, sigma - 2 p.b + p^T G p, used by the judge.
"""
from __future__ import annotations

import numpy as np

from paper_1004_1451_amd.chains import STREAM_MLP_INIT, uniform

D_IN, HID, D_OUT = 24, 64, 4
SHAPES = [("W1", (HID, D_IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (D_OUT, HID)), ("b3", (D_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)     # 6020


def unpack(theta: np.ndarray) -> dict:
    """Flat parameter vector -> named arrays (row-major, in SHAPES order)."""
    out, off = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights from u(seed, MLP_INIT, flat index); biases zero."""
    theta = np.zeros(N_PARAM)
    off = 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        if name.startswith("W"):
            fan_in = shp[1]
            u = uniform(seed, STREAM_MLP_INIT, np.arange(off, off + k, dtype=np.uint64))
            theta[off:off + k] = (2.0 * u - 1.0) * np.sqrt(6.0 / fan_in)
        off += k
    return theta


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to bfloat16 (nearest, ties to even), returned as
    float64.  The input is first taken to FP32, as the GPU holds it."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
    out = (rounded << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ----------------------------------------------------------------- features
# Offsets of the 8 operator-row features: Chebyshev-1 neighbours in
# lexicographic (da, db) order, the centre left out.
STENCIL_OFFSETS = [(da, db) for da in (-1, 0, 1) for db in (-1, 0, 1) if (da, db) != (0, 0)]


def features(G: np.ndarray, b: np.ndarray, sigma: float, valid: np.ndarray, stencil: np.ndarray) -> np.ndarray:
    """24 features of one fine point: [valid slot mask (4) | -b_ij / b_ii at the
    8 neighbour offsets (8) | b_s / G_ss (4) | b_s / sqrt(sigma G_ss) (4) |
    sqrt(G_ss / sigma) (4)]; the slot features are zero for empty slots.
    `stencil` holds -b_ij / b_ii in STENCIL_OFFSETS order (zero where the row
    has no entry)."""
    f = np.zeros(D_IN)
    f[0:4] = valid.astype(np.float64)
    f[4:12] = stencil
    for s in range(4):
        if not valid[s] or not (G[s, s] > 0) or not (sigma > 0):
            continue
        f[12 + s] = b[s] / G[s, s]
        f[16 + s] = b[s] / np.sqrt(sigma * G[s, s])
        f[20 + s] = np.sqrt(G[s, s] / sigma)
    return f


def ls_functional(G: np.ndarray, b: np.ndarray, sigma: float, p: np.ndarray) -> float:
    """sum_k w_k (x_i^k - sum_s p_s x_s^k)^2 written with the Gram."""
    return float(sigma - 2.0 * p @ b + p @ G @ p)


# ----------------------------------------------------------------- network
def forward(theta: np.ndarray, X: np.ndarray, bf16: bool = False):
    """Y = W3 relu(W2 relu(W1 X + b1) + b2) + b3 for the rows of X (n x 24).
    With bf16, the operands of every product (X, W, hidden activations) are
    rounded to bfloat16; sums and biases stay exact (FP64)."""
    P = unpack(theta)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x0 = r(X)
    z1 = x0 @ r(P["W1"]).T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    x1 = r(h1)
    z2 = x1 @ r(P["W2"]).T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    x2 = r(h2)
    y = x2 @ r(P["W3"]).T + P["b3"]
    return y, dict(x0=x0, z1=z1, x1=x1, z2=z2, x2=x2, P=P, r=r)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, M: np.ndarray, bf16: bool = False):
    """Masked mean squared error L = sum M (Y - T)^2 / max(1, sum M) and dL/dtheta.
    With bf16 the backward products take bfloat16 operands too (dY, dZ and
    the weights), as on the GPU."""
    y, c = forward(theta, X, bf16)
    r, P = c["r"], c["P"]
    cnt = max(1.0, float(M.sum()))
    diff = (y - T) * M
    L = float((diff * diff).sum() / cnt)
    dy = 2.0 * diff / cnt                         # n x 4
    g = {}
    dyr = r(dy)
    g["W3"] = dyr.T @ c["x2"]
    g["b3"] = dy.sum(axis=0)
    dh2 = dyr @ r(P["W3"])
    dz2 = dh2 * (c["z2"] > 0)
    dz2r = r(dz2)
    g["W2"] = dz2r.T @ c["x1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2r @ r(P["W2"])
    dz1 = dh1 * (c["z1"] > 0)
    dz1r = r(dz1)
    g["W1"] = dz1r.T @ c["x0"]
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------- data
def level_features(X: np.ndarray, w: np.ndarray, Bl, g):
    """Features of every point of a level from its test vectors X (n x R),
    weights w, operator Bl (CSR) and grid g, with the same slots and Gram as
    the oracle's ls_fit (Section 3.2).  Returns (F (n x 24), G, b, sigma,
    valid, isC); rows of C points are zero (they are not fitted)."""
    from oracle.bamg_oracle import c_points, is_c_point, neighbour_slots
    n = X.shape[0]
    slots = neighbour_slots(g)
    valid = slots >= 0
    isC = is_c_point(g)
    cpts = c_points(g)
    Xs = X[cpts[np.where(valid, slots, 0)]] * valid[:, :, None]
    G = np.einsum("pak,pbk,k->pab", Xs, Xs, w)
    b = np.einsum("pak,pk,k->pa", Xs, X, w)
    sigma = np.einsum("pk,pk,k->p", X, X, w)
    F = np.zeros((n, D_IN))
    F[:, 0:4] = valid
    # -b_ij / b_ii at the 8 neighbour offsets
    Bl = Bl.tocsr()
    rows = np.repeat(np.arange(n), np.diff(Bl.indptr))
    cols, vals = Bl.indices, Bl.data
    diag = np.zeros(n)
    on = rows == cols
    diag[rows[on]] = vals[on]
    off = ~on
    r_, c_, v_ = rows[off], cols[off], vals[off]
    da = c_ // g.ny - r_ // g.ny
    db = c_ % g.ny - r_ % g.ny
    if g.periodic:
        da = np.where(da > g.nx // 2, da - g.nx, np.where(da < -(g.nx // 2), da + g.nx, da))
        db = np.where(db > g.ny // 2, db - g.ny, np.where(db < -(g.ny // 2), db + g.ny, db))
    k = (da + 1) * 3 + (db + 1)
    k = np.where(k > 4, k - 1, k)                 # skip the centre
    F[r_, 4 + k] = -v_ / diag[r_]
    Gd = np.einsum("pss->ps", G)
    ok = valid & (Gd > 0) & (sigma[:, None] > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        F[:, 12:16] = np.where(ok, b / Gd, 0.0)
        F[:, 16:20] = np.where(ok, b / np.sqrt(sigma[:, None] * Gd), 0.0)
        F[:, 20:24] = np.where(ok, np.sqrt(Gd / sigma[:, None]), 0.0)
    F[isC] = 0.0
    return F, G, b, sigma, valid, isC


def slot_weights(P, g) -> np.ndarray:
    """Interpolation weights of every point in slot order (n x 4): entry s is
    P[i, N_i(s)] (zero for empty slots and for slots left out of J_i)."""
    from oracle.bamg_oracle import neighbour_slots
    slots = neighbour_slots(g)
    P = P.tocsr()
    out = np.zeros(slots.shape)
    for s in range(4):
        ok = slots[:, s] >= 0
        idx = np.nonzero(ok)[0]
        out[idx, s] = np.asarray(P[idx, slots[idx, s]]).ravel()
    return out
