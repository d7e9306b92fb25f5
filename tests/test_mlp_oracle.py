"""Pins of the learned-form oracle (oracle/mlp_oracle.py), all on the CPU.

Each check ties the oracle to something outside itself: central finite
differences for the backward pass, torch's own float32 -> bfloat16 conversion
for the rounding, the closed form of Adam's first step, the defining scale
invariances of the features, and the least-squares fit itself where a point has
a single slot (its one-point weight b_s / G_ss is then the fitted weight).
"""
import numpy as np
import pytest

from oracle import bamg_oracle as O
from oracle import mlp_oracle as M
from paper_1004_1451_amd import chains as C


def _batch(n=37, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, M.D_IN))
    T = rng.normal(size=(n, M.D_OUT))
    Mk = (rng.random((n, M.D_OUT)) < 0.7).astype(float)
    return X, T, Mk


def test_param_layout_and_init():
    assert M.N_PARAM == 64 * 24 + 64 + 64 * 64 + 64 + 4 * 64 + 4 == 6020
    th = M.init_params(3)
    P = M.unpack(th)
    for name, fan in (("W1", 24), ("W2", 64), ("W3", 64)):
        lim = np.sqrt(6.0 / fan)
        assert np.abs(P[name]).max() <= lim and np.abs(P[name]).max() > 0.9 * lim
    for name in ("b1", "b2", "b3"):
        assert not P[name].any()
    assert np.array_equal(M.init_params(3), th) and not np.array_equal(M.init_params(4), th)
    assert np.array_equal(M.pack(P), th)


def test_gradient_matches_central_differences():
    X, T, Mk = _batch()
    th = M.init_params(7)
    th += 0.05 * np.random.default_rng(2).normal(size=th.size)     # non-zero biases
    L, g = M.loss_and_grad(th, X, T, Mk)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(th.size, 60, replace=False),
                          [0, 64 * 24, 64 * 24 + 64, 6020 - 5, 6020 - 1]])
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (M.loss_and_grad(tp, X, T, Mk)[0] - M.loss_and_grad(tm, X, T, Mk)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_masked_loss_ignores_masked_outputs():
    X, T, Mk = _batch()
    th = M.init_params(1)
    L1, g1 = M.loss_and_grad(th, X, T, Mk)
    T2 = T + 100.0 * (1 - Mk)            # change only masked targets
    L2, g2 = M.loss_and_grad(th, X, T2, Mk)
    assert L1 == L2 and np.array_equal(g1, g2)
    y, _ = M.forward(th, X)
    assert abs(L1 - ((y - T) ** 2 * Mk).sum() / Mk.sum()) <= 1e-12 * L1


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-30, 30, 1000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0, 65504.0]])
    x32 = x.astype(np.float32)
    want = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x32), want)


def test_bf16_gradient_is_close_to_exact():
    X, T, Mk = _batch(n=256)
    th = M.init_params(9)
    L, g = M.loss_and_grad(th, X, T, Mk)
    Lb, gb = M.loss_and_grad(th, X, T, Mk, bf16=True)
    assert abs(Lb - L) <= 0.05 * L
    for name, a, b in zip([n for n, _ in M.SHAPES], M.unpack(g).values(), M.unpack(gb).values()):
        assert np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(a), name


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.normal(size=10)
    g = rng.normal(size=10)
    t1, m, v = M.adam_step(th, np.zeros(10), np.zeros(10), g, 1, lr=1e-3)
    # bias-corrected moments of the first step are g and g^2
    assert np.allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def _level0(N=31, r=8, seed=0):
    ch = C.tandem_queue(N)
    Bl = O.b_from_a(ch.to_scipy())
    g = O.Grid(ch.nx, ch.ny, ch.periodic)
    U = O.jacobi(Bl, O.initial_tvs(ch.n, r, seed), 0.7, 4)
    w = O.tv_weights(Bl, U)
    return ch, Bl, g, U, w


def test_features_are_scale_free():
    ch, Bl, g, U, w = _level0()
    F, *_ = M.level_features(U, w, Bl, g)
    # rescale every test vector (weights rescale with them) and every row of B
    c = np.linspace(0.5, 3.0, U.shape[1])
    U2 = U * c
    rs = 1.0 + np.arange(ch.n) % 5
    import scipy.sparse as sp
    B2 = sp.diags(rs) @ Bl
    w2 = O.tv_weights(B2, U2)
    F2, *_ = M.level_features(U2, w2, B2, g)
    # row scaling changes w (all by the same law), not the ratios
    assert np.abs(F2[:, :12] - F[:, :12]).max() <= 1e-12
    Fw, *_ = M.level_features(U2, O.tv_weights(Bl, U2), Bl, g)
    assert np.abs(Fw - F).max() <= 1e-9 * max(1.0, np.abs(F).max())


def test_one_slot_feature_is_the_least_squares_weight():
    ch, Bl, g, U, w = _level0(N=31)
    F, G, b, sigma, valid, isC = M.level_features(U, w, Bl, g)
    # caliber 1: every F point interpolates from the one slot Algorithm 2
    # picks, with the one-point least-squares weight b_s / G_ss
    P1, J1, _ = O.ls_fit(U, w, g, 1)
    W1 = M.slot_weights(P1, g)
    idx = np.nonzero(~isC)[0]
    assert np.all(J1[idx].sum(1) == 1)
    s = np.argmax(J1[idx], axis=1)
    assert np.allclose(F[idx, 12 + s], W1[idx, s], rtol=1e-12, atol=0)
    P, J, slots = O.ls_fit(U, w, g, 4)
    Ws = M.slot_weights(P, g)
    # the functional at the fitted weights is the fit's minimum, below the
    # value at any one-slot weight
    i = np.nonzero((~isC) & (valid.sum(1) == 4))[0][0]
    Lfit = M.ls_functional(G[i], b[i], sigma[i], Ws[i])
    for t in range(4):
        p = np.zeros(4)
        p[t] = b[i][t] / G[i][t, t]
        assert Lfit <= M.ls_functional(G[i], b[i], sigma[i], p) + 1e-12 * sigma[i]
    assert Lfit >= -1e-12 * sigma[i]


def test_stencil_features_by_geometric_offset():
    # one stored off-diagonal entry per row, at a known offset (da, db) in the
    # 3 x 3 box; its -b_ij / b_ii must land in the feature the offset names:
    # features 4..11 are the offsets in row-major order without the centre
    import scipy.sparse as sp
    order = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
    for periodic in (False, True):
        g = O.Grid(7, 6, periodic)
        n = g.n
        isC = O.is_c_point(g)
        X = np.random.default_rng(5).random((n, 3)) + 0.5
        w = np.ones(3)
        for f_idx, (da, db) in enumerate(order):
            rows, cols, vals = [], [], []
            for p in range(n):
                a, b = divmod(p, g.ny)
                a2, b2 = a + da, b + db
                if periodic:
                    a2, b2 = a2 % g.nx, b2 % g.ny
                rows.append(p); cols.append(p); vals.append(2.0 + p % 3)
                if 0 <= a2 < g.nx and 0 <= b2 < g.ny:
                    rows.append(p); cols.append(a2 * g.ny + b2); vals.append(-0.25 - 0.01 * (p % 7))
            Bm = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
            F, *_ = M.level_features(X, w, Bm, g)
            for p in np.nonzero(~isC)[0]:
                a, b = divmod(p, g.ny)
                inside = periodic or (0 <= a + da < g.nx and 0 <= b + db < g.ny)
                want = np.zeros(8)
                if inside:
                    want[f_idx] = (0.25 + 0.01 * (p % 7)) / (2.0 + p % 3)
                assert np.allclose(F[p, 4:12], want, rtol=1e-15, atol=0), (periodic, (da, db), p)
