"""Pins of the CPU oracle against facts that do not come from the oracle itself:
published generator outputs, dense textbook formulas, brute force on tiny
inputs, closed-form stationary vectors and the algebraic invariants the paper
states (Section 4: 1^T Q = 1^T, hence 1^T B_l = 0 on every level)."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


# --------------------------------------------------------------- generators
def test_splitmix64_published_outputs():
    # SplitMix64 reference outputs: seed 0 -> 0xE220A8397B1DCDAF; seed 1234567
    # -> 6457827717110365317, 3203168211198807973 (first two outputs).
    g = 0x9E3779B97F4A7C15
    m = (1 << 64) - 1
    # u = (h >> 11) 2^-53 with h = mix(key + GAMMA)
    u0 = O._splitmix_u01(0, 0, np.array([0], dtype=np.uint64))[0]
    assert u0 == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53
    # seed 1234567: consecutive states differ by GAMMA -> idx = 0 and GAMMA
    u = O._splitmix_u01(1234567, 0, np.array([0, g & m], dtype=np.uint64))
    assert u[0] == (6457827717110365317 >> 11) * 2.0 ** -53
    assert u[1] == (3203168211198807973 >> 11) * 2.0 ** -53
    # the generator module implements the same published definition
    assert C.uniform(1234567, 0, [0])[0] == u[0]


def test_tandem_counts_and_stochastic():
    ch = C.tandem_queue(32)
    assert ch.n == 1089 and ch.nnz == 3264
    A = ch.to_scipy()
    assert np.abs(np.asarray(A.sum(0)).ravel() - 1).max() < 1e-15
    B = O.b_from_a(A)
    assert B.nnz == 4225
    assert B.diagonal().min() >= 10 / 31 - 1e-15


def test_lattice_closed_form_is_stationary():
    ch = C.weighted_lattice(12, seed=3)
    A = ch.to_scipy()
    assert np.abs(A @ ch.exact - ch.exact).max() < 1e-15
    assert np.abs(np.asarray(A.sum(0)).ravel() - 1).max() < 1e-15


# --------------------------------------------------------------- grids
def test_coarse_positions_keep_both_ends():
    # Section 5 runs on sides 2^k + 1, where every other point keeps both ends
    # coarse; the reading keeps both ends coarse on every non-periodic side.
    for m in range(1, 40):
        want = sorted(set(range(0, m, 2)) | {m - 1})
        assert list(O.coarse_coords(m, False)) == want
        assert O.coarse_side(m, False) == m // 2 + 1
    for k in range(1, 8):
        m = 2 ** k + 1
        assert list(O.coarse_coords(m, False)) == list(range(0, m, 2))
    for m in (6, 8, 64, 1024):
        assert list(O.coarse_coords(m, True)) == list(range(0, m, 2))
    g = O.Grid(6, 9, False)
    isC = O.is_c_point(g).reshape(6, 9)
    assert [a for a in range(6) if isC[a, 0]] == [0, 2, 4, 5]
    assert [b for b in range(9) if isC[0, b]] == [0, 2, 4, 6, 8]
    # coarse index = rank of the coarse point in row-major order
    cp = O.c_points(g)
    assert np.all(np.diff(cp) > 0) and len(cp) == g.coarse().n == 4 * 5
    assert np.array_equal(np.nonzero(O.is_c_point(g))[0], cp)


def _slots_brute(g):
    """N_i by enumeration: coarse points within Chebyshev distance 1 of i
    that do not leave a direction in which i itself sits on a coarse line."""
    ca = set(O.coarse_coords(g.nx, g.periodic).tolist())
    cb = set(O.coarse_coords(g.ny, g.periodic).tolist())
    rank_a = {a: k for k, a in enumerate(sorted(ca))}
    rank_b = {b: k for k, b in enumerate(sorted(cb))}
    out = []
    for s in range(g.n):
        a, b = divmod(s, g.ny)
        want = []
        if not (a in ca and b in cb):
            for da, db in itertools.product((-1, 0, 1), repeat=2):
                if (da, db) == (0, 0):
                    continue
                if (a in ca and da != 0) or (b in cb and db != 0):
                    continue
                na, nb = a + da, b + db
                if g.periodic:
                    na %= g.nx; nb %= g.ny
                elif not (0 <= na < g.nx and 0 <= nb < g.ny):
                    continue
                if na in ca and nb in cb:
                    want.append(rank_a[na] * g.coarse().ny + rank_b[nb])
        out.append(want)
    return out


def test_neighbour_slots_brute_force():
    # grids whose coarse positions are the even ones: N_i is every coarse
    # point within Chebyshev distance 1 (the reading as first stated)
    for g in (O.Grid(7, 9, False), O.Grid(8, 6, True), O.Grid(5, 5, False)):
        slots = O.neighbour_slots(g)
        cg = g.coarse()
        for s in range(g.n):
            a, b = divmod(s, g.ny)
            want = []
            for da, db in itertools.product((-1, 0, 1), repeat=2):
                if (da, db) == (0, 0):
                    continue
                na, nb = a + da, b + db
                if g.periodic:
                    na %= g.nx; nb %= g.ny
                elif not (0 <= na < g.nx and 0 <= nb < g.ny):
                    continue
                if na % 2 == 0 and nb % 2 == 0 and not (a % 2 == 0 and b % 2 == 0):
                    want.append((na // 2) * cg.ny + nb // 2)
            got = [int(v) for v in slots[s] if v >= 0]
            assert got == want
    # even non-periodic sides (last position coarse too)
    for g in (O.Grid(8, 6, False), O.Grid(6, 9, False), O.Grid(4, 4, False), O.Grid(8, 6, True)):
        slots = O.neighbour_slots(g)
        for s, want in enumerate(_slots_brute(g)):
            assert [int(v) for v in slots[s] if v >= 0] == want
    # every F point has 2 or 4 slots, C points none
    g = O.Grid(10, 7, False)
    cnt = (O.neighbour_slots(g) >= 0).sum(1)
    isC = O.is_c_point(g)
    assert np.all(cnt[isC] == 0) and set(cnt[~isC].tolist()) <= {2, 4}


def _box_coarse_operator(g, slots, seed=0):
    """Q B P for a random 9-point B on grid g and a P with positive weights on
    the given slots (C points: unit rows); returns (Bc, Q, P, coarse grid)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for s in range(g.n):
        a, b = divmod(s, g.ny)
        for da, db in itertools.product((-1, 0, 1), repeat=2):
            na, nb = a + da, b + db
            if g.periodic:
                na %= g.nx; nb %= g.ny
            elif not (0 <= na < g.nx and 0 <= nb < g.ny):
                continue
            rows.append(s); cols.append(na * g.ny + nb)
            vals.append(4.0 if (da, db) == (0, 0) else -rng.random())
    B = sp.csr_matrix((vals, (rows, cols)), shape=(g.n, g.n))
    isC = O.is_c_point(g)
    cidx = np.cumsum(isC) - 1
    pr, pc, pv = [], [], []
    for s in range(g.n):
        if isC[s]:
            pr.append(s); pc.append(cidx[s]); pv.append(1.0)
            continue
        for J in slots[s]:
            if J >= 0:
                pr.append(s); pc.append(J); pv.append(0.1 + rng.random())
    P = sp.csr_matrix((pv, (pr, pc)), shape=(g.n, int(isC.sum())))
    Q = O.averaging_q(P)
    return O.galerkin(Q, B, P), Q, P, g.coarse()


def _in_box(M, cg):
    r, c = M.nonzero()
    da = np.abs(r // cg.ny - c // cg.ny)
    db = np.abs(r % cg.ny - c % cg.ny)
    if cg.periodic:
        da = np.minimum(da, cg.nx - da); db = np.minimum(db, cg.ny - db)
    return bool(np.all(da <= 1) and np.all(db <= 1))


def test_even_side_coarse_operators_keep_the_box():
    # Q, B and P each reach one grid step, so Q B P has a 3x3 coarse stencil
    # (every coarse operator of Sections 4-5 stays a 9-point operator)
    for g in (O.Grid(8, 6, False), O.Grid(6, 9, False), O.Grid(10, 10, False), O.Grid(9, 9, False),
              O.Grid(8, 8, True)):
        Bc, Q, P, cg = _box_coarse_operator(g, O.neighbour_slots(g))
        assert _in_box(Bc, cg)
        assert np.abs(np.asarray(Q.sum(0)).ravel() - 1).max() < 1e-15      # 1^T Q = 1^T
    # the plain Chebyshev-1 set next to the doubled coarse line would couple
    # coarse points two steps apart: the reason for the reading
    g = O.Grid(8, 8, False)
    ca = set(O.coarse_coords(8, False).tolist())
    rank = {a: k for k, a in enumerate(sorted(ca))}
    cheb = np.full((g.n, 4), -1)
    for s in range(g.n):
        a, b = divmod(s, g.ny)
        if a in ca and b in ca:
            continue
        k = 0
        for da, db in itertools.product((-1, 0, 1), repeat=2):
            na, nb = a + da, b + db
            if (da, db) != (0, 0) and 0 <= na < 8 and 0 <= nb < 8 and na in ca and nb in ca and k < 4:
                cheb[s, k] = rank[na] * 5 + rank[nb]; k += 1
    Bc, _, _, cg = _box_coarse_operator(g, cheb)
    assert not _in_box(Bc, cg)


def test_level_plan_configs():
    assert [g.n for g in O.level_plan(O.Grid(33, 33, False), 3)] == [1089, 289, 81]
    assert [g.nx for g in O.level_plan(O.Grid(1024, 1024, True), 5)] == [1024, 512, 256, 128, 64]
    assert [g.nx for g in O.level_plan(O.Grid(2048, 2048, False), 6)] == [2048, 1025, 513, 257, 129, 65]
    assert [g.nx for g in O.level_plan(O.Grid(129, 129, False), 6)] == [129, 65, 33, 17, 9, 5]
    with pytest.raises(ValueError):
        O.level_plan(O.Grid(10, 10, True), 3)     # 10 -> 5 is odd and periodic
    with pytest.raises(ValueError):
        O.level_plan(O.Grid(2, 2, False), 2)      # a side of two keeps both points
    assert not O.Grid(2, 2, False).can_coarsen() and O.Grid(3, 2, False).can_coarsen()


# --------------------------------------------------------------- relaxation
def test_jacobi_dense_formula():
    ch = C.tandem_queue(9)
    B = O.b_from_a(ch.to_scipy())
    X = np.random.default_rng(0).random((ch.n, 3))
    Bd = B.toarray()
    S = np.eye(ch.n) - 0.7 * np.diag(1 / np.diag(Bd)) @ Bd
    want = np.linalg.matrix_power(S, 3) @ X
    assert np.abs(O.jacobi(B, X, 0.7, 3) - want).max() < 1e-14
    f = np.random.default_rng(1).random(ch.n)
    e = np.zeros(ch.n)
    for _ in range(2):
        e = e + 0.7 * (f - Bd @ e) / np.diag(Bd)
    assert np.abs(O.jacobi(B, np.zeros(ch.n), 0.7, 2, F=f) - e).max() < 1e-14


def test_tv_weights_dense():
    ch = C.tandem_queue(7)
    B = O.b_from_a(ch.to_scipy())
    X = np.random.default_rng(2).random((ch.n, 4))
    want = 1 / np.linalg.norm(B.toarray() @ X, axis=0) ** 2
    assert np.allclose(O.tv_weights(B, X), want, rtol=1e-13)


# --------------------------------------------------------------- LS fit
def test_ls_fit_recovers_planted_weights():
    # TVs on the coarse points are random; F values are exact combinations of
    # their slots with planted weights, so the minimiser is the planted P.
    g = O.Grid(9, 8, False)
    rng = np.random.default_rng(4)
    R = 10
    X = rng.random((g.n, R)) + 0.5
    slots = O.neighbour_slots(g)
    cpts = O.c_points(g)
    isC = O.is_c_point(g)
    planted = np.zeros((g.n, 4))
    for i in np.nonzero(~isC)[0]:
        k = (slots[i] >= 0).sum()
        planted[i, :k] = rng.random(k) + 0.1
        X[i] = planted[i, :k] @ X[cpts[slots[i, :k]]]
    w = rng.random(R) + 0.5
    P, J, _ = O.ls_fit(X, w, g, caliber=4)
    for i in np.nonzero(~isC)[0]:
        k = (slots[i] >= 0).sum()
        row = P.getrow(i)
        got = dict(zip(row.indices, row.data))
        for s in range(k):
            assert abs(got[slots[i, s]] - planted[i, s]) < 1e-10
    for i in np.nonzero(isC)[0]:
        row = P.getrow(i)
        assert list(row.data) == [1.0]


def _brute_greedy(G, b, sigma, nslots, c):
    J = []
    while len(J) < c:
        best, bestL = None, np.inf
        for gi in range(nslots):
            if gi in J:
                continue
            S = sorted(J + [gi])
            # admissibility: Schur complement of gi w.r.t. J
            if J:
                piv = G[gi, gi] - G[gi, J] @ np.linalg.solve(G[np.ix_(J, J)], G[J, gi])
            else:
                piv = G[gi, gi]
            if piv <= 1e-10 * G[gi, gi]:
                continue
            # min_p L by weighted least squares on the raw data is checked
            # below; here the closed form
            L = sigma - b[S] @ np.linalg.solve(G[np.ix_(S, S)], b[S])
            if L < bestL:
                best, bestL = gi, L
        if best is None:
            break
        J.append(best)
    return sorted(J)


def test_ls_fit_greedy_brute_force_caliber2():
    g = O.Grid(7, 7, False)
    rng = np.random.default_rng(5)
    R = 6
    X = rng.random((g.n, R))
    w = rng.random(R) + 0.1
    P, J, slots = O.ls_fit(X, w, g, caliber=2)
    cpts = O.c_points(g)
    isC = O.is_c_point(g)
    for i in np.nonzero(~isC)[0]:
        k = int((slots[i] >= 0).sum())
        Xs = X[cpts[slots[i, :k]]]               # (k, R)
        G = (Xs * w) @ Xs.T
        bb = (Xs * w) @ X[i]
        sigma = (X[i] * w) @ X[i]
        want = _brute_greedy(G, bb, sigma, k, 2)
        got = sorted(np.nonzero(J[i])[0].tolist())
        assert got == want
        # the weights minimise the functional of eq. LSfuncrowi: weighted lstsq
        sw = np.sqrt(w)
        p_ls = np.linalg.lstsq((Xs[want] * sw).T, X[i] * sw, rcond=None)[0]
        row = P.getrow(i)
        got_w = dict(zip(row.indices, row.data))
        for s, pv in zip(want, p_ls):
            assert abs(got_w[slots[i, s]] - pv) < 1e-10


def test_ls_fit_greedy_order_matters_only_by_value():
    # caliber 1: the chosen slot is the argmin of the one-point functional
    g = O.Grid(5, 5, False)
    rng = np.random.default_rng(6)
    X = rng.random((g.n, 5))
    w = np.ones(5)
    P, J, slots = O.ls_fit(X, w, g, caliber=1)
    cpts = O.c_points(g)
    for i in np.nonzero(~O.is_c_point(g))[0]:
        k = int((slots[i] >= 0).sum())
        Ls = []
        for s in range(k):
            xs = X[cpts[slots[i, s]]]
            Ls.append(X[i] @ X[i] - (xs @ X[i]) ** 2 / (xs @ xs))
        assert np.nonzero(J[i])[0].tolist() == [int(np.argmin(Ls))]


# --------------------------------------------------------------- Q, Galerkin
def _small_level(N=12, r=6, seed=0):
    ch = C.tandem_queue(N)
    g = _grid(ch)
    B = O.b_from_a(ch.to_scipy())
    U = O.jacobi(B, O.initial_tvs(ch.n, r, seed), 0.7, 4)
    w = O.tv_weights(B, U)
    P, J, _ = O.ls_fit(U, w, g, 4)
    return ch, g, B, U, P


def test_averaging_q_invariants():
    ch, g, B, U, P = _small_level()
    Q = O.averaging_q(P)
    assert np.abs(np.asarray(Q.sum(0)).ravel() - 1).max() < 1e-15
    assert (Q.astype(bool) != P.T.astype(bool)).nnz == 0
    for i in range(P.shape[0]):
        col = Q.getcol(i).data
        assert np.all(col == col[0])


def test_galerkin_dense_and_zero_column_sums():
    ch, g, B, U, P = _small_level()
    Q = O.averaging_q(P)
    Bc = O.galerkin(Q, B, P)
    want = Q.toarray() @ B.toarray() @ P.toarray()
    assert np.abs(Bc.toarray() - want).max() < 1e-15
    assert np.abs(np.asarray(Bc.sum(0)).ravel()).max() < 1e-14 * abs(B).max()
    # coarse stencil lies within the coarse 3x3 box
    cg = g.coarse()
    r, c = Bc.nonzero()
    assert np.all(np.abs(r // cg.ny - c // cg.ny) <= 1) and np.all(np.abs(r % cg.ny - c % cg.ny) <= 1)
    # pattern is the symbolic product
    symb = (abs(Q).astype(bool).astype(int) @ abs(B).astype(bool).astype(int) @ abs(P).astype(bool).astype(int)).astype(bool)
    assert (symb != Bc.astype(bool)).nnz == 0 or Bc.nnz == symb.nnz
    Tc = O.galerkin(Q, sp.identity(ch.n, format="csr"), P)
    assert np.abs(Tc.toarray() - Q.toarray() @ P.toarray()).max() < 1e-15


def test_inject():
    g = O.Grid(5, 4, False)
    X = np.arange(20 * 3, dtype=float).reshape(20, 3)
    Xc = O.inject(X, g)
    # side 4 keeps positions 0, 2 and 3 (both ends), side 5 keeps 0, 2, 4
    want = np.array([X[a * 4 + b] for a in (0, 2, 4) for b in (0, 2, 3)])
    assert np.array_equal(Xc, want)


# --------------------------------------------------------------- coarsest
def _coarse_ops(N=16, levels=2):
    ch = C.tandem_queue(N)
    g = _grid(ch)
    B = O.b_from_a(ch.to_scipy())
    U = O.jacobi(B, O.initial_tvs(ch.n, 8, 0), 0.7, 4)
    lv = O.Level(g, B, sp.identity(ch.n, format="csr"))
    P, Q, J, Bc, Tc = O.build_level(lv, U, O.Options())
    return Bc.toarray(), Tc.toarray()


def test_coarsest_null_and_pinv():
    Bd, Td = _coarse_ops()
    y = O.coarsest_null(Bd, Td)
    assert np.abs(Bd @ y).max() < 1e-13 * np.abs(Bd).max() * np.abs(y).max()
    assert abs(np.ones(len(y)) @ Td @ y - 1) < 1e-13
    assert np.abs(O.coarsest_pinv(Bd) - np.linalg.pinv(Bd)).max() < 1e-8 * np.abs(np.linalg.pinv(Bd)).max()


def test_coarsest_eigs_dense_and_arpack_agree():
    Bd, Td = _coarse_ops(N=40)        # 21x21 = 441 coarse points
    n = Bd.shape[0]
    assert n > O.DENSE_EIG_MAX
    y, entries, V = O.coarsest_eigs(Bd, Td, 6)          # ARPACK path
    lam_all = sla.eigvals(Bd, Td)
    lam_sorted = lam_all[np.argsort(np.abs(lam_all))][1:]
    got = []
    for e in entries[1:]:
        got.append(e.lam)
        if len(e.cols) == 2:
            got.append(np.conj(e.lam))
    for lam in got:
        assert np.min(np.abs(lam_sorted - lam)) < 1e-10 * abs(lam) + 1e-14
    assert np.abs(np.abs(np.array(got)).max() - np.sort(np.abs(lam_sorted))[len(got) - 1]) < 1e-10
    for e in entries[1:]:
        v = V[:, e.cols[0]] + (1j * V[:, e.cols[1]] if len(e.cols) == 2 else 0)
        assert np.linalg.norm(Bd @ v - e.lam * (Td @ v)) < 1e-10 * np.linalg.norm(Bd, 1)
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        i = np.argmax(np.abs(v) ** 2)
        assert abs(v[i].imag) < 1e-14 and v[i].real > 0
    # the dense path on the same operator (forced)
    old = O.DENSE_EIG_MAX
    try:
        O.DENSE_EIG_MAX = 10 ** 6
        y2, entries2, V2 = O.coarsest_eigs(Bd, Td, 6)
    finally:
        O.DENSE_EIG_MAX = old
    assert len(entries2) == len(entries)
    for a, b in zip(entries, entries2):
        assert abs(a.lam - b.lam) <= 1e-9 * abs(b.lam) + 1e-15
    assert np.abs(np.abs(V) - np.abs(V2)).max() < 1e-6


def test_eig_relax_formula():
    Bd, Td = _coarse_ops()
    B, T = sp.csr_matrix(Bd), sp.csr_matrix(Td)
    rng = np.random.default_rng(7)
    V = rng.random((Bd.shape[0], 3))
    entries = [O.EigEntry(0.0, (0,)), O.EigEntry(0.01 + 0.002j, (1, 2))]
    V2, e2 = O.eig_relax(B, T, V, entries, 0.7, 1)
    x = V[:, 1] + 1j * V[:, 2]
    lam = 0.01 + 0.002j
    D = np.diag(Bd) - lam * np.diag(Td)
    x1 = x - 0.7 * ((Bd - lam * Td) @ x) / D
    assert np.abs(V2[:, 1] - x1.real).max() < 1e-14 and np.abs(V2[:, 2] - x1.imag).max() < 1e-14
    assert abs(e2[1].lam - (np.conj(x1) @ Bd @ x1) / (np.conj(x1) @ Td @ x1)) < 1e-14
    y1 = V[:, 0] - 0.7 * (Bd @ V[:, 0]) / np.diag(Bd)
    assert np.abs(V2[:, 0] - y1).max() < 1e-14 and e2[0].lam == 0


# --------------------------------------------------------------- cycles
def test_vcycle_equals_dense_error_propagator():
    # E = (I - M B)^nu2 (I - P B_c^+ Q B) (I - M B)^nu1 (eq. mgerrorprop, two
    # levels) must equal I - C B for the oracle's cycle C.
    ch = C.tandem_queue(10)
    h = O.setup(ch.to_scipy(), _grid(ch), 6, O.Options(levels=2))
    B = h.levels[0].B.toarray()
    P = h.levels[0].P.toarray(); Q = h.levels[0].Q.toarray()
    Bc = h.levels[1].B.toarray()
    n = B.shape[0]
    S = np.eye(n) - 0.7 * np.diag(1 / np.diag(B)) @ B
    E = S @ S @ (np.eye(n) - P @ np.linalg.pinv(Bc) @ Q @ B) @ S @ S
    Cmat = np.stack([O.vcycle(h, np.eye(n)[:, j]) for j in range(n)], axis=1)
    assert np.abs((np.eye(n) - Cmat @ B) - E).max() < 1e-10


def test_setup_invariants_every_level():
    ch = C.tandem_queue(32)
    h = O.setup(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3))
    for lv in h.levels:
        colsum = np.abs(np.asarray(lv.B.sum(0)).ravel()).max()
        assert colsum < 1e-13
    for lv in h.levels[:-1]:
        assert np.abs(np.asarray(lv.Q.sum(0)).ravel() - 1).max() < 1e-15
        # C rows of P are unit rows
        isC = O.is_c_point(lv.grid)
        for i in np.nonzero(isC)[0][:50]:
            row = lv.P.getrow(i)
            assert list(row.data) == [1.0]


# --------------------------------------------------------------- end to end
def test_stationary_tandem_c0_vs_dense_null_vector():
    ch = C.tandem_queue(32)
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3), tol=1e-14)
    assert info.converged
    B = O.b_from_a(ch.to_scipy()).toarray()
    ns = sla.null_space(B)[:, 0]
    ns = ns / ns.sum()
    assert np.abs(x - ns).sum() < 1e-12
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-15


def test_stationary_lattice_closed_form():
    ch = C.weighted_lattice(32, seed=5)
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3), tol=1e-14)
    assert info.converged
    assert np.abs(x - ch.exact).sum() < 1e-12


def test_stationary_uniform_network_closed_form():
    # the paper's uniform network (Section 5, Table 1): x proportional to the
    # out-degree of every state
    ch = C.weighted_lattice(17, periodic=False, uniform_weights=True)
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 6, O.Options(levels=3), tol=1e-13)
    assert info.converged
    assert np.abs(x - ch.exact).sum() < 1e-11


@pytest.mark.parametrize("N", [127, 511])
def test_cycle_counts_stay_flat_on_even_sides(N):
    # Section 5, Tables 1-2: the number of cycles stays roughly constant as
    # the grid grows; an even side (N + 1) must not cost more than the odd
    # side next to it by more than two cycles, and six levels on side 1024
    # reach 1e-10 within ten cycles
    counts = []
    for M in (N, N + 1):
        ch = C.tandem_queue(M)
        _, info, h = O.stationary(ch.to_scipy(), _grid(ch), 12, O.Options(levels=6), tol=1e-10)
        assert info.converged
        counts.append(info.cycles)
    assert counts[0] <= counts[1] + 2 and counts[0] <= 10, counts


def test_tv_weights_floor_for_null_vectors():
    # omega_k = 1 / max(||B x_k||^2, (1e-14 ||x_k||)^2): a vector B maps to
    # zero exactly (a symmetric two-state chain and the constant vector) gets
    # the floor's finite weight, a scaled copy the same weight over c^2, and
    # an ordinary vector the plain inverse squared residual
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[0.5, 0.5], [0.5, 0.5]]))
    B = O.b_from_a(A)
    X = np.array([[1.0, 3.0, 1.0], [1.0, 3.0, 0.0]])
    w = O.tv_weights(B, X)
    assert np.all(np.abs(B @ X[:, :2]) == 0.0)
    assert w[0] == 1.0 / (1e-28 * 2.0)
    assert w[1] == 1.0 / (1e-28 * 18.0)
    r = B.toarray() @ X[:, 2]
    assert w[2] == 1.0 / float(r @ r)
