"""Pins of the oracle's coarsening without a grid (Section 3.1, Algorithm 1;
eq. neighbor_def) and of the unstructured planar graph workload (Section 5,
Table 4): brute force over every independent set of tiny graphs, the exact
F-relaxation factors of cycle graphs, a hand-derived run of Algorithm 1,
matrix-power reachability, weighted least squares by a library routine, and
the closed-form stationary vector of a random walk on an undirected graph."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C


def _cycle_b(n):
    """B = I - A for the random walk on a cycle of n states (a_ij = 1/2)."""
    i = np.arange(n)
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([i, (i + 1) % n, (i - 1) % n])
    vals = np.concatenate([np.ones(n), -0.5 * np.ones(n), -0.5 * np.ones(n)])
    B = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    B.sort_indices()
    return B


def _random_graph(n, p, rng):
    M = rng.random((n, n)) < p
    M = np.triu(M, 1)
    M = M | M.T
    return sp.csr_matrix(M)


# ------------------------------------------------------- independent sets
@pytest.mark.parametrize("seed", range(6))
def test_independent_set_is_lexicographically_first_maximal(seed):
    rng = np.random.default_rng(seed)
    n = 10
    G = _random_graph(n, 0.3, rng)
    cand = rng.random(n) < 0.8
    D = G.toarray()
    got = O.independent_set(G, cand)
    # brute force: every subset of the candidates that is independent and
    # maximal within them; the greedy in index order takes the one whose
    # indicator vector is largest in lexicographic order
    cidx = np.nonzero(cand)[0]
    best = None
    for bits in itertools.product([1, 0], repeat=len(cidx)):
        S = cidx[np.array(bits, dtype=bool)]
        if D[np.ix_(S, S)].any():
            continue
        inS = np.zeros(n, dtype=bool); inS[S] = True
        maximal = all(inS[i] or D[i, S].any() for i in cidx)
        if not maximal:
            continue
        key = tuple(inS.astype(int))
        if best is None or key > best:
            best = key
    assert tuple(got.astype(int)) == best


def test_independent_set_empty_and_isolated():
    G = sp.csr_matrix((5, 5), dtype=bool)
    assert O.independent_set(G, np.zeros(5, dtype=bool)).sum() == 0
    assert O.independent_set(G, np.ones(5, dtype=bool)).all()


# ------------------------------------------------------- F-relaxation, CR
def test_f_relax_isolated_f_points_exact_factor():
    # every other point coarse on a cycle: B_FF = I, so each sweep multiplies
    # u_F by 1 - omega exactly
    n, omega = 16, 0.7
    B = _cycle_b(n)
    isC = np.arange(n) % 2 == 0
    u0 = np.where(isC, 0.0, 1.0 + np.arange(n) / n)
    prev, last = O.f_relax(B, isC, u0, omega, 8)
    assert np.allclose(last[~isC], (1 - omega) ** 8 * u0[~isC], rtol=1e-14, atol=0)
    assert np.allclose(prev[~isC], (1 - omega) ** 7 * u0[~isC], rtol=1e-14, atol=0)
    assert not last[isC].any()


def test_f_relax_rate_of_path_blocks():
    # every fifth point coarse: B_FF has blocks tridiag(-1/2, 1, -1/2) of
    # size 4, so E_F = I - omega B_FF has spectral radius
    # 1 - omega (1 - cos(pi/5)); many sweeps reach it
    n, omega = 20, 0.7
    B = _cycle_b(n)
    isC = np.arange(n) % 5 == 0
    u0 = np.where(isC, 0.0, 1.0 + (np.arange(n) % 3) / 3)
    prev, last = O.f_relax(B, isC, u0, omega, 400)
    rho = 1 - omega * (1 - np.cos(np.pi / 5))
    F = ~isC
    assert np.allclose(np.abs(last[F]) / np.abs(prev[F]), rho, rtol=1e-12)


def test_cr_adds_independent_slow_points_and_stops():
    # Algorithm 1 by hand on a cycle of 20 with C_0 = every fifth point and
    # theta = 0.8: the F blocks of four relax at ~0.866 > theta, every F point
    # passes the ratio test, and the independent set of them (index order)
    # takes the first and third point of each block; what remains is
    # isolated F points, which relax at exactly 1 - omega = 0.3
    n = 20
    B = _cycle_b(n)
    C0 = np.arange(n) % 5 == 0
    isC, rounds, rhos = O.cr_coarsen(B, 0, 0.7, 0.8, 8, 0, 64, C0=C0)
    want = np.isin(np.arange(n) % 5, [0, 1, 3])
    assert (isC == want).all()
    assert rounds == 2
    assert 0.8 < rhos[0] <= 1 - 0.7 * (1 - np.cos(np.pi / 5)) + 1e-12
    assert abs(rhos[1] - 0.3) < 1e-14


def test_cr_default_start_is_independent_set_of_all_points():
    # every other point of an even cycle: F points isolated, rho = 0.3 <= theta
    B = _cycle_b(12)
    isC, rounds, rhos = O.cr_coarsen(B, 0, 0.7, 0.85, 8, 3, 64)
    assert (isC == (np.arange(12) % 2 == 0)).all()
    assert rounds == 1 and abs(rhos[0] - 0.3) < 1e-14


def test_cr_estimate_from_the_published_generator():
    # round 0 at level 2 with seed 7: u^0_i = 1 + u(7, 16 + 2, i) on F, and
    # rho_f = (||E_F^8 u^0|| / ||u^0||)^(1/8) with the dense E_F = I - omega
    # D_FF^-1 B_FF (eq. meas1); theta = 0.99 ends the loop after it
    n, omega = 20, 0.7
    B = _cycle_b(n)
    C0 = np.arange(n) % 5 == 0
    F = ~C0
    u = 1.0 + C.uniform(7, 16 + 2, np.arange(n))[F]
    E = np.eye(F.sum()) - omega * B.toarray()[np.ix_(F, F)]
    want = (np.linalg.norm(np.linalg.matrix_power(E, 8) @ u) / np.linalg.norm(u)) ** (1 / 8)
    isC, rounds, rhos = O.cr_coarsen(B, 2, omega, 0.99, 8, 7, 64, C0=C0)
    assert rounds == 1 and (isC == C0).all()
    assert abs(rhos[0] - want) < 1e-14


def test_graph_of_rejects_unsymmetric_pattern():
    B = sp.csr_matrix(np.array([[1.0, -1.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 1.0]]))
    with pytest.raises(ValueError):
        O.graph_of(B)


# ------------------------------------------------------- N_i by distance
@pytest.mark.parametrize("z", [1, 2, 3])
def test_graph_slots_match_matrix_powers(z):
    rng = np.random.default_rng(11 + z)
    n = 30
    G = _random_graph(n, 0.12, rng).astype(float)
    B = sp.csr_matrix(sp.identity(n) * 3.0 - G)
    isC = rng.random(n) < 0.35
    slots = O.graph_slots(B, isC, z)
    # reachable in <= z steps: (I + G)^z > 0, minus i itself
    M = np.linalg.matrix_power(np.eye(n) + G.toarray(), z) > 0
    cidx = np.cumsum(isC) - 1
    for i in range(n):
        want = [cidx[j] for j in range(n) if j != i and M[i, j] and isC[j]]
        got = [s for s in slots[i] if s >= 0]
        assert got == want


# ------------------------------------------------------- LS fit on lists
def test_ls_fit_on_candidate_lists_greedy_steps_are_optimal():
    # K = 7 candidates per point, caliber 4: each greedy step takes the
    # candidate whose addition minimises eq. LSfuncrowi, evaluated here by a
    # weighted least-squares library solve; the weights are that solve's
    rng = np.random.default_rng(21)
    n, nc, K, R = 40, 12, 7, 9
    isC = np.zeros(n, dtype=bool); isC[:nc] = True
    cpts = np.arange(nc)
    slots = np.full((n, K), -1)
    for i in range(nc, n):
        k = rng.integers(1, K + 1)
        slots[i, :k] = np.sort(rng.choice(nc, size=k, replace=False))
    cs = O.Coarsening(isC, cpts, slots)
    X = rng.random((n, R))
    w = rng.random(R) + 0.2
    P, J, _, steps = O.ls_fit(X, w, cs, 4, order=True)
    sw = np.sqrt(w)

    def L_of(i, S):
        A = (X[cpts[slots[i, S]]] * sw).T
        p = np.linalg.lstsq(A, X[i] * sw, rcond=None)[0]
        return np.sum((X[i] * sw - A @ p) ** 2), p

    for i in range(nc, n):
        k = int((slots[i] >= 0).sum())
        chosen = []
        for st in steps[i]:
            if st < 0:
                break
            Ls = {g: L_of(i, chosen + [g])[0] for g in range(k) if g not in chosen}
            assert Ls[st] <= min(Ls.values()) * (1 + 1e-9) + 1e-14
            chosen.append(int(st))
        assert len(chosen) == min(k, 4)
        _, p = L_of(i, sorted(chosen))
        row = P.getrow(i)
        got = dict(zip(row.indices, row.data))
        for s, pv in zip(sorted(chosen), p):
            assert abs(got[slots[i, s]] - pv) < 1e-9
    for i in range(nc):
        row = P.getrow(i)
        assert row.indices.tolist() == [i] and row.data.tolist() == [1.0]


def test_ls_fit_grid_and_list_forms_agree():
    # a Grid and the same splitting given as lists select the same P
    g = O.Grid(9, 9, False)
    rng = np.random.default_rng(2)
    X = rng.random((g.n, 6))
    w = rng.random(6) + 0.1
    P1, J1, _ = O.ls_fit(X, w, g, 4)
    P2, J2, _ = O.ls_fit(X, w, O.grid_coarsening(g), 4)
    assert (P1 != P2).nnz == 0 and (J1 == J2).all()


# ------------------------------------------------------- the UPG workload
def test_upg_generator_is_a_reversible_planar_walk():
    ch = C.upg(300, seed=4)
    A = ch.to_scipy()
    assert ch.nx == 0 and ch.ny == 0
    assert np.abs(np.asarray(A.sum(0)).ravel() - 1).max() < 1e-15
    pat = A.astype(bool)
    assert (pat != pat.T).nnz == 0
    # a planar triangulation has at most 3 n - 6 edges
    assert A.nnz // 2 <= 3 * ch.n - 6
    assert np.abs(A @ ch.exact - ch.exact).max() < 1e-17


def test_upg_setup_invariants():
    ch = C.upg(512, seed=1)
    h = O.setup(ch.to_scipy(), None, 6, O.Options(levels=3))
    assert len(h.levels) == 3
    for lv in h.levels:
        assert np.abs(np.asarray(lv.B.sum(0)).ravel()).max() < 1e-13
        O.graph_of(lv.B)                     # coarse patterns stay symmetric
    for lv in h.levels[:-1]:
        cs = lv.cs
        G = O.graph_of(lv.B)
        # C_0 is maximal: every F point has a C neighbour, so N_i is not empty
        F = ~cs.isC
        assert (G[F][:, cs.isC].sum(1) > 0).all()
        assert np.abs(np.asarray(lv.Q.sum(0)).ravel() - 1).max() < 1e-15
        assert lv.P.shape == (lv.B.shape[0], cs.nc)
        # the last CR estimate met theta (or the round limit was hit)
        assert cs.rho[-1] <= 0.85 or cs.rounds == 64


@pytest.mark.parametrize("N", [256, 1024])
def test_upg_stationary_closed_form(N):
    ch = C.upg(N, seed=0)
    x, info, h = O.stationary(ch.to_scipy(), None, 6, O.Options(levels=3), tol=1e-13)
    assert info.converged
    assert np.abs(x - ch.exact).sum() < 1e-11


def test_upg_mle_iteration_cycle_counts_near_table_4():
    # Table 4 prints 15 and 20 MLE cycles for N = 256 and 1024 (different
    # random graphs); the iteration here needs a similar number
    for N in (256, 1024):
        ch = C.upg(N, seed=0)
        x, info, _ = O.mle_iteration(ch.to_scipy(), None, 6, O.Options(levels=3), tol=1e-8, max_cycles=40)
        assert info.converged and 10 <= info.cycles <= 25
        assert np.abs(x - ch.exact).sum() < 1e-6
