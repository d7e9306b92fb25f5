"""Pins of the oracle's multilevel eigensolver cycle (Algorithm 3) with cycle
index mu and of the MLE iteration used as a stand-alone solver (Section 4.1):
the recursion visits the coarsest level mu^(L) times, the two-level W-cycle
equals the steps of Algorithm 3 written out by hand from the (separately
pinned) primitives, and the iteration reaches the dense null vector and the
closed-form stationary vector."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


@pytest.mark.parametrize("mu,levels,visits", [(1, 3, 1), (2, 3, 4), (2, 4, 8), (1, 4, 1)])
def test_coarsest_visits(monkeypatch, mu, levels, visits):
    calls = []
    real = O.coarsest_eigs

    def counting(*a, **k):
        calls.append(1)
        return real(*a, **k)
    monkeypatch.setattr(O, "coarsest_eigs", counting)
    ch = C.tandem_queue(32)
    plan, lv = O._first_level(ch.to_scipy(), _grid(ch), 6, O.Options(levels=levels, mu=mu))
    O.mle_cycle(lv, 0, plan, O.Options(levels=levels, mu=mu), use_v=False)
    assert len(calls) == visits


def test_two_level_w_cycle_by_hand():
    ch = C.tandem_queue(16)
    opts = O.Options(levels=2, mu=2)
    plan, lv = O._first_level(ch.to_scipy(), _grid(ch), 6, opts)
    O.mle_cycle(lv, 0, plan, opts, use_v=False)
    # Algorithm 3 with mu = 2 on two levels, step by step
    B0 = O.b_from_a(ch.to_scipy())
    T0 = sp.identity(ch.n, format="csr")
    top = O.Level(plan[0], B0, T0)
    U = O.jacobi(B0, O.initial_tvs(ch.n, 6, 0), 0.7, 4)
    V = None
    for m in range(2):
        X = U if m == 0 else np.concatenate([U, V], axis=1)
        P, Q, J, Bc, Tc = O.build_level(top, X, opts)
        _, ents, Vc = O.coarsest_eigs(Bc.toarray(), Tc.toarray(), 6)
        V, ents = O.eig_relax(B0, T0, P @ Vc, ents, 0.7, 4)
    assert np.array_equal(lv[0].U, U)
    assert (abs(lv[0].P - P)).max() == 0.0
    assert np.array_equal(lv[0].V, V)


@pytest.mark.parametrize("mu", [1, 2])
def test_mle_iteration_reaches_the_null_vector(mu):
    ch = C.tandem_queue(16)
    x, info, _ = O.mle_iteration(ch.to_scipy(), _grid(ch), 6, O.Options(levels=3, mu=mu), tol=1e-11,
                                 max_cycles=80)
    assert info.converged
    ns = sla.null_space(O.b_from_a(ch.to_scipy()).toarray())[:, 0]
    assert np.abs(x - ns / ns.sum()).sum() < 1e-9
    h = np.array(info.history)
    assert np.all(h[1:] < h[:-1])            # every cycle improves the iterate here


def test_mle_iteration_closed_form():
    ch = C.weighted_lattice(32, seed=5)
    x, info, _ = O.mle_iteration(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3, mu=2), tol=1e-11, max_cycles=40)
    assert info.converged
    assert np.abs(x - ch.exact).sum() < 1e-9


@pytest.mark.parametrize("N", [127, 255])
def test_mle_iteration_converges_on_even_sided_six_level_tandems(N):
    # Section 4.1 / Table 2: the MLE iteration converges in a roughly constant
    # number of cycles as the grid grows; on sides 128 and 256 (even, not
    # periodic) with six levels it must reach the paper's 1e-8
    ch = C.tandem_queue(N)
    x, info, _ = O.mle_iteration(ch.to_scipy(), _grid(ch), 12, O.Options(levels=6), tol=1e-8, max_cycles=25)
    assert info.converged and info.cycles <= 20, (info.cycles, info.history)
