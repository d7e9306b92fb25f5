"""GPU parity at the full size of the headline workload: the tandem queue
N = 2047 (n = 4,194,304), r = 12 test vectors, 6 levels (2048^2 -> ... ->
65^2), in the form bench.py times (and in FP64).

Every step of the setup is checked element by element against the oracle
applied to the GPU's own inputs of that step (the same comparisons as
test_gpu_parity.py, at full size): initial test vectors bit-exact, Jacobi
sweeps <= 1e-13 of max |U|, P patterns exact and weights <= 1e-9, Galerkin
patterns exact and rows <= 1e-12 of the row maximum, injection exact, the
65 x 65 coarsest pseudo-inverse <= 1e-8 and its eigenpairs (FP64 path); one
V-cycle of the whole hierarchy <= 1e-9 (FP64); the mixed form's steps within
FP32 rounding (<= 1e-5 relative); the solutions satisfy x >= 0, sum x = 1
and ||Bx||_1/||x||_1 <= 1e-10 by a host SpMV, and the mixed and FP64
solutions agree.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU, skipped there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402

N, R, LEVELS = 2047, 12, 6


@pytest.fixture(scope="module")
def chain():
    ch = C.tandem_queue(N)
    return ch, B.device_csr(ch), O.b_from_a(ch.to_scipy())


def _hier(chain, **kw):
    ch, (rp, ci, v), _ = chain
    return B.Hierarchy(ch.n, rp, ci, v, (ch.nx, ch.ny, 0), R, B.default_options(levels=LEVELS, **kw))


def _csr(h, l, which):
    li = h.level_info(l)
    if which == "B":
        rp, ci, v = h.export(l, B.X_B_ROWPTR), h.export(l, B.X_B_COL), h.export(l, B.X_B_VAL)
    else:
        rp, ci, v = h.export(l, B.X_T_ROWPTR), h.export(l, B.X_T_COL), h.export(l, B.X_T_VAL)
    return sp.csr_matrix((v, ci, rp), shape=(li.n, li.n))


def _p(h, l, nc):
    pc = h.export(l, B.X_P_COL).reshape(-1, 4)
    pv = h.export(l, B.X_P_VAL).reshape(-1, 4)
    ok = pc >= 0
    rows = np.repeat(np.arange(pc.shape[0]), 4).reshape(-1, 4)[ok]
    P = sp.csr_matrix((pv[ok], (rows, pc[ok])), shape=(pc.shape[0], nc))
    P.sort_indices()
    return P


def _same_pattern(A, Bm):
    A = A.tocsr(); Bm = Bm.tocsr()
    A.sort_indices(); Bm.sort_indices()
    return np.array_equal(A.indptr, Bm.indptr) and np.array_equal(A.indices, Bm.indices)


def _rowrel(A, Bm):
    D = abs(A - Bm).tocsr()
    rmax = np.maximum(np.asarray(abs(Bm).max(axis=1).todense()).ravel(), 1e-300)
    return float(np.max(np.asarray(D.max(axis=1).todense()).ravel() / rmax))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fullsize_downleg_matches_oracle(chain, precision):
    ch, _, B0 = chain
    mixed = precision == "mixed"
    print(f"case full-size down-leg {precision}", flush=True)
    h = _hier(chain, precision=B.MIXED if mixed else B.FP64, stop_after=1)
    plan = O.level_plan(O.Grid(ch.nx, ch.ny, False), LEVELS)
    assert [h.level_info(l).n for l in range(LEVELS)] == [g.n for g in plan]
    U0 = h.export(0, B.X_U0).reshape(ch.n, R)
    want0 = O.initial_tvs(ch.n, R, 0)
    if mixed:           # the FP32 form stores the generator's values rounded to FP32
        want0 = want0.astype(np.float32).astype(np.float64)
    assert np.array_equal(U0, want0)
    # the FP32 form rounds every sweep and stores P, B, T in FP32
    tol_relax, tol_p, tol_gal = (1e-5, 1e-6, 1e-6) if mixed else (1e-13, 1e-9, 1e-12)
    Bl, Tl, Uin = B0, sp.identity(ch.n, format="csr"), U0
    for l in range(LEVELS - 1):
        g = plan[l]
        U = h.export(l, B.X_U).reshape(g.n, R)
        want = O.jacobi(Bl, Uin, 0.7, 4)
        assert np.abs(U - want).max() <= tol_relax * np.abs(want).max(), l
        w = O.tv_weights(Bl, U)
        Po, _, _ = O.ls_fit(U, w, g, 4)
        Pg = _p(h, l, g.coarse().n)
        assert _same_pattern(Pg, Po), l
        assert np.abs((Pg - Po).data).max() <= tol_p * max(1.0, np.abs(Po.data).max()), l
        Q = O.averaging_q(Pg)
        Bc, Tc = _csr(h, l + 1, "B"), _csr(h, l + 1, "T")
        Bo, To = O.galerkin(Q, Bl, Pg), O.galerkin(Q, Tl, Pg)
        assert _same_pattern(Bc, Bo) and _same_pattern(Tc, To), l
        assert _rowrel(Bc, Bo) <= tol_gal and _rowrel(Tc, To) <= tol_gal, l
        Uin = O.inject(U, g)
        if l + 1 == LEVELS - 1:
            assert np.array_equal(h.export(l + 1, B.X_U).reshape(-1, R), Uin)
        Bl, Tl = Bc, Tc
        print(f"  level {l}: n={g.n} P, B, T ok", flush=True)
    h.close()


def test_fullsize_coarsest_matches_oracle(chain):
    print("case full-size coarsest (65 x 65, bordered)", flush=True)
    h = _hier(chain, precision=B.FP64, stop_after=2)
    L = LEVELS - 1
    BL = _csr(h, L, "B").toarray()
    TL = _csr(h, L, "T").toarray()
    nL = BL.shape[0]
    assert nL == 65 * 65
    svd = O.coarsest_svd(BL)
    Wo = O.coarsest_pinv(BL, svd)
    W = h.export(L, B.X_W).reshape(nL, nL)
    assert np.abs(W - Wo).max() <= 1e-8 * np.abs(Wo).max()
    yo = O.coarsest_null(BL, TL, svd)
    V = h.export(L, B.X_V).reshape(nL, -1)
    assert np.abs(V[:, 0] - yo).max() <= 1e-9 * np.abs(yo).max()
    lam = h.export(L, B.X_LAMBDA).reshape(-1, 2)
    _, entries, Vo = O.coarsest_eigs(BL, TL, 6, svd)
    assert V.shape[1] == Vo.shape[1]
    for e in entries[1:]:
        c = e.cols[0]
        assert abs(complex(lam[c, 0], lam[c, 1]) - e.lam) <= 1e-7 * abs(e.lam)
        for cc in e.cols:
            assert np.abs(V[:, cc] - Vo[:, cc]).max() <= 1e-5, cc
    st = h.stats()
    assert st.coarsest_min_pivot > 1e-12
    h.close()


def test_fullsize_vcycle_and_solution(chain):
    ch, _, B0 = chain
    print("case full-size V-cycle and solve (FP64), then the mixed form", flush=True)
    h = _hier(chain, precision=B.FP64)
    plan = O.level_plan(O.Grid(ch.nx, ch.ny, False), LEVELS)
    lvls = []
    for l in range(LEVELS):
        lv = O.Level(plan[l], _csr(h, l, "B"), None)
        if l < LEVELS - 1:
            Pg = _p(h, l, plan[l + 1].n)
            lv.P, lv.Q = Pg, O.averaging_q(Pg)
        lvls.append(lv)
    ho = O.Hierarchy(lvls, O.Options(levels=LEVELS), O.coarsest_pinv(lvls[-1].B.toarray()), None, [], None)
    f0 = np.random.default_rng(3).random(ch.n)
    f0 -= f0.mean()
    want = O.vcycle(ho, f0)
    f = torch.tensor(f0, device="cuda")
    e = torch.empty_like(f)
    h.apply_vcycle(f, e)
    assert np.abs(e.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.solve(x, 1e-10, 200)
    assert info.converged
    x64 = x.cpu().numpy()
    h.close()
    A = ch.to_scipy()
    for xx in (x64,):
        assert xx.min() >= 0 and abs(xx.sum() - 1) < 1e-13
        assert np.abs(A @ xx - xx).sum() / xx.sum() <= 1e-10
    hm = _hier(chain, precision=B.MIXED)
    info = hm.solve(x, 1e-10, 200)
    assert info.converged
    xm = x.cpu().numpy()
    hm.close()
    assert xm.min() >= 0 and abs(xm.sum() - 1) < 1e-13
    assert np.abs(A @ xm - xm).sum() / xm.sum() <= 1e-10
    # both stop at 1e-10 in the residual; ||B^#||_1 ~ 1e5 here bounds the gap
    assert np.abs(xm - x64).sum() <= 1e-6
    print(f"  |x_mixed - x_fp64|_1 = {np.abs(xm - x64).sum():.3e}", flush=True)
