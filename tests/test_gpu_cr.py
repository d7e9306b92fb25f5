"""GPU parity of the coarsening without a grid (Section 3.1, Algorithm 1) and
of the hierarchy built on it, on unstructured planar graphs (Section 5,
Table 4), through the C ABI.

Integer results are compared exactly: the coarse points of every level (the
independent sets and the compatible-relaxation decisions, which both sides
take in FP64 with the same roundings), the sparsity of P and of the Galerkin
products, the injected test vectors.  Tolerances (FP64): CR estimates 1e-12
relative (different reduction order), least-squares weights 1e-9, Galerkin
products 1e-12 of the row's largest entry, the V-cycle 1e-9, the stationary
vector 1e-10 in the 1-norm against the closed form (x proportional to the
degree) and against the oracle.
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


def _csr(h, l, which):
    li = h.level_info(l)
    if which == "B":
        rp, ci, v = h.export(l, B.X_B_ROWPTR), h.export(l, B.X_B_COL), h.export(l, B.X_B_VAL)
    else:
        rp, ci, v = h.export(l, B.X_T_ROWPTR), h.export(l, B.X_T_COL), h.export(l, B.X_T_VAL)
    return sp.csr_matrix((v, ci, rp), shape=(li.n, li.n))


def _p_from_ell(h, l, nc):
    pc = h.export(l, B.X_P_COL).reshape(-1, 4)
    pv = h.export(l, B.X_P_VAL).reshape(-1, 4)
    n = pc.shape[0]
    rows, cols, vals = [], [], []
    for s in range(4):
        ok = pc[:, s] >= 0
        rows.append(np.nonzero(ok)[0]); cols.append(pc[ok, s]); vals.append(pv[ok, s])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
    P.sort_indices()
    return P


def _same_pattern(A, Bm):
    A = A.tocsr(); Bm = Bm.tocsr()
    A.sort_indices(); Bm.sort_indices()
    return np.array_equal(A.indptr, Bm.indptr) and np.array_equal(A.indices, Bm.indices)


def _rowrel(A, Bm):
    D = abs(A - Bm).tocsr()
    Bm = abs(Bm).tocsr()
    rmax = np.maximum(np.asarray(Bm.max(axis=1).todense()).ravel(), 1e-300)
    dmax = np.asarray(D.max(axis=1).todense()).ravel()
    return float(np.max(dmax / rmax)) if len(dmax) else 0.0


CASES = [
    ("upg256", 256, 0),
    ("upg700_ragged", 700, 3),
    ("upg2048", 2048, 0),
]
OPTS = O.Options(levels=3)


@pytest.mark.parametrize("name,N,seed", CASES)
def test_cr_downleg_matches_oracle(name, N, seed):
    ch = C.upg(N, seed=seed)
    r = 6
    print(f"case {name}", flush=True)
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=3, stop_after=1))
    U0 = h.export(0, B.X_U0).reshape(ch.n, r)
    assert np.array_equal(U0, O.initial_tvs(ch.n, r, 0))
    Bl = O.b_from_a(ch.to_scipy())
    assert _same_pattern(_csr(h, 0, "B"), Bl)
    Tl = sp.identity(ch.n, format="csr")
    Uin = U0
    for l in range(2):
        n = Bl.shape[0]
        # compatible relaxation: the same C points, the same estimates
        isC, rounds, rhos = O.cr_coarsen(Bl, l, OPTS.omega, OPTS.cr_theta, OPTS.cr_nu, 0, OPTS.cr_rounds)
        cmap = h.export(l, B.X_CMAP)
        want = np.where(isC, np.cumsum(isC) - 1, -1)
        assert np.array_equal(cmap, want), l
        li = h.level_info(l)
        assert li.cr_rounds == rounds, l
        rho = h.export(l, B.X_CR_RHO)
        assert np.allclose(rho, rhos, rtol=1e-12, atol=0), (l, rho, rhos)
        cs = O.Coarsening(isC, np.nonzero(isC)[0], O.graph_slots(Bl, isC, 1))
        nc = cs.nc
        assert h.level_info(l + 1).n == nc
        # relaxed test vectors
        U = h.export(l, B.X_U).reshape(n, r)
        wantU = O.jacobi(Bl, Uin, OPTS.omega, OPTS.nu_setup)
        assert np.abs(U - wantU).max() <= 1e-13 * np.abs(wantU).max(), l
        # least-squares interpolation on the candidate lists
        w = O.tv_weights(Bl, U)
        Po, _, _ = O.ls_fit(U, w, cs, 4)
        Pg = _p_from_ell(h, l, nc)
        assert _same_pattern(Pg, Po), l
        assert np.abs((Pg - Po).toarray()).max() <= 1e-9 * max(1.0, np.abs(Po.data).max()), l
        # Petrov-Galerkin products on the GPU's own P
        Q = O.averaging_q(Pg)
        Bc_o = O.galerkin(Q, Bl, Pg)
        Tc_o = O.galerkin(Q, Tl, Pg)
        Bc_g = _csr(h, l + 1, "B")
        Tc_g = _csr(h, l + 1, "T")
        assert _same_pattern(Bc_g, Bc_o) and _same_pattern(Tc_g, Tc_o), l
        assert _rowrel(Bc_g, Bc_o) <= 1e-12 and _rowrel(Tc_g, Tc_o) <= 1e-12, l
        # injection is exact
        Uc = O.inject(U, cs)
        if l == 0:
            Uin = Uc
            Bl, Tl = Bc_g, Tc_g
        else:
            assert np.array_equal(h.export(l + 1, B.X_U).reshape(-1, r), Uc)


@pytest.mark.parametrize("name,N,seed", CASES)
def test_cr_vcycle_matches_oracle(name, N, seed):
    ch = C.upg(N, seed=seed)
    print(f"case {name}", flush=True)
    h = B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3))
    lvls = []
    for l in range(3):
        lv = O.Level(None, _csr(h, l, "B"), None)
        if l < 2:
            Pg = _p_from_ell(h, l, h.level_info(l + 1).n)
            lv.P, lv.Q = Pg, O.averaging_q(Pg)
        lvls.append(lv)
    BL = lvls[-1].B.toarray()
    ho = O.Hierarchy(lvls, O.Options(levels=3), O.coarsest_pinv(BL), None, [], None)
    f0 = np.random.default_rng(3).random(ch.n)
    f0 -= f0.mean()
    want = O.vcycle(ho, f0)
    f = torch.tensor(f0, device="cuda")
    e = torch.empty_like(f)
    h.apply_vcycle(f, e)
    assert np.abs(e.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("name,N,seed", CASES)
def test_cr_stationary_matches_closed_form_and_oracle(name, N, seed):
    ch = C.upg(N, seed=seed)
    print(f"case {name}", flush=True)
    x, info, h = B.stationary(ch, 6, tol=1e-13, max_cycles=200, levels=3)
    assert info.converged, info.residual_l1
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-14
    assert np.abs(x - ch.exact).sum() <= 1e-10
    xo, oinfo, ho = O.stationary(ch.to_scipy(), None, 6, O.Options(levels=3), tol=1e-13)
    assert np.abs(x - xo).sum() <= 1e-10
    assert [h.level_info(l).n for l in range(3)] == [lv.B.shape[0] for lv in ho.levels]


def test_cr_dense_coarsest_inverse_at_1234_points():
    # the coarsest level without a grid takes the dense Gauss-Jordan inverse:
    # 20 blocks of 64 (the last one partial) against the SVD pseudo-inverse
    ch = C.upg(16384, seed=0)
    h = B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3, stop_after=2))
    BL = _csr(h, 2, "B").toarray()
    nL = BL.shape[0]
    assert nL > 1200
    W = h.export(2, B.X_W).reshape(nL, nL)
    Wo = O.coarsest_pinv(BL)
    assert np.abs(W - Wo).max() <= 1e-8 * np.abs(Wo).max()


def test_cr_mixed_precision_converges():
    ch = C.upg(2048, seed=0)
    x, info, h = B.stationary(ch, 6, tol=1e-10, max_cycles=200, levels=3, precision=B.MIXED)
    assert info.converged, info.residual_l1
    assert np.abs(x - ch.exact).sum() <= 1e-8
    # level 0 is coarsened from the FP64 B_0 in both precisions
    h64 = B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3, stop_after=1))
    assert np.array_equal(h.export(0, B.X_CMAP), h64.export(0, B.X_CMAP))


def test_cr_mle_iteration_near_table_4():
    # Table 4: 15 MLE cycles at N = 256 (another random graph)
    ch = C.upg(256, seed=0)
    h = B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3))
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.mle_iterate(x, tol=1e-8, max_cycles=40)
    assert info.converged and 8 <= info.cycles <= 25, info.cycles
    assert np.abs(x.cpu().numpy() - ch.exact).sum() <= 1e-6


def test_cr_automatic_depth_and_default_levels():
    # levels = 0: coarsen while n_l > coarse_max
    ch = C.upg(2048, seed=5)
    x, info, h = B.stationary(ch, 6, tol=1e-10, max_cycles=200, levels=0, coarse_max=200)
    assert info.converged
    st = h.stats()
    assert st.n_levels >= 3 and h.level_info(st.n_levels - 1).n <= 200
    assert np.abs(x - ch.exact).sum() <= 1e-8


def _directed_cycle(n):
    # A[i+1, i] = 1: column stochastic, pattern not symmetric
    rp = np.arange(n + 1, dtype=np.int32)
    ci = ((np.arange(n) - 1) % n).astype(np.int32)
    return C.Chain(n, rp, ci, np.ones(n), 0, 0, False, name="dcycle")


def test_cr_errors():
    ch = C.upg(256, seed=0)
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3, nbr_dist=2))
    assert e.value.code == B.EUNSUPPORTED
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3, relax=B.RELAX_MCGS))
    assert e.value.code == B.EUNSUPPORTED
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(ch, 6, B.default_options(levels=3, cr_theta=1.5))
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(_directed_cycle(64), 6, B.default_options(levels=2))
    assert e.value.code == B.EUNSUPPORTED
    with pytest.raises(B.BamgError) as e:
        B.BatchedHierarchy([ch, C.upg(300, seed=1)], 6, B.default_options(levels=3))
    assert e.value.code == B.EUNSUPPORTED
