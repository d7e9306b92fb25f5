"""GPU parity: every step of the HIP path against the CPU oracle on the same
inputs, element by element (through the C ABI).

Tolerances (FP64 path): relaxation 1e-13 relative to max |X|; least-squares
weights 1e-9 (small Gram solves, condition ~1e5); Galerkin products 1e-12 of
the row's largest entry; coarsest pseudo-inverse 1e-8 relative (condition of
B_11 ~ 3e4, no pivoting vs SVD); eigenvalues 1e-7 relative (Arnoldi vs QZ);
final state vector ||x - x_oracle||_1 <= 1e-9.  Sparsity patterns and the
injected test vectors are compared exactly.
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


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


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
    return P, pc


def _same_pattern(A, Bm):
    A = A.tocsr(); Bm = Bm.tocsr()
    A.sort_indices(); Bm.sort_indices()
    return np.array_equal(A.indptr, Bm.indptr) and np.array_equal(A.indices, Bm.indices)


def _rowrel(A, Bm):
    """max over rows of |A - B| / max |B row|."""
    D = abs(A - Bm).tocsr()
    Bm = abs(Bm).tocsr()
    worst = 0.0
    rmax = np.maximum(np.asarray(Bm.max(axis=1).todense()).ravel(), 1e-300)
    dmax = np.asarray(D.max(axis=1).todense()).ravel()
    if len(dmax):
        worst = float(np.max(dmax / rmax))
    return worst


CASES = [
    ("tandem32", lambda: C.tandem_queue(32), 8, 3),
    ("tandem40_ragged", lambda: C.tandem_queue(40), 12, 3),
    ("lattice48p", lambda: C.weighted_lattice(48, seed=3), 12, 3),
    ("uniform21", lambda: C.weighted_lattice(21, periodic=False, uniform_weights=True), 6, 3),
    # even non-periodic sides: the last row and column stay coarse
    ("tandem39_even", lambda: C.tandem_queue(39), 12, 3),
    ("tandem63_even", lambda: C.tandem_queue(63), 12, 4),
    ("uniform20_even", lambda: C.weighted_lattice(20, periodic=False, uniform_weights=True), 6, 3),
    ("lattice14x9_mixed", lambda: C.weighted_lattice(14, seed=4, periodic=False, my=9), 8, 3),
]


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_relax_matches_oracle(name, make, r, levels):
    ch = make()
    rp, ci, v = B.device_csr(ch)
    X0 = np.random.default_rng(1).random((ch.n, r))
    X = torch.tensor(X0, device="cuda")
    B.relax(rp, ci, v, X, r, omega=0.7, nu=3)
    want = O.jacobi(O.b_from_a(ch.to_scipy()), X0, 0.7, 3)
    got = X.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # inhomogeneous form with a right-hand side, R = 1
    f0 = np.random.default_rng(2).random(ch.n)
    e = torch.zeros(ch.n, dtype=torch.float64, device="cuda")
    B.relax(rp, ci, v, e, 1, omega=0.7, nu=2, F=torch.tensor(f0, device="cuda"))
    want = O.jacobi(O.b_from_a(ch.to_scipy()), np.zeros(ch.n), 0.7, 2, F=f0)
    assert np.abs(e.cpu().numpy() - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_downleg_steps_match_oracle(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=1))
    plan = O.level_plan(_grid(ch), levels)
    # initial test vectors: same counter-based generator, bit for bit
    U0 = h.export(0, B.X_U0).reshape(ch.n, r)
    assert np.array_equal(U0, O.initial_tvs(ch.n, r, 0))
    Bl = O.b_from_a(ch.to_scipy())
    assert _same_pattern(_csr(h, 0, "B"), Bl)
    assert np.abs(_csr(h, 0, "B") - Bl).max() == 0.0
    Tl = sp.identity(ch.n, format="csr")
    Uin = U0
    for l in range(levels - 1):
        g = plan[l]
        U = h.export(l, B.X_U).reshape(g.n, r)
        want = O.jacobi(Bl, Uin, 0.7, 4)
        assert np.abs(U - want).max() <= 1e-13 * np.abs(want).max(), l
        w = O.tv_weights(Bl, U)
        Po, Jo, _ = O.ls_fit(U, w, g, 4)
        nc = g.coarse().n
        Pg, pc = _p_from_ell(h, l, nc)
        assert _same_pattern(Pg, Po), l
        assert np.abs((Pg - Po).toarray()).max() <= 1e-9 * max(1.0, np.abs(Po.data).max()), l
        # Galerkin products on the GPU's own P
        Q = O.averaging_q(Pg)
        Bc_o = O.galerkin(Q, Bl, Pg)
        Tc_o = O.galerkin(Q, Tl, Pg)
        Bc_g = _csr(h, l + 1, "B")
        Tc_g = _csr(h, l + 1, "T")
        assert _same_pattern(Bc_g, Bc_o) and _same_pattern(Tc_g, Tc_o), l
        assert _rowrel(Bc_g, Bc_o) <= 1e-12 and _rowrel(Tc_g, Tc_o) <= 1e-12, l
        # injection is exact
        Uc = O.inject(U, g)
        if l + 1 < levels - 1:
            Uin = Uc
            Bl, Tl = Bc_g, Tc_g
        else:
            Ug = h.export(l + 1, B.X_U).reshape(-1, r)
            assert np.array_equal(Ug, Uc)


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_coarsest_matches_oracle(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=2))
    L = levels - 1
    BL = _csr(h, L, "B").toarray()
    TL = _csr(h, L, "T").toarray()
    nL = BL.shape[0]
    W = h.export(L, B.X_W).reshape(nL, nL)
    Wo = O.coarsest_pinv(BL)
    assert np.abs(W - Wo).max() <= 1e-8 * np.abs(Wo).max()
    yo = O.coarsest_null(BL, TL)
    V = h.export(L, B.X_V).reshape(nL, -1)
    assert np.abs(V[:, 0] - yo).max() <= 1e-9 * np.abs(yo).max()
    lam = h.export(L, B.X_LAMBDA).reshape(-1, 2)
    kind = h.export(L, B.X_VKIND)
    _, entries, Vo = O.coarsest_eigs(BL, TL, 6)
    assert V.shape[1] == Vo.shape[1]
    for e in entries[1:]:
        c = e.cols[0]
        got = complex(lam[c, 0], lam[c, 1])
        assert abs(got - e.lam) <= 1e-7 * abs(e.lam), (got, e.lam)
        assert kind[c] == (0 if len(e.cols) == 1 else 1)
        for cc in e.cols:
            # eigenvectors: same normalisation rule on both sides
            assert np.abs(V[:, cc] - Vo[:, cc]).max() <= 1e-5, cc


def test_arnoldi_convergence_checks(monkeypatch):
    # A 65 x 65 coarsest level (tandem 128^2, two levels) runs 40 Arnoldi
    # steps unless the wanted Ritz pairs of the first m = 20 (or else 30)
    # already have relative residuals |h_{m+1,m} s_m| / |theta| <= 1e-9.
    # Both ways the eigenpairs meet the oracle's bar (lam 1e-7, vectors 1e-5).
    ch = C.tandem_queue(127)
    out = {}
    for chk in ("0", "1"):
        monkeypatch.setenv("BAMG_ARNOLDI_CHECK", chk)
        h = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=2, stop_after=2))
        BL = _csr(h, 1, "B").toarray()
        TL = _csr(h, 1, "T").toarray()
        nL = BL.shape[0]
        assert nL == 65 * 65
        out[chk] = (h.stats().arnoldi_steps, h.export(1, B.X_LAMBDA).reshape(-1, 2),
                    h.export(1, B.X_V).reshape(nL, -1))
        h.close()
    assert out["0"][0] == 40 and out["1"][0] in (20, 30, 40)
    _, entries, Vo = O.coarsest_eigs(BL, TL, 6)
    for chk in ("0", "1"):
        lam, V = out[chk][1], out[chk][2]
        for e in entries[1:]:
            c = e.cols[0]
            assert abs(complex(lam[c, 0], lam[c, 1]) - e.lam) <= 1e-7 * abs(e.lam), (chk, c)
            for cc in e.cols:
                assert np.abs(V[:, cc] - Vo[:, cc]).max() <= 1e-5, (chk, cc)
    print("arnoldi steps with the check:", out["1"][0], flush=True)


# Coarsest grids with few block rows: the two-sided block factorisation of
# grids without the periodic arrow meets in block row m = (K + 1) / 2 of the
# K + 1 rows, so one and two rows (no top or no bottom part), three rows and
# rectangular blocks are the edge cases.
SMALL_COARSEST = [
    ("tandem2_2x2", lambda: C.tandem_queue(2), 2),
    ("tandem4_3x3", lambda: C.tandem_queue(4), 2),
    ("tandem4_2x2", lambda: C.tandem_queue(4), 3),
    ("tandem8_5x5", lambda: C.tandem_queue(8), 2),
    ("lattice7x13_4x7", lambda: C.weighted_lattice(7, seed=1, periodic=False, my=13), 2),
    ("lattice2x20_2x11", lambda: C.weighted_lattice(2, seed=2, periodic=False, my=20), 2),
    # rows of 65 points: the main part (64 columns) by the block path and the
    # last column as a border (Schur complement)
    ("lattice9x129_5x65", lambda: C.weighted_lattice(9, seed=5, periodic=False, my=129), 2),
    ("lattice2x129_2x65", lambda: C.weighted_lattice(2, seed=6, periodic=False, my=129), 2),
    ("lattice1x65_1x65", lambda: C.weighted_lattice(1, seed=7, periodic=False, my=65), 1),
    ("tandem127_65x65", lambda: C.tandem_queue(127), 2),
]


@pytest.mark.parametrize("name,make,levels", SMALL_COARSEST)
def test_coarsest_inverse_small_grids(name, make, levels):
    ch = make()
    print(f"case {name}", flush=True)
    h = B.Hierarchy.from_chain(ch, 4, B.default_options(levels=levels, stop_after=2))
    L = levels - 1
    BL = _csr(h, L, "B").toarray()
    nL = BL.shape[0]
    W = h.export(L, B.X_W).reshape(nL, nL)
    Wo = O.coarsest_pinv(BL)
    assert np.abs(W - Wo).max() <= 1e-8 * np.abs(Wo).max()


@pytest.mark.parametrize("name,make,r,levels", CASES[:3])
def test_upleg_matches_oracle(name, make, r, levels):
    ch = make()
    # coarsest eigenpairs as the up-leg received them (same seed, same setup)
    h2 = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=2))
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=3))
    L = levels - 1
    nv = h.level_info(L).n_v
    V = h2.export(L, B.X_V).reshape(-1, nv)
    assert np.array_equal(V, h.export(L, B.X_V).reshape(-1, nv))
    lam = h2.export(L, B.X_LAMBDA).reshape(-1, 2)
    kind = h2.export(L, B.X_VKIND)
    # rebuild the oracle's entry list from the GPU's coarsest result
    ents = [O.EigEntry(0.0, (0,))]
    c = 1
    while c < nv:
        if kind[c] == 0:
            ents.append(O.EigEntry(complex(lam[c, 0], 0.0), (c,))); c += 1
        else:
            ents.append(O.EigEntry(complex(lam[c, 0], lam[c, 1]), (c, c + 1))); c += 2
    # the first-pass hierarchy is what the up-leg used; stop_after=3 keeps it
    for l in range(L - 1, -1, -1):
        nc = h.level_info(l + 1).n
        Pg, _ = _p_from_ell(h, l, nc)
        Bl = _csr(h, l, "B")
        Tl = sp.identity(Bl.shape[0], format="csr") if l == 0 else _csr(h, l, "T")
        Vf = Pg @ V
        Vw, ents = O.eig_relax(Bl, Tl, Vf, ents, 0.7, 4)
        V = h.export(l, B.X_V).reshape(-1, nv)
        assert np.abs(V - Vw).max() <= 1e-10 * np.abs(Vw).max(), l
    # the eigenvalue table holds the finest level's quotients at the end
    lam = h.export(0, B.X_LAMBDA).reshape(-1, 2)
    for e in ents[1:]:
        got = complex(lam[e.cols[0], 0], lam[e.cols[0], 1])
        assert abs(got - e.lam) <= 1e-10 * abs(e.lam)
    x0 = h.export(0, B.X_X0)
    assert np.abs(x0 - V[:, 0] / V[:, 0].sum()).max() <= 1e-14


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_vcycle_matches_oracle(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels))
    # oracle hierarchy assembled from the GPU's final operators
    lvls = []
    plan = O.level_plan(_grid(ch), levels)
    for l in range(levels):
        Bl = _csr(h, l, "B")
        lv = O.Level(plan[l], Bl, None)
        if l < levels - 1:
            Pg, _ = _p_from_ell(h, l, plan[l + 1].n)
            lv.P, lv.Q = Pg, O.averaging_q(Pg)
        lvls.append(lv)
    BL = lvls[-1].B.toarray()
    ho = O.Hierarchy(lvls, O.Options(levels=levels), O.coarsest_pinv(BL), None, [], None)
    f0 = np.random.default_rng(3).random(ch.n)
    f0 -= f0.mean()                     # in range(B): 1^T f = 0
    want = O.vcycle(ho, f0)
    f = torch.tensor(f0, device="cuda")
    e = torch.empty_like(f)
    h.apply_vcycle(f, e)
    got = e.cpu().numpy()
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("relax", ["jacobi", "mcgs"])
@pytest.mark.parametrize("name,make,r,levels", [CASES[1], CASES[2], CASES[5]])
def test_fused_cycle_passes_give_the_same_bits(name, make, r, levels, relax, precision, monkeypatch):
    # On small coarse grid levels the cycle forms the prolongation inside the
    # first post-smoothing sweep; BAMG_CYCLE_FUSE=0 takes the separate
    # launches.  Both are the same sums in the same order, so the cycle's
    # output must agree bit for bit.
    ch = make()
    opts = B.default_options(levels=levels, cycle_mode=1,
                             precision=B.MIXED if precision == "mixed" else B.FP64,
                             relax=B.RELAX_MCGS if relax == "mcgs" else B.RELAX_JACOBI)
    h = B.Hierarchy.from_chain(ch, r, opts)
    f0 = np.random.default_rng(5).random(ch.n)
    f0 -= f0.mean()
    f = torch.tensor(f0, device="cuda")
    out = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("BAMG_CYCLE_FUSE", fuse)
        e = torch.empty_like(f)
        h.apply_vcycle(f, e)
        out[fuse] = e.cpu().numpy()
    h.close()
    assert np.abs(out["1"]).max() > 0
    assert np.array_equal(out["0"], out["1"]), np.abs(out["0"] - out["1"]).max()


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_stationary_matches_oracle(name, make, r, levels):
    ch = make()
    x, info, h = B.stationary(ch, r, tol=1e-13, max_cycles=200, levels=levels)
    assert info.converged, info.residual_l1
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-14
    xo, oinfo, _ = O.stationary(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels), tol=1e-13)
    assert np.abs(x - xo).sum() <= 1e-9
    if ch.exact is not None:
        assert np.abs(x - ch.exact).sum() <= 1e-9
    A = ch.to_scipy()
    assert np.abs(A @ x - x).sum() / x.sum() <= 1e-12


def test_paper_tolerance_and_restart_path():
    # the solve stops at the requested 1-norm tolerance and reports the history
    ch = C.tandem_queue(64)
    x, info, h = B.stationary(ch, 8, tol=1e-10, max_cycles=100, levels=4)
    assert info.converged and info.residual_l1 <= 1e-10
    assert info.history_len >= 1 and info.history[info.history_len - 1] <= 1e-10
    st = h.stats()
    assert st.n_levels == 4 and 1.0 < st.op_complexity < 2.5


def test_errors_are_reported():
    ch = C.tandem_queue(8)
    rp, ci, v = B.device_csr(ch)
    g = (ch.nx, ch.ny, 0)
    bad = v.clone(); bad[0] = -0.1
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy(ch.n, rp, ci, bad, g, 4)
    assert e.value.code == B.ENOTSTOCH
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy(ch.n, rp, ci, v, (ch.nx + 1, ch.ny, 0), 4)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy(ch.n, rp, ci, v, g, 0)
    assert e.value.code == B.EINVAL
    # a stencil wider than the 3x3 box: reorder the grid as 1 x n
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy(ch.n, rp, ci, v, (3, ch.n // 3, 0), 4)
    assert e.value.code in (B.EUNSUPPORTED, B.EINVAL)
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy(ch.n, rp, ci, v, g, 4, B.default_options(mem_budget=1024))
    assert e.value.code == B.ENOMEM
    h = B.Hierarchy(ch.n, rp, ci, v, g, 4, B.default_options(levels=2))
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.solve(x, 1e-30, 2)
    assert not info.converged and info.cycles == 2
