"""Mixed-precision form: FP32 relaxation, LS-fit storage, Galerkin products and
V-cycle; FP64 weights, coarsest solve, outer FGMRES and normalisation.

The FP64 outer iteration still converges to the unique stationary vector, so
x is compared with the oracle to the FP64 bar (||x - x_oracle||_1 <= 1e-9).
FP32 steps are compared with the oracle applied to the same (FP32) inputs:
relaxation within 1e-5 of max |X| (a few FP32 roundings per sweep), Galerkin
rows within 1e-5 of the row maximum (FP32 accumulation of <= ~100 products
with cancellation in the diagonal).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402
from tests.test_gpu_parity import CASES, _csr, _grid, _p_from_ell, _rowrel, _same_pattern  # noqa: E402


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_mixed_stationary_matches_oracle(name, make, r, levels):
    ch = make()
    x, info, h = B.stationary(ch, r, tol=1e-13, max_cycles=300, levels=levels, precision=B.MIXED)
    assert info.converged, info.residual_l1
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-14
    xo, _, _ = O.stationary(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels), tol=1e-13)
    assert np.abs(x - xo).sum() <= 1e-9


@pytest.mark.parametrize("name,make,r,levels", CASES[:3])
def test_mixed_downleg_steps(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=1, precision=B.MIXED))
    plan = O.level_plan(_grid(ch), levels)
    U0 = O.initial_tvs(ch.n, r, 0).astype(np.float32).astype(np.float64)
    assert np.array_equal(h.export(0, B.X_U0).reshape(ch.n, r), U0)
    Bl = O.b_from_a(ch.to_scipy())
    Bl32 = Bl.copy(); Bl32.data = Bl32.data.astype(np.float32).astype(np.float64)
    Tl = sp.identity(ch.n, format="csr")
    U = h.export(0, B.X_U).reshape(ch.n, r)
    want = O.jacobi(Bl, U0, 0.7, 4)
    assert np.abs(U - want).max() <= 1e-5 * np.abs(want).max()
    for l in range(levels - 1):
        g = plan[l]
        U = h.export(l, B.X_U).reshape(g.n, r)
        w = O.tv_weights(Bl32 if l == 0 else Bl, U)
        Po, _, _ = O.ls_fit(U, w, g, 4)
        Pg, _ = _p_from_ell(h, l, g.coarse().n)
        assert _same_pattern(Pg, Po), l
        # FP32 storage of FP64-computed weights
        assert np.abs((Pg - Po).toarray()).max() <= 1e-6 * max(1.0, np.abs(Po.data).max()), l
        Q = O.averaging_q(Pg)
        Bc_o = O.galerkin(Q, Bl32 if l == 0 else Bl, Pg)
        Tc_o = O.galerkin(Q, Tl, Pg)
        Bc_g = _csr(h, l + 1, "B")
        Tc_g = _csr(h, l + 1, "T")
        assert _same_pattern(Bc_g, Bc_o) and _same_pattern(Tc_g, Tc_o), l
        assert _rowrel(Bc_g, Bc_o) <= 1e-5 and _rowrel(Tc_g, Tc_o) <= 1e-5, l
        Bl, Tl = Bc_g, Tc_g


def test_mixed_hierarchy_close_to_fp64():
    ch = C.tandem_queue(64)
    h64 = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=4))
    h32 = B.Hierarchy.from_chain(ch, 8, B.default_options(levels=4, precision=B.MIXED))
    for l in range(1, 4):
        a, b = _csr(h32, l, "B"), _csr(h64, l, "B")
        rel = sp.linalg.norm(a - b) / sp.linalg.norm(b)
        assert rel <= 1e-3, (l, rel)


@pytest.mark.parametrize("name,make,r,levels", CASES[:5])
def test_mixed_coarsest_eigenpairs(name, make, r, levels):
    # The mixed form's Arnoldi multiplies by W rounded to FP32 (vectors, sums
    # and the Hessenberg problem stay FP64).  Entrywise rounding 2^-24 moves
    # an eigenvalue theta of W by at most kappa * 2^-24 ||W||_F, and the
    # wanted theta are the largest, of the order of ||W||_2 >= ||W||_F /
    # sqrt(n): for these coarsest grids (n <= 121) that is below 1e-6 kappa
    # relative, so lam = 1/theta within 1e-5 and eigenvectors within 1e-3
    # allow kappa ~ 10.  An error in the product's indexing moves them by O(1).
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=2, precision=B.MIXED))
    L = levels - 1
    BL = _csr(h, L, "B").toarray()
    TL = _csr(h, L, "T").toarray()
    nL = BL.shape[0]
    V = h.export(L, B.X_V).reshape(nL, -1)
    lam = h.export(L, B.X_LAMBDA).reshape(-1, 2)
    _, entries, Vo = O.coarsest_eigs(BL, TL, 6)
    assert V.shape[1] == Vo.shape[1]
    for e in entries[1:]:
        c = e.cols[0]
        got = complex(lam[c, 0], lam[c, 1])
        assert abs(got - e.lam) <= 1e-5 * abs(e.lam), (nL, got, e.lam)
        for cc in e.cols:
            assert np.abs(V[:, cc] - Vo[:, cc]).max() <= 1e-3, (nL, cc)
    h.close()
