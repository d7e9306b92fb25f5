"""Multicolour Gauss-Seidel relaxation on the GPU against the oracle (same
colouring, same colour order): the test-vector sweeps and P patterns of the
down-leg, the eigenvector sweeps of the up-leg, one V-cycle on the GPU's own
operators, the stationary vector (FP64 within 1e-9, mixed to the tolerance),
several chains in one handle, and the rejection of an operator that couples
two points of one colour.  Tolerances as in the Jacobi parity tests."""
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
from tests.test_gpu_parity import _csr, _grid, _p_from_ell, _rowrel, _same_pattern  # noqa: E402

GS = dict(relax=B.RELAX_MCGS)
OGS = dict(relax="mcgs")

CASES = [
    ("tandem32", lambda: C.tandem_queue(32), 8, 3),
    ("lattice48p", lambda: C.weighted_lattice(48, seed=3), 12, 3),
    ("uniform21", lambda: C.weighted_lattice(21, periodic=False, uniform_weights=True), 6, 3),
]


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_mcgs_downleg_matches_oracle(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=1, **GS))
    plan = O.level_plan(_grid(ch), levels)
    Bl = O.b_from_a(ch.to_scipy())
    Uin = h.export(0, B.X_U0).reshape(ch.n, r)
    for l in range(levels - 1):
        g = plan[l]
        col, ncol = O.colours(g)
        U = h.export(l, B.X_U).reshape(g.n, r)
        want = O.mcgs(Bl, Uin, col, ncol, 1.0, 4)
        assert np.abs(U - want).max() <= 1e-13 * np.abs(want).max(), l
        Po, _, _ = O.ls_fit(U, O.tv_weights(Bl, U), g, 4)
        Pg, _ = _p_from_ell(h, l, g.coarse().n)
        assert _same_pattern(Pg, Po), l
        assert np.abs((Pg - Po).toarray()).max() <= 1e-9 * max(1.0, np.abs(Po.data).max()), l
        Uin = O.inject(U, g)
        Bl = _csr(h, l + 1, "B")


@pytest.mark.parametrize("name,make,r,levels", CASES[:2])
def test_mcgs_upleg_matches_oracle(name, make, r, levels):
    ch = make()
    h2 = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=2, **GS))
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, stop_after=3, **GS))
    L = levels - 1
    nv = h.level_info(L).n_v
    V = h2.export(L, B.X_V).reshape(-1, nv)
    lam = h2.export(L, B.X_LAMBDA).reshape(-1, 2)
    kind = h2.export(L, B.X_VKIND)
    ents = [O.EigEntry(0.0, (0,))]
    c = 1
    while c < nv:
        if kind[c] == 0:
            ents.append(O.EigEntry(complex(lam[c, 0], 0.0), (c,))); c += 1
        else:
            ents.append(O.EigEntry(complex(lam[c, 0], lam[c, 1]), (c, c + 1))); c += 2
    plan = O.level_plan(_grid(ch), levels)
    for l in range(L - 1, -1, -1):
        Pg, _ = _p_from_ell(h, l, h.level_info(l + 1).n)
        Bl = _csr(h, l, "B")
        Tl = sp.identity(Bl.shape[0], format="csr") if l == 0 else _csr(h, l, "T")
        col, ncol = O.colours(plan[l])
        Vw, ents = O.eig_relax(Bl, Tl, Pg @ V, ents, 0.7, 4, gs=(col, ncol, 1.0))
        V = h.export(l, B.X_V).reshape(-1, nv)
        assert np.abs(V - Vw).max() <= 1e-10 * np.abs(Vw).max(), l


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_mcgs_vcycle_matches_oracle(name, make, r, levels):
    ch = make()
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, **GS))
    plan = O.level_plan(_grid(ch), levels)
    lvls = []
    for l in range(levels):
        lv = O.Level(plan[l], _csr(h, l, "B"), None)
        if l < levels - 1:
            Pg, _ = _p_from_ell(h, l, plan[l + 1].n)
            lv.P, lv.Q = Pg, O.averaging_q(Pg)
        lvls.append(lv)
    ho = O.Hierarchy(lvls, O.Options(levels=levels, **OGS), O.coarsest_pinv(lvls[-1].B.toarray()), None, [], None)
    f0 = np.random.default_rng(3).random(ch.n)
    f0 -= f0.mean()
    want = O.vcycle(ho, f0)
    f = torch.tensor(f0, device="cuda")
    e = torch.empty_like(f)
    h.apply_vcycle(f, e)
    assert np.abs(e.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_mcgs_stationary_matches_oracle(name, make, r, levels):
    ch = make()
    x, info, h = B.stationary(ch, r, tol=1e-13, max_cycles=200, levels=levels, **GS)
    assert info.converged, info.residual_l1
    xo, oinfo, _ = O.stationary(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels, **OGS), tol=1e-13)
    assert np.abs(x - xo).sum() <= 1e-9
    # the mixed form reaches the tolerance too
    xm, im, _ = B.stationary(ch, r, tol=1e-10, max_cycles=200, levels=levels, precision=B.MIXED, **GS)
    assert im.converged and np.abs(xm - xo).sum() <= 1e-7


def test_mcgs_batched_equals_single_and_graph_replays():
    chains = [C.tandem_queue(24, jitter=0.2, seed=1, chain_id=1), C.weighted_lattice(32, seed=4),
              C.tandem_queue(40, jitter=0.2, seed=2, chain_id=2)]
    res = []
    for mode in (1, 2):
        h = B.BatchedHierarchy(chains, 8, B.default_options(levels=3, cycle_mode=mode, **GS))
        x = torch.empty(h.n, dtype=torch.float64, device="cuda")
        info, status, resid = h.solve_batched(x, tol=1e-12, max_cycles=300)
        assert status.all(), resid
        res.append(x.cpu().numpy())
    assert np.array_equal(res[0], res[1])
    off = np.cumsum([0] + [c.n for c in chains])
    for c, ch in enumerate(chains):
        x1, i1, _ = B.stationary(ch, 8, tol=1e-12, max_cycles=300, levels=3, **GS)
        assert i1.converged
        assert np.array_equal(res[0][off[c]:off[c + 1]], x1)


def test_mcgs_options_and_reach():
    # an operator reaching beyond the 3 x 3 box (here: coupling two points of
    # one colour) is refused by bamg_setup whatever the relaxation, so every
    # hierarchy it builds can be swept by colours
    ch = C.tandem_queue(8)
    A = ch.to_scipy().tolil()
    col, _ = O.colours(_grid(ch))
    j = 0
    i = next(k for k in range(2, ch.n) if col[k] == col[j] and k > ch.ny + 1)
    eps = 0.5 * A[j, j]
    A[i, j] += eps          # move probability from the self-loop of j to i
    A[j, j] -= eps
    A = A.tocsr()
    A.sort_indices()
    bad = C.Chain(ch.n, A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
                  ch.nx, ch.ny, ch.periodic, "tandem8+long")
    for kw in (GS, {}):
        with pytest.raises(B.BamgError) as e:
            B.Hierarchy.from_chain(bad, 4, B.default_options(levels=2, **kw))
        assert e.value.code == B.EUNSUPPORTED
    for kw in (dict(relax=2), dict(gs_omega=2.0, **GS), dict(gs_omega=0.0, **GS)):
        with pytest.raises(B.BamgError) as e:
            B.Hierarchy.from_chain(ch, 4, B.default_options(levels=2, **kw))
        assert e.value.code == B.EINVAL
