"""The setup W-cycle (options.mu = 2) and the stand-alone MLE iteration
(bamg_mle_iterate) on the GPU against the oracle's Algorithm 3 recursion:
hierarchy and stationary vector of the W-cycle setup, the MLE iterates and
their cycle counts, the hierarchy left behind usable by the solver, and the
refusals.  Tolerances as in the other parity tests (x within 1e-9)."""
import numpy as np
import pytest

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402
from tests.test_gpu_parity import _grid, _p_from_ell, _same_pattern  # noqa: E402

CASES = [
    ("tandem32", lambda: C.tandem_queue(32), 8, 3),
    ("lattice48p", lambda: C.weighted_lattice(48, seed=3), 12, 3),
    ("uniform21", lambda: C.weighted_lattice(21, periodic=False, uniform_weights=True), 6, 3),
]


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_w_cycle_setup_matches_oracle(name, make, r, levels):
    ch = make()
    ho = O.setup(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels, mu=2))
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, mu=2))
    for l in range(levels - 1):
        Pg, _ = _p_from_ell(h, l, h.level_info(l + 1).n)
        Po = ho.levels[l].P
        assert _same_pattern(Pg, Po), l
        assert np.abs((Pg - Po).toarray()).max() <= 1e-8 * max(1.0, np.abs(Po.data).max()), l
    assert np.abs(h.export(0, B.X_X0) - ho.x0).max() <= 1e-8 * np.abs(ho.x0).max()
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.solve(x, tol=1e-13, max_cycles=200)
    assert info.converged
    xo, _ = O.solve(ho, tol=1e-13, max_cycles=200)
    assert np.abs(x.cpu().numpy() - xo).sum() <= 1e-9


@pytest.mark.parametrize("mu", [1, 2])
@pytest.mark.parametrize("name,make,r,levels", CASES[:2])
def test_mle_iteration_matches_oracle(name, make, r, levels, mu):
    ch = make()
    tol = 1e-9
    xo, oinfo, _ = O.mle_iteration(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels, mu=mu), tol=tol,
                                   max_cycles=60)
    assert oinfo.converged
    h = B.Hierarchy.from_chain(ch, r, B.default_options(levels=levels, mu=mu))
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.mle_iterate(x, tol=tol, max_cycles=60)
    assert info.converged, info.residual_l1
    # the setup ran the oracle's first cycle; the handle then ran the others
    assert abs((info.cycles + 1) - oinfo.cycles) <= 1, (info.cycles, oinfo.cycles)
    xg = x.cpu().numpy()
    assert xg.min() >= 0 and abs(xg.sum() - 1) < 1e-14
    assert np.abs(xg - np.maximum(xo, 0) / np.maximum(xo, 0).sum()).sum() <= 1e-7
    # the hierarchy left behind still solves
    info2 = h.solve(x, tol=1e-12, max_cycles=200)
    assert info2.converged


def test_mle_refusals():
    chains = [C.tandem_queue(16), C.weighted_lattice(16, seed=1)]
    hb = B.BatchedHierarchy(chains, 6, B.default_options(levels=2))
    x = torch.empty(hb.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.BamgError) as e:
        hb.mle_iterate(x)
    assert e.value.code == B.EUNSUPPORTED
    with pytest.raises(B.BamgError) as e:
        B.Hierarchy.from_chain(chains[0], 6, B.default_options(levels=2, mu=3))
    assert e.value.code == B.EINVAL
