"""The multigrid-preconditioned Arnoldi method (Section 4.3) on the GPU
(bamg_solve with BAMG_PARNOLDI) against the oracle's: the stationary vector
within 1e-9 (FP64), the number of preconditioner applications within two of
the oracle's (the two orthogonalise in different orders), restarts, the mixed
form, several chains in one handle, and flag validation."""
import numpy as np
import pytest

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


CASES = [
    ("tandem32", lambda: C.tandem_queue(32), 8, 3),
    ("tandem40_ragged", lambda: C.tandem_queue(40), 12, 3),
    ("lattice48p", lambda: C.weighted_lattice(48, seed=3), 12, 3),
    ("uniform21", lambda: C.weighted_lattice(21, periodic=False, uniform_weights=True), 6, 3),
]


@pytest.mark.parametrize("name,make,r,levels", CASES)
def test_parnoldi_matches_oracle(name, make, r, levels):
    ch = make()
    x, info, h = B.stationary(ch, r, tol=1e-13, max_cycles=200, levels=levels, parnoldi=True)
    assert info.converged, info.residual_l1
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-14
    xo, oinfo, _ = O.stationary(ch.to_scipy(), _grid(ch), r, O.Options(levels=levels), tol=1e-13,
                                max_cycles=200, method="parnoldi")
    assert oinfo.converged
    assert np.abs(x - xo).sum() <= 1e-9
    assert abs(info.cycles - oinfo.cycles) <= 2, (info.cycles, oinfo.cycles)
    # the residual history is one entry per step plus the start
    assert info.history_len == info.cycles + 1


def test_parnoldi_restarts_and_mixed():
    ch = C.weighted_lattice(48, seed=3)
    x, info, _ = B.stationary(ch, 12, tol=1e-13, max_cycles=300, levels=3, gmres_m=3, parnoldi=True)
    assert info.converged and info.restarts >= 2
    assert np.abs(x - ch.exact).sum() <= 1e-9
    xm, im, _ = B.stationary(ch, 12, tol=1e-10, max_cycles=300, levels=3, precision=B.MIXED, parnoldi=True)
    assert im.converged and np.abs(xm - ch.exact).sum() <= 1e-7


def test_parnoldi_batched_equals_single():
    chains = [C.tandem_queue(24, jitter=0.2, seed=1, chain_id=1), C.weighted_lattice(32, seed=4),
              C.tandem_queue(40, jitter=0.2, seed=2, chain_id=2)]
    h = B.BatchedHierarchy(chains, 8, B.default_options(levels=3))
    x = torch.empty(h.n, dtype=torch.float64, device="cuda")
    info, status, resid = h.solve_batched(x, tol=1e-12, max_cycles=300, parnoldi=True)
    assert status.all(), resid
    xb = x.cpu().numpy()
    off = np.cumsum([0] + [c.n for c in chains])
    for c, ch in enumerate(chains):
        x1, i1, _ = B.stationary(ch, 8, tol=1e-12, max_cycles=300, levels=3, parnoldi=True)
        assert i1.converged
        assert np.array_equal(xb[off[c]:off[c + 1]], x1)


def test_unknown_solve_flags():
    ch = C.tandem_queue(8)
    h = B.Hierarchy.from_chain(ch, 4, B.default_options(levels=2))
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    rc = B.load().bamg_solve(h._h, B.C.c_void_p(x.data_ptr()), 1e-10, 10, 4, None)
    assert rc == B.EINVAL
