"""Pins of the oracle's multicolour Gauss-Seidel relaxation (the Gauss-Seidel
option next to omega-Jacobi in Section 3): brute-force scalar Gauss-Seidel in
colour order on tiny chains, validity of the colouring on every level, the
two-level error propagator written out densely, and the closed-form
stationary vectors reached with the option."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


def _scalar_gs(Bd, x, f, order, w, nu):
    """Textbook Gauss-Seidel with pure-Python loops: points in the given
    order, each from the latest values of all others."""
    x = [float(v) for v in x]
    n = len(x)
    for _ in range(nu):
        for i in order:
            s = 0.0
            for j in range(n):
                s += Bd[i][j] * x[j]
            x[i] = x[i] + w * (f[i] - s) / Bd[i][i]
    return np.array(x)


@pytest.mark.parametrize("make", [lambda: C.tandem_queue(5), lambda: C.weighted_lattice(6, seed=2),
                                  lambda: C.weighted_lattice(5, periodic=False, uniform_weights=True)])
@pytest.mark.parametrize("w", [1.0, 1.3])
def test_mcgs_is_gauss_seidel_in_colour_order(make, w):
    ch = make()
    g = _grid(ch)
    B = O.b_from_a(ch.to_scipy())
    col, ncol = O.colours(g)
    order = sorted(range(ch.n), key=lambda i: (col[i], i))
    rng = np.random.default_rng(0)
    x0 = rng.random(ch.n)
    f = rng.random(ch.n)
    want = _scalar_gs(B.toarray().tolist(), x0, f.tolist(), order, w, 2)
    got = O.mcgs(B, x0, col, ncol, w, 2, F=f)
    assert np.abs(got - want).max() < 1e-13
    # several columns at once, homogeneous
    X = rng.random((ch.n, 3))
    got = O.mcgs(B, X, col, ncol, w, 1)
    for k in range(3):
        want = _scalar_gs(B.toarray().tolist(), X[:, k], [0.0] * ch.n, order, w, 1)
        assert np.abs(got[:, k] - want).max() < 1e-13


@pytest.mark.parametrize("nx,ny,periodic", [(8, 8, False), (7, 9, False), (6, 6, True), (5, 7, True), (3, 4, True)])
def test_colouring_separates_the_3x3_box(nx, ny, periodic):
    g = O.Grid(nx, ny, periodic)
    col, ncol = O.colours(g)
    assert ncol == (3 if periodic and nx % 2 else 2) * (3 if periodic and ny % 2 else 2)
    assert set(np.unique(col)) <= set(range(ncol))
    # every point against its Chebyshev-1 neighbours (brute force)
    for a in range(nx):
        for b in range(ny):
            for da in (-1, 0, 1):
                for db in (-1, 0, 1):
                    if da == 0 and db == 0:
                        continue
                    na, nb = a + da, b + db
                    if periodic:
                        na %= nx; nb %= ny
                    elif not (0 <= na < nx and 0 <= nb < ny):
                        continue
                    if (na, nb) == (a, b):
                        continue
                    assert col[a * ny + b] != col[na * ny + nb]


def test_colouring_check_rejects_a_long_coupling():
    ch = C.tandem_queue(6)
    B = O.b_from_a(ch.to_scipy()).tolil()
    col, _ = O.colours(_grid(ch))
    O.check_colouring(B.tocsr(), col)
    i = 0
    j = next(k for k in range(2, ch.n) if col[k] == col[i] and abs(k - i) > 1)
    B[i, j] = -1e-3
    with pytest.raises(ValueError):
        O.check_colouring(B.tocsr(), col)


def test_null_vector_is_a_fixed_point():
    ch = C.weighted_lattice(8, seed=1)
    B = O.b_from_a(ch.to_scipy())
    col, ncol = O.colours(_grid(ch))
    x = ch.exact.copy()
    y = O.mcgs(B, x, col, ncol, 1.0, 3)
    assert np.abs(y - x).max() < 1e-15 * np.abs(x).max() * 10


def test_vcycle_with_mcgs_equals_dense_error_propagator():
    # two levels: E = S_post (I - P B_c^+ Q B) S_pre with the Gauss-Seidel
    # iteration matrices written out per colour, G_c = I - w D_c^-1 B on the
    # rows of colour c (identity elsewhere), S = G_{ncol-1} ... G_0
    ch = C.tandem_queue(10)
    opts = O.Options(levels=2, relax="mcgs")
    h = O.setup(ch.to_scipy(), _grid(ch), 6, opts)
    B = h.levels[0].B.toarray()
    P = h.levels[0].P.toarray(); Q = h.levels[0].Q.toarray()
    Bc = h.levels[1].B.toarray()
    n = B.shape[0]
    col, ncol = O.colours(_grid(ch))
    S = np.eye(n)
    for c in range(ncol):
        Gc = np.eye(n)
        rows = col == c
        Gc[rows] -= (B[rows] / np.diag(B)[rows][:, None])
        S = Gc @ S
    E = S @ S @ (np.eye(n) - P @ np.linalg.pinv(Bc) @ Q @ B) @ S @ S
    Cmat = np.stack([O.vcycle(h, np.eye(n)[:, j]) for j in range(n)], axis=1)
    assert np.abs((np.eye(n) - Cmat @ B) - E).max() < 1e-10


def test_stationary_with_mcgs_closed_form():
    ch = C.weighted_lattice(32, seed=5)
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3, relax="mcgs"), tol=1e-14)
    assert info.converged
    assert np.abs(x - ch.exact).sum() < 1e-12
    ch = C.tandem_queue(32)
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3, relax="mcgs"), tol=1e-14)
    assert info.converged
    B = O.b_from_a(ch.to_scipy()).toarray()
    import scipy.linalg as sla
    ns = sla.null_space(B)[:, 0]
    assert np.abs(x - ns / ns.sum()).sum() < 1e-12
