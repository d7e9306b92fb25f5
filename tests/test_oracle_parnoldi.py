"""Pins of the oracle's multigrid-preconditioned Arnoldi method (Section 4.3):
the Arnoldi relation (C B) V_k = V_{k+1} H_k with C written out densely, the
orthonormal basis, H_k = V_k^t (C B) V_k, the nearest-to-zero Ritz pair on a
planted spectrum, and the dense / closed-form stationary vectors it reaches."""
import numpy as np
import scipy.linalg as sla

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C


def _grid(ch):
    return O.Grid(ch.nx, ch.ny, ch.periodic)


def test_arnoldi_relation_with_the_dense_cycle():
    ch = C.tandem_queue(10)
    h = O.setup(ch.to_scipy(), _grid(ch), 6, O.Options(levels=2))
    n = ch.n
    B = h.levels[0].B.toarray()
    Cm = np.stack([O.vcycle(h, np.eye(n)[:, j]) for j in range(n)], axis=1)
    k = 8
    V, H = O.parnoldi_basis(h, h.x0, k)
    assert np.abs(V.T @ V - np.eye(k + 1)).max() < 1e-12
    assert np.abs(Cm @ B @ V[:, :k] - V @ H).max() < 1e-11 * np.abs(H).max()
    assert np.abs(V[:, :k].T @ Cm @ B @ V[:, :k] - H[:k]).max() < 1e-11 * np.abs(H).max()
    assert np.allclose(np.tril(H, -2), 0.0)


def test_ritz_nearest_zero_on_a_planted_spectrum():
    rng = np.random.default_rng(4)
    k = 7
    S = rng.normal(size=(k, k))
    theta = np.array([0.9, -0.5, 1e-3, 2.0, 0.3 + 0.4j, 0.3 - 0.4j, 1.5])
    # a real matrix with that spectrum: real Schur-like block for the pair
    D = np.diag(theta.real)
    D[4, 5], D[5, 4] = 0.4, -0.4
    Hk = S @ D @ np.linalg.inv(S)
    Vk = np.linalg.qr(rng.normal(size=(30, k)))[0]
    x = O.ritz_nearest_zero(Hk, Vk)
    want = Vk @ S[:, 2]
    assert np.abs(x - want / want.sum()).max() < 1e-10


def test_parnoldi_reaches_the_dense_null_vector():
    ch = C.tandem_queue(16)
    h = O.setup(ch.to_scipy(), _grid(ch), 8, O.Options(levels=3))
    x, info = O.solve(h, tol=1e-13, max_cycles=100, method="parnoldi")
    assert info.converged
    ns = sla.null_space(O.b_from_a(ch.to_scipy()).toarray())[:, 0]
    assert np.abs(x - ns / ns.sum()).sum() < 1e-12
    assert x.min() >= 0 and abs(x.sum() - 1) < 1e-15


def test_parnoldi_restarts_and_closed_form():
    ch = C.weighted_lattice(32, seed=5)
    opts = O.Options(levels=3, gmres_m=3)          # forces restarts
    x, info, h = O.stationary(ch.to_scipy(), _grid(ch), 8, opts, tol=1e-13, max_cycles=200, method="parnoldi")
    assert info.converged and info.restarts >= 2
    assert np.abs(x - ch.exact).sum() < 1e-12
