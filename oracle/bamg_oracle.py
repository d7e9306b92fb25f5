"""Plain FP64 CPU oracle of the Bootstrap AMG method for Markov chains.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP library and imports nothing
from the package (its counter-based generator is its own implementation of the
published SplitMix64 definition).

Every function cites the passage of Bolten, Brandt, Brannick, Frommer, Kahl and
Livshits, "A Bootstrap Algebraic Multilevel method for Markov Chains"
(arXiv:1004.1451) it follows.  Where the operation has a plain definition the
code is that definition (sparse products via scipy, dense null space, pinv and
the generalised eigenproblem via LAPACK); the setup follows Algorithm 3 and
the interpolation Algorithm 2, step by step.  Vectorisation runs across
independent rows or fine points only.

Readings of points the paper leaves open are listed in the design notes; the
code states each one where it is used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# Counter-based generator for the initial test vectors (SplitMix64, Steele,
# Lea and Flood 2014): h = mix(key + GAMMA), key = (seed ^ stream*GAMMA) + idx,
# u = (h >> 11) * 2^-53.
# ---------------------------------------------------------------------------
_GAMMA = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1
STREAM_TV = 1


def _splitmix_u01(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    g = np.uint64(_GAMMA)
    with np.errstate(over="ignore"):
        key = (np.uint64(seed & _MASK) ^ (np.uint64(stream) * g)) + idx.astype(np.uint64)
        z = key + g
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def initial_tvs(n: int, r: int, seed: int) -> np.ndarray:
    """Random initial test vectors, entry (i, k) = u(seed, TV, i*r + k) in [0,1)
    (Section 1, step 1: r test vectors per level; uniform(0,1) reading)."""
    idx = np.arange(n * r, dtype=np.uint64)
    return _splitmix_u01(seed, STREAM_TV, idx).reshape(n, r)


# ---------------------------------------------------------------------------
# Problem (Section 2): A column stochastic, B = I - A.
# ---------------------------------------------------------------------------
def b_from_a(A: sp.csr_matrix) -> sp.csr_matrix:
    """B = I - A (Section 1, eq. ax and the definition of B).  The diagonal is
    always stored, so the structural pattern of B is that of A plus I."""
    n = A.shape[0]
    B = (sp.identity(n, format="csr") - A).tocsr()
    # keep explicit zeros out of the picture: structure = pattern(A) U diag
    pat = (abs(A).astype(bool) + sp.identity(n, format="csr", dtype=bool)).tocsr()
    pat.sort_indices()
    vals = np.asarray(B[pat.nonzero()]).ravel()
    rows, cols = pat.nonzero()
    out = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return _with_pattern(out, pat)


def _with_pattern(M: sp.csr_matrix, pat: sp.csr_matrix) -> sp.csr_matrix:
    """Return M's values on exactly the structural pattern ``pat`` (entries of
    pat absent from M are stored as explicit zeros)."""
    pat = pat.tocsr(); pat.sort_indices()
    Mc = M.tocsr(); Mc.sum_duplicates(); Mc.sort_indices()
    rows = np.repeat(np.arange(pat.shape[0]), np.diff(pat.indptr))
    vals = np.asarray(Mc[rows, pat.indices]).ravel() if pat.nnz else np.zeros(0)
    out = sp.csr_matrix((vals.astype(np.float64), pat.indices.copy(), pat.indptr.copy()), shape=pat.shape)
    out.has_sorted_indices = True
    return out


# ---------------------------------------------------------------------------
# Grids and full coarsening (Section 3; Section 5: every other grid point in
# both directions).  State s = a*ny + b.
#
# Along one grid direction of length m the coarse coordinates are the even
# positions, and on a side that is not periodic also the last position m-1:
# the experiments of Section 5 use sides 2^k + 1, where "every other point"
# keeps both ends of the side coarse, and this keeps both ends coarse on
# sides of any length.  A coarse coordinate y has rank (y + 1) // 2 among the
# coarse coordinates of its side, so a non-periodic side of m points leaves
# m // 2 + 1 of them and a periodic side (m even) m / 2.
# ---------------------------------------------------------------------------
def coarse_coords(m: int, periodic: bool) -> np.ndarray:
    """The coarse positions 0 <= y < m of one grid direction, ascending."""
    c = np.arange(m) % 2 == 0
    if not periodic and m > 0:
        c[m - 1] = True
    return np.nonzero(c)[0]


def coarse_side(m: int, periodic: bool) -> int:
    return len(coarse_coords(m, periodic))


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    periodic: bool

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def coarse(self) -> "Grid":
        return Grid(coarse_side(self.nx, self.periodic), coarse_side(self.ny, self.periodic), self.periodic)

    def can_coarsen(self) -> bool:
        """Full coarsening keeps every coarse stencil within the 3x3 box only
        for even periodic sides with coarse side >= 3; a non-periodic grid
        must get smaller (a side of 1 or 2 points keeps every point)."""
        if self.periodic:
            return all(m % 2 == 0 and m // 2 >= 3 for m in (self.nx, self.ny))
        return self.coarse().n < self.n


def level_plan(grid: Grid, levels: int, coarse_max: int = 1024) -> list[Grid]:
    """Grids of levels 0..L.  ``levels`` counts the finest level; 0 = coarsen
    while n > coarse_max."""
    plan = [grid]
    while True:
        g = plan[-1]
        if levels > 0 and len(plan) >= levels:
            break
        if levels == 0 and g.n <= coarse_max:
            break
        if not g.can_coarsen():
            if levels > 0:
                raise ValueError("grid cannot be coarsened to the requested depth")
            break
        plan.append(g.coarse())
    return plan


def c_points(g: Grid) -> np.ndarray:
    """Fine indices of the coarse points (both coordinates coarse), in coarse
    order (row-major over the coarse coordinates)."""
    ca = coarse_coords(g.nx, g.periodic)
    cb = coarse_coords(g.ny, g.periodic)
    a, b = np.meshgrid(ca, cb, indexing="ij")
    return (a * g.ny + b).ravel()


def _dir_table(m: int, periodic: bool):
    """Per position y of a direction of length m: whether it is coarse, its
    rank among the coarse positions (-1 if fine), and the positions of the
    coarse neighbours that interpolate to it: y itself at a coarse position
    (one), y - 1 and y + 1 elsewhere (two; both exist since an F position is
    odd and the last position of a non-periodic side is coarse; periodic
    sides wrap)."""
    cc = coarse_coords(m, periodic)
    isc = np.zeros(m, dtype=bool); isc[cc] = True
    rank = np.full(m, -1, dtype=np.int64); rank[cc] = np.arange(len(cc))
    y = np.arange(m)
    lo = np.where(isc, y, (y - 1) % m)
    hi = np.where(isc, y, (y + 1) % m)
    return isc, rank, lo, hi, np.where(isc, 1, 2)


def neighbour_slots(g: Grid) -> np.ndarray:
    """Coarse neighbourhood N_i of every point (eq. neighbor_def).  Reading:
    the coarse points (a', b') with a' among the coarse neighbours of a in
    its direction and b' among those of b (``_dir_table``), leaving out the
    point itself.  When the coarse positions are exactly the even ones this
    is the set of coarse points within Chebyshev distance 1; next to the last
    coarse position of a non-periodic even side it leaves out the coarse
    point across a coarse row or column, so that Q, B and P each reach one
    coarse step and every coarse operator keeps the 3x3 box stencil.
    Returns an (n, 4) int array of coarse indices, -1 where a slot is empty,
    slots in lexicographic order of the offset (da, db)."""
    cg = g.coarse()
    isa, ra, loa, hia, na_ = _dir_table(g.nx, g.periodic)
    isb, rb, lob, hib, nb_ = _dir_table(g.ny, g.periodic)
    s = np.arange(g.n)
    a, b = s // g.ny, s % g.ny
    fine = ~(isa[a] & isb[b])
    slots = np.full((g.n, 4), -1, dtype=np.int64)
    for ka in (0, 1):
        for kb in (0, 1):
            ok = fine & (ka < na_[a]) & (kb < nb_[b])
            idx = np.nonzero(ok)[0]
            pa = (loa if ka == 0 else hia)[a[idx]]
            pb = (lob if kb == 0 else hib)[b[idx]]
            slots[idx, ka * nb_[b[idx]] + kb] = ra[pa] * cg.ny + rb[pb]
    return slots


def is_c_point(g: Grid) -> np.ndarray:
    isa = np.zeros(g.nx, dtype=bool); isa[coarse_coords(g.nx, g.periodic)] = True
    isb = np.zeros(g.ny, dtype=bool); isb[coarse_coords(g.ny, g.periodic)] = True
    s = np.arange(g.n)
    return isa[s // g.ny] & isb[s % g.ny]



@dataclass
class Coarsening:
    """The C/F splitting of one level and the candidate sets N_i: ``isC`` per
    point, ``cpts`` the fine index of every coarse point (ascending, so coarse
    index = rank among the C points), ``slots`` (n, K) the coarse indices of
    N_i, -1 where empty."""
    isC: np.ndarray
    cpts: np.ndarray
    slots: np.ndarray
    rounds: int = 0                              # CR relaxations performed
    rho: list = field(default_factory=list)      # CR estimate of each

    @property
    def nc(self) -> int:
        return len(self.cpts)


def grid_coarsening(g: Grid) -> Coarsening:
    """Full coarsening of a grid level (Section 5)."""
    return Coarsening(is_c_point(g), c_points(g), neighbour_slots(g))


# ---------------------------------------------------------------------------
# Coarsening without a grid: compatible relaxation (Section 3.1, Algorithm 1,
# eqs. frelax and meas1) from a standard independent set.
# ---------------------------------------------------------------------------
STREAM_CR = 16      # + level: the random start vectors of the CR relaxations


def graph_of(B: sp.csr_matrix) -> sp.csr_matrix:
    """G(B) without self-loops as a boolean CSR (edge i -> j for b_ij != 0).
    The stored pattern counts, not the values.  The coarsening needs a
    symmetric pattern (so that G(B) is an undirected graph); every coarse
    operator Q B P then has one too."""
    B = B.tocsr()
    G = sp.csr_matrix((np.ones(B.nnz, dtype=bool), B.indices.copy(), B.indptr.copy()), shape=B.shape)
    G.setdiag(False)
    G.eliminate_zeros()
    G.sort_indices()
    if (G != G.T).nnz:
        raise ValueError("coarsening without a grid needs a structurally symmetric matrix")
    return G


def independent_set(G: sp.csr_matrix, cand: np.ndarray) -> np.ndarray:
    """Maximal independent set of the candidate points in graph G (the
    standard independent set of Section 3.1): the candidates are visited in
    increasing index and one joins when none of its neighbours has joined
    (reading: index order, no weights)."""
    taken = np.zeros(G.shape[0], dtype=bool)
    ip, ix = G.indptr, G.indices
    for i in np.nonzero(cand)[0]:
        if not taken[ix[ip[i]:ip[i + 1]]].any():
            taken[i] = True
    return taken


def f_relax(B: sp.csr_matrix, isC: np.ndarray, u: np.ndarray, omega: float, nu: int):
    """nu sweeps of eq. frelax with omega-Jacobi, M = diag(B)/omega:
    u_F <- u_F - omega D_FF^-1 B_FF u_F (the homogeneous F-relaxation; u stays
    zero on C).  Returns (u^{nu-1}, u^nu)."""
    F = ~isC
    Bff = B[F][:, F]
    s = omega / B.diagonal()[F]
    uf = u[F].copy()
    prev = uf
    for _ in range(nu):
        prev = uf
        uf = uf - s * (Bff @ uf)
    a = np.zeros_like(u); b = np.zeros_like(u)
    a[F] = prev; b[F] = uf
    return a, b


def cr_coarsen(B: sp.csr_matrix, level: int, omega: float, theta: float, nu: int, seed: int,
               max_rounds: int, C0: np.ndarray | None = None):
    """Algorithm 1 (compatible_relaxation).  C starts from C0, by default the
    independent set of all points in G(B).  Each round relaxes nu times from
    u^0_i ~ U[1, 2] on F (zero on C; u^0 of round k at point i is
    1 + u(seed, STREAM_CR + level, k n + i)) and estimates rho_f =
    (||u^nu||_2 / ||u^0||_2)^(1/nu) (eq. meas1).  While rho_f > theta, the
    F points with |u_i^nu| > theta |u_i^(nu-1)| (the ratio test written as a
    product) form the candidate set N, and an independent set of N (in the
    graph restricted to N) joins C.  Readings: the loop also ends when N is
    empty and after max_rounds relaxations.  Returns (isC, rounds, rhos)."""
    n = B.shape[0]
    G = graph_of(B)
    isC = independent_set(G, np.ones(n, dtype=bool)) if C0 is None else C0.astype(bool).copy()
    rhos = []
    for k in range(max_rounds):
        F = ~isC
        u0 = np.where(F, 1.0 + _splitmix_u01(seed, STREAM_CR + level, np.arange(n, dtype=np.uint64) + k * n), 0.0)
        prev, last = f_relax(B, isC, u0, omega, nu)
        n0 = np.sqrt(np.sum(u0 * u0))
        rho = (np.sqrt(np.sum(last * last)) / n0) ** (1.0 / nu) if n0 > 0 else 0.0
        rhos.append(rho)
        if not rho > theta:
            break
        N = F & (np.abs(last) > theta * np.abs(prev))
        if not N.any():
            break
        isC = isC | independent_set(G, N)
    return isC, len(rhos), rhos


def graph_slots(B: sp.csr_matrix, isC: np.ndarray, z: int) -> np.ndarray:
    """N_i of eq. neighbor_def without a grid: the C points j != i reachable
    from i by a path of length <= z in G(B), as coarse indices in ascending
    order, padded with -1 to the largest |N_i|."""
    G = graph_of(B).astype(np.int64)
    reach = G.copy()
    for _ in range(z - 1):
        reach = ((reach + reach @ G) > 0).astype(np.int64)
    reach = reach.tocsr()
    reach.setdiag(0)
    reach.eliminate_zeros()
    reach.sort_indices()
    cidx = np.cumsum(isC) - 1
    lists = []
    for i in range(B.shape[0]):
        js = reach.indices[reach.indptr[i]:reach.indptr[i + 1]]
        lists.append(cidx[js[isC[js]]])
    K = max(1, max(len(x) for x in lists))
    slots = np.full((B.shape[0], K), -1, dtype=np.int64)
    for i, x in enumerate(lists):
        slots[i, :len(x)] = x
    return slots


def cr_coarsening(B: sp.csr_matrix, level: int, opts) -> Coarsening:
    """Coarsening of a level without a grid: compatible relaxation, then the
    candidate sets N_i at graph distance <= opts.nbr_dist."""
    isC, rounds, rhos = cr_coarsen(B, level, opts.omega, opts.cr_theta, opts.cr_nu, opts.seed, opts.cr_rounds)
    slots = graph_slots(B, isC, opts.nbr_dist)
    return Coarsening(isC, np.nonzero(isC)[0], slots, rounds, rhos)


# ---------------------------------------------------------------------------
# Relaxation: omega-Jacobi, M = diag(B)/omega (Section 3, eq. amg_relax).
# ---------------------------------------------------------------------------
def jacobi(B: sp.csr_matrix, X: np.ndarray, omega: float, nu: int, F: np.ndarray | None = None) -> np.ndarray:
    """nu sweeps of X <- X + omega D^-1 (F - B X), D = diag(B); F = 0 for the
    homogeneous test-vector relaxation (Algorithm 3)."""
    s = omega / B.diagonal()
    s = s[:, None] if X.ndim == 2 else s
    for _ in range(nu):
        R = -(B @ X) if F is None else F - B @ X
        X = X + s * R
    return X


# Multicolour Gauss-Seidel, the other deterministic relaxation of Section 3
# (Gauss-Seidel is named next to Jacobi there): the points are split into
# colours such that no two points of one colour are coupled, and one sweep
# updates the colours in order, each colour from the latest values of the
# others (so within a colour the order does not matter).
# ---------------------------------------------------------------------------
def _dir_colour(a: np.ndarray, m: int, periodic: bool) -> tuple[np.ndarray, int]:
    """Colours of positions a along one grid direction of length m: 0 and 1
    alternate; on a periodic direction of odd length the last position gets
    colour 2, so neighbours a, a+1 (mod m) always differ."""
    if periodic and m % 2 == 1 and m > 1:
        return np.where(a == m - 1, 2, a % 2), 3
    return a % 2, 2


def colours(g: Grid) -> tuple[np.ndarray, int]:
    """Colour of every state s = a*ny + b and the number of colours: the pair
    of direction colours (ca, cb) numbered ca * (colours of b) + cb.  Two
    distinct states within Chebyshev distance 1 differ by one step in some
    direction, hence in that direction's colour."""
    s = np.arange(g.n)
    ca, na = _dir_colour(s // g.ny, g.nx, g.periodic)
    cb, nb = _dir_colour(s % g.ny, g.ny, g.periodic)
    return ca * nb + cb, na * nb


def check_colouring(M: sp.csr_matrix, col: np.ndarray) -> None:
    """Raise if an off-diagonal entry of M couples two points of one colour
    (Gauss-Seidel by colours needs them independent)."""
    C = sp.coo_matrix(M)
    bad = (C.row != C.col) & (col[C.row] == col[C.col])
    if np.any(bad):
        raise ValueError("multicolour Gauss-Seidel: %d couplings inside one colour" % int(bad.sum()))


def mcgs(B: sp.csr_matrix, X: np.ndarray, col: np.ndarray, ncol: int, w: float, nu: int,
         F: np.ndarray | None = None) -> np.ndarray:
    """nu multicolour Gauss-Seidel sweeps on B X = F (F = 0 when None): for
    each colour c in order, x_i <- x_i + w (f_i - (B x)_i) / b_ii on the points
    of colour c, with the current values of all other points."""
    X = X.copy()
    D = B.diagonal()
    for _ in range(nu):
        for c in range(ncol):
            rows = np.nonzero(col == c)[0]
            if len(rows) == 0:
                continue
            Bc = B[rows]
            Rr = -(Bc @ X) if F is None else F[rows] - Bc @ X
            d = D[rows][:, None] if X.ndim == 2 else D[rows]
            X[rows] = X[rows] + w * Rr / d
    return X


def relax(lv, X: np.ndarray, opts, nu: int, F: np.ndarray | None = None) -> np.ndarray:
    """The configured relaxation on B_l X = F: omega-Jacobi or multicolour
    Gauss-Seidel."""
    if opts.relax == "mcgs":
        col, ncol = colours(lv.grid)
        return mcgs(lv.B, X, col, ncol, opts.gs_omega, nu, F)
    return jacobi(lv.B, X, opts.omega, nu, F)


def tv_weights(B: sp.csr_matrix, X: np.ndarray) -> np.ndarray:
    """omega_k = 1/||B x_k||_2^2 (Section 3.2: the squared inverse of the
    residual norm of B x = 0), floored at (1e-14 ||x_k||_2)^2 so that an exact
    null vector gets a finite weight."""
    res2 = np.sum((B @ X) ** 2, axis=0)
    x2 = np.sum(X ** 2, axis=0)
    return 1.0 / np.maximum(res2, 1e-28 * x2)


# ---------------------------------------------------------------------------
# Least-squares interpolation, Algorithm 2 (greedy choice of J_i) with the
# functional of eq. LSfuncrowi.
# ---------------------------------------------------------------------------
PIVOT_RTOL = 1e-10


def _masked_solve(G: np.ndarray, rhs: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Solve G_SS z = rhs_S per point; z = 0 outside S (batched over points)."""
    m = S[:, :, None] & S[:, None, :]
    M = np.where(m, G, 0.0) + np.eye(G.shape[1])[None] * (~S)[:, :, None]
    return np.linalg.solve(M, (rhs * S)[..., None])[..., 0]


def ls_fit(X: np.ndarray, w: np.ndarray, g, caliber: int, order: bool = False):
    """Interpolation P (n_f x n_c) for a coarsening ``g``: a Grid (full
    coarsening) or a Coarsening (isC, cpts, slots).

    C points get a unit row at their coarse index.  For every F point i with
    slots N_i: G_st = sum_k w_k x_s^k x_t^k, b_s = sum_k w_k x_s^k x_i^k,
    sigma = sum_k w_k (x_i^k)^2, so min_P L(P; S) = sigma - b_S^T G_SS^-1 b_S.
    Greedy (Algorithm 2): starting from J = {}, add the admissible g in
    N_i \\ J with the smallest min L(J u {g}) (strict minimum, ties to the lower
    slot) until |J| >= c or no admissible candidate is left.  g is admissible
    when its Schur-complement pivot G_gg - G_gJ G_JJ^-1 G_Jg exceeds
    1e-10 G_gg.  If no slot is admissible, the first slot gets weight 1.
    Weights p = G_JJ^-1 b_J.  Returns (P csr with ascending columns, J mask
    (n, K), slots (n, K)), and with ``order`` also the (n, K) slot chosen at
    each greedy step (-1 after the last).
    """
    cs = grid_coarsening(g) if isinstance(g, Grid) else g
    n, R = X.shape
    slots, isC, cpts = cs.slots, cs.isC, cs.cpts
    K = slots.shape[1]
    nc = len(cpts)
    fine_of_coarse = cpts                       # coarse index -> fine index
    valid = slots >= 0
    Xs = X[fine_of_coarse[np.where(valid, slots, 0)]]          # (n, K, R)
    Xs = Xs * valid[:, :, None]
    G = np.einsum("pak,pbk,k->pab", Xs, Xs, w)
    b = np.einsum("pak,pk,k->pa", Xs, X, w)
    sigma = np.einsum("pk,pk,k->p", X, X, w)

    J = np.zeros((n, K), dtype=bool)
    steps = np.full((n, K), -1, dtype=np.int64)
    done = isC.copy()
    for step in range(min(K, caliber)):
        best_L = np.full(n, np.inf)
        best_g = np.full(n, -1)
        for s_ in range(K):
            cand = (~done) & valid[:, s_] & (~J[:, s_]) & (J.sum(1) < caliber)
            ix = np.nonzero(cand)[0]
            if len(ix) == 0:
                continue
            Gi, bi, Ji = G[ix], b[ix], J[ix]
            Gjg = Gi[:, :, s_]
            piv = Gi[:, s_, s_] - np.einsum("pa,pa->p", Gjg * Ji, _masked_solve(Gi, Gjg, Ji))
            adm = piv > PIVOT_RTOL * Gi[:, s_, s_]
            # the functional only for admissible candidates (an inadmissible
            # one may make G_SS exactly singular)
            S = Ji.copy(); S[:, s_] = True
            L = np.full(len(ix), np.inf)
            if np.any(adm):
                L[adm] = sigma[ix[adm]] - np.einsum("pa,pa->p", bi[adm] * S[adm], _masked_solve(Gi[adm], bi[adm], S[adm]))
            better = adm & (L < best_L[ix])
            best_L[ix] = np.where(better, L, best_L[ix])
            best_g[ix] = np.where(better, s_, best_g[ix])
        took = best_g >= 0
        J[np.nonzero(took)[0], best_g[took]] = True
        steps[took, step] = best_g[took]
        done |= ~took
    fpts = np.nonzero((~isC) & (J.sum(1) > 0))[0]
    p = np.zeros((n, K))
    p[fpts] = _masked_solve(G[fpts], b[fpts], J[fpts])
    empty = (~isC) & (J.sum(1) == 0)
    if np.any(empty & ~valid[:, 0]):
        raise ValueError("an F point has no coarse neighbour")
    J[empty, 0] = True
    p[empty, 0] = 1.0

    rows, cols, vals = [], [], []
    ci = np.nonzero(isC)[0]
    cidx = np.cumsum(isC) - 1
    rows.append(ci); cols.append(cidx[ci]); vals.append(np.ones(len(ci)))
    fi = np.nonzero(~isC)[0]
    for s_ in range(K):
        sel = fi[J[fi, s_]]
        rows.append(sel); cols.append(slots[sel, s_]); vals.append(p[sel, s_])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))
    P.sort_indices()
    # structural pattern must hold even a weight that is exactly zero
    pat = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, nc)).astype(bool)
    P = _with_pattern(P, pat)
    J[isC] = False
    steps[isC] = -1
    if order:
        return P, J, slots, steps
    return P, J, slots


def averaging_q(P: sp.csr_matrix) -> sp.csr_matrix:
    """Q with sparsity(Q) = sparsity(P)^T and equal entries 1/|J_i| in column i
    (Section 4: averaging restriction, so 1^T Q = 1^T)."""
    P = P.tocsr()
    cnt = np.diff(P.indptr)
    vals = np.repeat(1.0 / np.maximum(cnt, 1), cnt)
    Pq = sp.csr_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)
    Q = Pq.T.tocsr()
    Q.sort_indices()
    return Q


def galerkin(Q: sp.csr_matrix, M: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Petrov-Galerkin product Q (M P) (Algorithm 3: B_{l+1} = Q B P and
    T_{l+1} = Q T P).  The stored pattern is the symbolic product of the three
    patterns (nothing dropped, even an entry that cancels to zero)."""
    def ones(X):
        X = X.tocsr()
        return sp.csr_matrix((np.ones(X.nnz), X.indices, X.indptr), shape=X.shape)
    pat = (ones(Q) @ (ones(M) @ ones(P))).astype(bool)
    return _with_pattern(Q @ (M @ P), pat)


def inject(X: np.ndarray, g) -> np.ndarray:
    """R x: the values at the coarse points (Section 1, step 4; injection);
    g is a Grid or a Coarsening."""
    return X[c_points(g) if isinstance(g, Grid) else g.cpts]


# ---------------------------------------------------------------------------
# Coarsest level (Algorithm 3, l = L; Section 4.2, eq. mgerrorprop).
# ---------------------------------------------------------------------------
@dataclass
class EigEntry:
    lam: complex          # eigenvalue (Im > 0 member of a conjugate pair)
    cols: tuple           # one column (real) or two (Re, Im)


def coarsest_svd(B: np.ndarray):
    """Singular value decomposition of B_L.  B_L has rank n-1 (1^T B_L = 0 and
    an irreducible fine chain), so the right singular vector of the smallest
    singular value spans null(B_L)."""
    return np.linalg.svd(B)


def coarsest_null(B: np.ndarray, T: np.ndarray, svd=None) -> np.ndarray:
    """Null vector y of B_L, scaled so that 1^T T_L y = 1."""
    _, _, vt = coarsest_svd(B) if svd is None else svd
    y = vt[-1].copy()
    return y / (np.ones(len(y)) @ T @ y)


def coarsest_pinv(B: np.ndarray, svd=None) -> np.ndarray:
    """Moore-Penrose inverse of the rank n-1 matrix B_L: the minimal-norm
    coarsest solve of the V-cycle (Section 4.2, after eq. mgerrorprop)."""
    u, s, vt = coarsest_svd(B) if svd is None else svd
    if len(s) == 1:
        return np.zeros_like(B)
    return (vt[:-1].T / s[:-1]) @ u[:, :-1].T


def normalise_eigvec(v: np.ndarray) -> np.ndarray:
    """||v||_2 = 1 and the largest-modulus entry (lowest index on ties, modulus
    compared as re^2 + im^2) real and positive."""
    v = v / np.sqrt(np.sum(v.real ** 2 + v.imag ** 2))
    m2 = v.real ** 2 + v.imag ** 2
    i = int(np.argmax(m2))
    ph = np.conj(v[i]) / np.sqrt(m2[i])
    return v * ph


DENSE_EIG_MAX = 256


def _nonzero_spectrum(B: np.ndarray, T: np.ndarray, want: int):
    """Eigenpairs of B v = lam T v with lam != 0 and the smallest |lam|.

    Small levels: the full generalised problem (QZ), dropping the null
    eigenvalue.  Larger levels: ARPACK (implicitly restarted Arnoldi) on the
    exact shift-invert operator v -> u with [[B, 1], [1^T T, 0]] [u; mu] =
    [T v; 0], whose eigenvalues on {1^T T v = 0} are 1/lam; every eigenvector
    of a nonzero lam lies in that set because 1^T B = 0."""
    n = B.shape[0]
    if n <= DENSE_EIG_MAX:
        lam, vec = sla.eig(B, T)
        order = np.argsort(np.abs(lam), kind="stable")
        keep = order[1:]
        return lam[keep], vec[:, keep]
    import scipy.sparse.linalg as spla
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = B
    K[:n, n] = 1.0
    K[n, :n] = np.ones(n) @ T
    lu = sla.lu_factor(K)

    def op(v):
        rhs = np.zeros(n + 1, dtype=np.result_type(v, np.float64))
        rhs[:n] = T @ v
        return sla.lu_solve(lu, rhs)[:n]

    L = spla.LinearOperator((n, n), matvec=op, dtype=np.float64)
    theta, vec = spla.eigs(L, k=min(want + 2, n - 2), which="LM", tol=1e-14,
                           ncv=min(n - 1, max(2 * want + 10, 40)), maxiter=5000)
    return 1.0 / theta, vec


def coarsest_eigs(B: np.ndarray, T: np.ndarray, k: int, svd=None):
    """The k eigenpairs of B_L x = lam T_L x of smallest |lam| (Algorithm 3,
    l = L).  lam_0 = 0 with the null vector y; the other k-1 follow in order of
    |lam| (a conjugate pair counts as two and is never split, so a pair at the
    cut adds one more).  A real eigenvector gives one column, a pair the real
    and imaginary parts of the member with Im(lam) > 0.  Returns (y, entries,
    V) with V the real columns [y, ...]."""
    n = B.shape[0]
    y = coarsest_null(B, T, svd)
    cols = [y]
    entries = [EigEntry(0.0, (0,))]
    if n > 1 and k > 1:
        lam, vec = _nonzero_spectrum(B, T, k - 1)
        # order by |lam|; conjugates are adjacent with the Im > 0 member first
        idx = sorted(range(len(lam)), key=lambda i: (round(abs(lam[i]), 12), -np.sign(lam[i].imag), i))
        taken, used = 0, set()
        for j in idx:
            if taken >= k - 1:
                break
            if j in used:
                continue
            if lam[j].imag == 0.0 or abs(lam[j].imag) <= 1e-12 * abs(lam[j]):
                v = normalise_eigvec(vec[:, j].astype(np.complex128)).real
                entries.append(EigEntry(complex(lam[j].real, 0.0), (len(cols),)))
                cols.append(v)
                taken += 1
                used.add(j)
            else:
                v = vec[:, j] if lam[j].imag > 0 else np.conj(vec[:, j])
                lj = lam[j] if lam[j].imag > 0 else np.conj(lam[j])
                v = normalise_eigvec(v)
                entries.append(EigEntry(complex(lj), (len(cols), len(cols) + 1)))
                cols.append(v.real.copy()); cols.append(v.imag.copy())
                taken += 2
                used.add(j)
                # the conjugate partner: the nearest eigenvalue to conj(lam_j)
                partner = min((i for i in idx if i not in used), key=lambda i: abs(lam[i] - np.conj(lam[j])), default=None)
                if partner is not None:
                    used.add(partner)
    return y, entries, np.stack(cols, axis=1)


# ---------------------------------------------------------------------------
# Up-leg eigenvector relaxation and eigenvalue update (Algorithm 3).
# ---------------------------------------------------------------------------
def eig_relax(B, T, V: np.ndarray, entries, omega: float, nu: int, gs=None):
    """Relax (B - lam_i T) x_i = 0 with omega-Jacobi, D_lam = diag(B) -
    lam diag(T), complex arithmetic for a conjugate pair (x = Re + i Im); then
    lam_i = <B x, x>/<T x, x> = x^H B x / x^H T x for i >= 1 (lam_0 = 0 is not
    updated).  With gs = (colours, ncol, w) the sweeps are multicolour
    Gauss-Seidel with weight w instead.  Returns new V and entries."""
    V = V.copy()
    dB = B.diagonal(); dT = T.diagonal()
    out = []
    for e in entries:
        if len(e.cols) == 1:
            x = V[:, e.cols[0]].astype(np.complex128)
        else:
            x = V[:, e.cols[0]] + 1j * V[:, e.cols[1]]
        lam = e.lam
        D = dB - lam * dT
        for _ in range(nu):
            if gs is None:
                x = x - omega * (B @ x - lam * (T @ x)) / D
                continue
            col, ncol, w = gs
            for c in range(ncol):
                rows = np.nonzero(col == c)[0]
                if len(rows) == 0:
                    continue
                x[rows] = x[rows] - w * (B[rows] @ x - lam * (T[rows] @ x)) / D[rows]
        if e.cols != (0,):
            lam = np.vdot(x, B @ x) / np.vdot(x, T @ x)
            if len(e.cols) == 1:
                lam = complex(lam.real, 0.0)
        if len(e.cols) == 1:
            V[:, e.cols[0]] = x.real
        else:
            V[:, e.cols[0]] = x.real; V[:, e.cols[1]] = x.imag
        out.append(EigEntry(complex(lam), e.cols))
    return V, out


# ---------------------------------------------------------------------------
# Setup: the MLE cycle of Algorithm 3 (mu = 1) followed by the recomputation
# of every P, B and T with the enriched test sets (Section 1).
# ---------------------------------------------------------------------------
@dataclass
class Options:
    levels: int = 0
    nu_setup: int = 4
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.7
    caliber: int = 4
    n_eig: int = 6
    gmres_m: int = 50
    seed: int = 0
    coarse_max: int = 1024
    mu: int = 1                # cycle index of Algorithm 3: 1 = V, 2 = W
    relax: str = "jacobi"      # or "mcgs": multicolour Gauss-Seidel
    gs_omega: float = 1.0      # weight of the Gauss-Seidel update
    # coarsening without a grid (Algorithm 1 and eq. neighbor_def)
    cr_theta: float = 0.85     # CR tolerance theta
    cr_nu: int = 8             # CR sweeps per estimate
    cr_rounds: int = 64        # at most this many CR relaxations per level
    nbr_dist: int = 1          # z: path length of the candidate sets N_i


@dataclass
class Level:
    grid: Grid | None          # None: no grid, coarsened by compatible relaxation
    B: sp.csr_matrix
    T: sp.csr_matrix
    P: sp.csr_matrix | None = None
    Q: sp.csr_matrix | None = None
    J: np.ndarray | None = None
    U: np.ndarray | None = None       # relaxed random test vectors
    V: np.ndarray | None = None       # eigenvector approximations (real columns)
    cs: Coarsening | None = None      # C/F splitting and N_i (None on the coarsest level)
    decided: bool = False             # cs fixed (it is decided once, on the first pass)


@dataclass
class Hierarchy:
    levels: list
    opts: Options
    pinv: np.ndarray
    y: np.ndarray
    entries: list
    x0: np.ndarray
    first_pass: list = field(default_factory=list)   # (P, B, T) of the down-leg


# Optional progress report: a callable taking one string, called after each
# level is built (long runs print through it; no effect on any result).
PROGRESS = None


def build_level(lv: Level, X: np.ndarray, opts: Options):
    """One level of the hierarchy from test set X: weights, LS fit, Q,
    B_{l+1}, T_{l+1} (Algorithm 3)."""
    w = tv_weights(lv.B, X)
    P, J, _ = ls_fit(X, w, lv.cs if lv.cs is not None else lv.grid, opts.caliber)
    Q = averaging_q(P)
    Bc = galerkin(Q, lv.B, P)
    Tc = galerkin(Q, lv.T, P)
    if PROGRESS is not None:
        PROGRESS(f"level of {lv.B.shape[0]} rows built from {X.shape[1]} test vectors")
    return P, Q, J, Bc, Tc


def _coarsening(levels: list, l: int, plan, opts: Options) -> Coarsening | None:
    """The coarsening of level l, fixed the first time the level is reached;
    None marks the coarsest level.  On a grid it follows the level plan;
    without one (plan None) level l is coarsened by compatible relaxation
    while l + 1 < opts.levels (or, with opts.levels = 0, while n_l >
    opts.coarse_max)."""
    lv = levels[l]
    if lv.decided:
        return lv.cs
    if plan is not None:
        cs = grid_coarsening(plan[l]) if l < len(plan) - 1 else None
    else:
        n = lv.B.shape[0]
        more = (l + 1 < opts.levels) if opts.levels > 0 else (n > opts.coarse_max)
        cs = cr_coarsening(lv.B, l, opts) if more else None
        if cs is not None and not (1 <= cs.nc < n):
            if opts.levels > 0:
                raise ValueError("compatible relaxation cannot coarsen level %d to the requested depth" % l)
            cs = None
    lv.cs, lv.decided = cs, True
    return cs


def mle_cycle(levels: list, l: int, plan, opts: Options, use_v: bool):
    """Algorithm 3 (bootamg_mle) from level l.  levels[l] holds B_l, T_l and
    U_l (and V_l from an earlier cycle when use_v).  Relax U_l; then mu times:
    fit P_l to U_l (joined by V_l after the first round, or from the start
    when use_v), Q_l, B_{l+1}, T_{l+1}, inject U_{l+1} = R U_l, recurse, and
    bring the coarse eigenvector approximations up: V_l = P_l V_{l+1},
    relaxed on (B_l - lam T_l) v = 0 with lam updated.  The coarsest level
    solves its eigenproblem.  Returns the eigenvalue entries."""
    lv = levels[l]
    if _coarsening(levels, l, plan, opts) is None:
        _, entries, V = coarsest_eigs(lv.B.toarray(), lv.T.toarray(), opts.n_eig)
        lv.V = V
        return entries
    if opts.relax == "mcgs":
        check_colouring(lv.B, colours(lv.grid)[0])
    lv.U = relax(lv, lv.U, opts, opts.nu_setup)
    entries = None
    for m in range(opts.mu):
        X = np.concatenate([lv.U, lv.V], axis=1) if (use_v or m > 0) else lv.U
        P, Q, J, Bc, Tc = build_level(lv, X, opts)
        lv.P, lv.Q, lv.J = P, Q, J
        if len(levels) == l + 1:
            levels.append(Level(plan[l + 1] if plan is not None else None, Bc, Tc))
        else:
            levels[l + 1].B, levels[l + 1].T = Bc, Tc
        levels[l + 1].U = inject(lv.U, lv.cs)
        entries = mle_cycle(levels, l + 1, plan, opts, use_v)
        gs = None
        if opts.relax == "mcgs":
            col, ncol = colours(lv.grid)
            check_colouring(lv.T, col)
            gs = (col, ncol, opts.gs_omega)
        lv.V, entries = eig_relax(lv.B, lv.T, lv.P @ levels[l + 1].V, entries, opts.omega, opts.nu_setup, gs)
    return entries


def _first_level(A: sp.csr_matrix, grid: Grid | None, r: int, opts: Options):
    """Level 0 with the random test vectors; grid None: no grid (compatible
    relaxation coarsens every level)."""
    if grid is None and opts.relax != "jacobi":
        raise ValueError("multicolour Gauss-Seidel needs a grid")
    plan = level_plan(grid, opts.levels, opts.coarse_max) if grid is not None else None
    n = A.shape[0]
    lv = Level(grid, b_from_a(A.tocsr()), sp.identity(n, format="csr"))
    lv.U = initial_tvs(n, r, opts.seed)
    return plan, [lv]


def setup(A: sp.csr_matrix, grid: Grid, r: int, opts: Options) -> Hierarchy:
    """The setup of Section 1: one MLE cycle (Algorithm 3 with opts.mu) from
    the random test vectors, then every P, B, T recomputed from U u V."""
    plan, levels = _first_level(A, grid, r, opts)
    entries = mle_cycle(levels, 0, plan, opts, use_v=False)
    first = [(lv.P, lv.B, lv.T) for lv in levels]
    x0 = levels[0].V[:, 0] / np.sum(levels[0].V[:, 0])
    # recompute every P, B, T from the enriched sets U u V
    for l in range(len(levels) - 1):
        lv = levels[l]
        X = np.concatenate([lv.U, lv.V], axis=1)
        P, Q, J, Bc, Tc = build_level(lv, X, opts)
        lv.P, lv.Q, lv.J = P, Q, J
        levels[l + 1].B, levels[l + 1].T = Bc, Tc
    if opts.relax == "mcgs":
        for lv in levels[:-1]:
            check_colouring(lv.B, colours(lv.grid)[0])
    cl = levels[-1]
    Bd = cl.B.toarray()
    svd = coarsest_svd(Bd)
    return Hierarchy(levels, opts, coarsest_pinv(Bd, svd), coarsest_null(Bd, cl.T.toarray(), svd), entries, x0, first)


def mle_iteration(A: sp.csr_matrix, grid: Grid, r: int, opts: Options | None = None, tol: float = 1e-8,
                  max_cycles: int = 50):
    """The MLE iteration as a stand-alone solver (Section 4.1): setup cycles
    (Algorithm 3 with opts.mu) repeated, the first from the random test
    vectors and each later one fitting P_l to U_l u V_l of the previous cycle
    on every level (the enriched test sets of Section 1); after each cycle
    x = V_0[:, 0] / sum is the iterate, until ||B x||_1 / ||x||_1 <= tol.
    Returns (x, info with cycles = MLE cycles, levels)."""
    opts = opts or Options()
    plan, levels = _first_level(A, grid, r, opts)
    B = levels[0].B
    info = SolveInfo()
    x = None
    for k in range(max_cycles):
        mle_cycle(levels, 0, plan, opts, use_v=k > 0)
        info.cycles += 1
        v = levels[0].V[:, 0]
        x = v / np.sum(v)
        rel = np.sum(np.abs(B @ x)) / np.sum(np.abs(x))
        info.residual_l1 = rel
        info.history.append(rel)
        if rel <= tol:
            info.converged = True
            break
    return x, info, levels


# ---------------------------------------------------------------------------
# Solve: V(nu1, nu2)-cycle (eq. mgerrorprop) as right preconditioner of
# flexible GMRES on B x = 0 (Section 4.2).
# ---------------------------------------------------------------------------
def vcycle(h: Hierarchy, f: np.ndarray, l: int = 0) -> np.ndarray:
    lv = h.levels[l]
    if l == len(h.levels) - 1:
        return h.pinv @ f
    o = h.opts
    e = relax(lv, np.zeros_like(f), o, o.nu_pre, F=f)
    r = f - lv.B @ e
    ec = vcycle(h, lv.Q @ r, l + 1)
    e = e + lv.P @ ec
    return relax(lv, e, o, o.nu_post, F=f)


@dataclass
class SolveInfo:
    cycles: int = 0
    restarts: int = 0
    residual_l1: float = np.inf
    clamped_mass: float = 0.0
    history: list = field(default_factory=list)
    converged: bool = False


def fgmres(h: Hierarchy, x: np.ndarray, tol: float, max_cycles: int):
    """Right-preconditioned flexible GMRES(m) for B x = 0 from x (Section 4.2;
    the flexible form because the preconditioner is applied as given).
    Arnoldi by modified Gram-Schmidt with one reorthogonalisation; the small
    least-squares problem min ||beta e1 - H y|| is solved with lstsq.  Inner
    iterations stop when the least-squares residual falls below
    0.5 * tol * ||x||_1 * ||r0||_2 / ||r0||_1; after every restart cycle x is
    scaled to sum one and the true ||B x||_1 / ||x||_1 decides convergence."""
    B = h.levels[0].B
    m = h.opts.gmres_m
    info = SolveInfo()
    x = x / np.sum(x)
    while True:
        r = -(B @ x)
        rel = np.sum(np.abs(r)) / np.sum(np.abs(x))
        info.residual_l1 = rel
        info.history.append(rel)
        if rel <= tol:
            info.converged = True
            break
        if info.cycles >= max_cycles:
            break
        beta = np.linalg.norm(r)
        inner_tol = 0.5 * tol * np.sum(np.abs(x)) * beta / np.sum(np.abs(r))
        Vk = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        y = np.zeros(0)
        for j in range(m):
            if info.cycles >= max_cycles:
                break
            z = vcycle(h, Vk[j])
            info.cycles += 1
            w = B @ z
            for _ in range(2):
                for i in range(j + 1):
                    c = np.dot(Vk[i], w)
                    H[i, j] += c
                    w = w - c * Vk[i]
            H[j + 1, j] = np.linalg.norm(w)
            Z.append(z)
            e1 = np.zeros(j + 2); e1[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            est = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y)
            if H[j + 1, j] == 0.0 or est <= inner_tol:
                break
            Vk.append(w / H[j + 1, j])
        if Z:
            x = x + np.stack(Z, axis=1) @ y
        x = x / np.sum(x)
        info.restarts += 1
    return x, info


# ---------------------------------------------------------------------------
# Multigrid-preconditioned Arnoldi (Section 4.3): Arnoldi on the operator C B
# (C = one V-cycle) from the setup's state-vector approximation y; the
# eigenvalue of H_k = V_k^t (C B) V_k closest to 0 and its eigenvector eta give
# the Ritz vector V_k eta as the approximation of the state vector.
# ---------------------------------------------------------------------------
def parnoldi_basis(h: Hierarchy, y: np.ndarray, k: int):
    """k Arnoldi steps on C B from y (modified Gram-Schmidt, two passes):
    returns V (n x (k+1), orthonormal columns) and H ((k+1) x k) with
    (C B) V[:, :k] = V H."""
    B = h.levels[0].B
    V = [y / np.linalg.norm(y)]
    H = np.zeros((k + 1, k))
    for j in range(k):
        w = vcycle(h, B @ V[j])
        for _ in range(2):
            for i in range(j + 1):
                c = np.dot(V[i], w)
                H[i, j] += c
                w = w - c * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
    return np.stack(V, axis=1), H


def ritz_nearest_zero(Hk: np.ndarray, Vk: np.ndarray) -> np.ndarray:
    """The eigenvalue of the square Hk closest to 0 (LAPACK's QR algorithm)
    and the Ritz vector Vk eta of its eigenvector, scaled to sum 1; the phase
    of eta makes its largest entry real (a real eigenvalue has a real
    eigenvector up to that phase)."""
    theta, S = np.linalg.eig(Hk)
    i = int(np.argmin(np.abs(theta)))
    eta = S[:, i]
    eta = eta * np.exp(-1j * np.angle(eta[np.argmax(np.abs(eta))]))
    x = Vk @ eta.real
    return x / np.sum(x)


def parnoldi(h: Hierarchy, x: np.ndarray, tol: float, max_cycles: int):
    """Multigrid-preconditioned Arnoldi (Section 4.3) restarted every m
    (= gmres_m) steps from the current Ritz vector.  After each step the Ritz
    vector of the eigenvalue of H_j closest to 0, scaled to sum 1, is the
    iterate; it stops when ||B x||_1/||x||_1 <= tol (the stopping rule of the
    GMRES path), at a breakdown, or after max_cycles applications of C."""
    B = h.levels[0].B
    m = h.opts.gmres_m
    info = SolveInfo()
    x = x / np.sum(x)
    while True:
        V = [x / np.linalg.norm(x)]
        H = np.zeros((m + 1, m))
        stop = False
        for j in range(m):
            w = vcycle(h, B @ V[j])
            info.cycles += 1
            for _ in range(2):
                for i in range(j + 1):
                    c = np.dot(V[i], w)
                    H[i, j] += c
                    w = w - c * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            x = ritz_nearest_zero(H[: j + 1, : j + 1], np.stack(V, axis=1))
            rel = np.sum(np.abs(B @ x)) / np.sum(np.abs(x))
            info.residual_l1 = rel
            info.history.append(rel)
            if rel <= tol:
                info.converged = True
                stop = True
            if stop or H[j + 1, j] == 0.0 or info.cycles >= max_cycles:
                stop = stop or info.cycles >= max_cycles
                break
            V.append(w / H[j + 1, j])
        info.restarts += 1
        if stop:
            break
    return x, info


def normalise(x: np.ndarray):
    """x >= 0 and sum(x) = 1 (Section 2: the state vector is non-negative);
    returns the vector and the mass removed by the clamp."""
    neg = np.sum(-x[x < 0])
    x = np.maximum(x, 0.0)
    return x / np.sum(x), neg


def solve(h: Hierarchy, tol: float = 1e-10, max_cycles: int = 200, x: np.ndarray | None = None,
          method: str = "fgmres"):
    """The state vector from the hierarchy: flexible GMRES (Section 4.2) or
    the multigrid-preconditioned Arnoldi method (Section 4.3)."""
    x = h.x0.copy() if x is None else x
    x, info = (parnoldi if method == "parnoldi" else fgmres)(h, x, tol, max_cycles)
    x, info.clamped_mass = normalise(x)
    B = h.levels[0].B
    info.residual_l1 = np.sum(np.abs(B @ x)) / np.sum(np.abs(x))
    return x, info


def stationary(A: sp.csr_matrix, grid: Grid, r: int, opts: Options | None = None,
               tol: float = 1e-10, max_cycles: int = 200, method: str = "fgmres"):
    opts = opts or Options()
    h = setup(A, grid, r, opts)
    x, info = solve(h, tol, max_cycles, method=method)
    return x, info, h
