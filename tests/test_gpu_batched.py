"""Batched form: several chains in one handle (bamg_setup_batched /
bamg_solve_batched), and replays of the captured V-cycle graph.

Chains never interact, so every chain's arithmetic in a batch is the same as
in a single-chain handle (same kernels, same per-chain reduction chunks):
batched and single-chain stationary vectors must agree to rounding (1e-13 in
the 1-norm; in practice bit for bit), and each must match the oracle to the
FP64 bar ||x - x_oracle||_1 <= 1e-9.  The caller's chain order is not the
depth order, so the row permutation in and out of the handle is exercised.
"""
import numpy as np
import pytest

from oracle import bamg_oracle as O
from paper_1004_1451_amd import chains as C

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1004_1451_amd import bamg as B  # noqa: E402
from tests.test_gpu_parity import _csr, _grid, _p_from_ell  # noqa: E402

COARSE_MAX = 100
R = 8


def _mix():
    # shallow chains first: depth order differs from the caller's order
    return [
        C.weighted_lattice(21, periodic=False, uniform_weights=True),   # 441 states, 3 levels
        C.tandem_queue(32),                                             # 1089, 3 levels
        C.weighted_lattice(48, seed=3),                                 # 2304 periodic, 4 levels
        C.tandem_queue(40),                                             # 1681, 4 levels
        C.tandem_queue(6),                                              # 49, 1 level (coarsest only)
    ]


def _blocks(x, off):
    return [x[off[c]:off[c + 1]] for c in range(len(off) - 1)]


@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
def test_batched_matches_single_and_oracle(precision):
    chains = _mix()
    opts = dict(levels=0, coarse_max=COARSE_MAX, precision=precision)
    h = B.BatchedHierarchy(chains, R, B.default_options(**opts))
    x = torch.empty(h.n, dtype=torch.float64, device="cuda")
    info, status, resid = h.solve_batched(x, tol=1e-13, max_cycles=300)
    assert info.converged and status.tolist() == [1] * len(chains), (status, resid)
    assert np.all(resid <= 1e-13)
    xs = _blocks(x.cpu().numpy(), h.offsets)
    for c, ch in enumerate(chains):
        xb = xs[c]
        assert xb.min() >= 0 and abs(xb.sum() - 1) < 1e-14, c
        x1, info1, h1 = B.stationary(ch, R, tol=1e-13, max_cycles=300, **opts)
        assert info1.converged
        assert np.abs(xb - x1).sum() <= 1e-13, (c, np.abs(xb - x1).sum())
        xo, _, _ = O.stationary(ch.to_scipy(), _grid(ch), R, O.Options(levels=0, coarse_max=COARSE_MAX), tol=1e-13)
        assert np.abs(xb - xo).sum() <= 1e-9, (c, np.abs(xb - xo).sum())
        h1.close()
    st = h.stats()
    assert st.n_levels == 4


def test_batched_per_chain_status_and_guess():
    chains = _mix()[:3]
    h = B.BatchedHierarchy(chains, R, B.default_options(levels=0, coarse_max=COARSE_MAX))
    x = torch.empty(h.n, dtype=torch.float64, device="cuda")
    info, status, resid = h.solve_batched(x, tol=1e-30, max_cycles=3)
    assert not info.converged and status.tolist() == [0, 0, 0]
    assert info.cycles == 3 and np.all(resid > 0)
    # continue from the caller's iterate (caller order in, caller order out)
    info, status, resid = h.solve_batched(x, tol=1e-12, max_cycles=300, use_guess=True)
    assert info.converged and status.tolist() == [1, 1, 1]
    for c, (ch, xb) in enumerate(zip(chains, _blocks(x.cpu().numpy(), h.offsets))):
        A = ch.to_scipy()
        assert np.abs(A @ xb - xb).sum() / xb.sum() <= 1e-11, c


def test_batched_errors():
    a, b = C.tandem_queue(8), C.tandem_queue(10)
    off, rp, ci, v, grids = B.concat_chains([a, b])
    # a column outside its own chain's block
    ci_bad = ci.copy()
    ci_bad[0] = off[1]
    import ctypes as Ct
    lib = B.load()

    def setup(ci_arr, grid_arr, offs, opts=None):
        h = Ct.c_void_p()
        drp = torch.as_tensor(rp, device="cuda")
        dci = torch.as_tensor(ci_arr, device="cuda")
        dv = torch.as_tensor(v, device="cuda")
        g = (B.Grid * len(grid_arr))(*[B.Grid(int(x), int(y), int(z)) for x, y, z in grid_arr])
        o = opts if opts is not None else B.default_options(levels=2)
        rc = lib.bamg_setup_batched(len(grid_arr), offs.ctypes.data_as(Ct.c_void_p), Ct.c_void_p(drp.data_ptr()),
                                    Ct.c_void_p(dci.data_ptr()), Ct.c_void_p(dv.data_ptr()), g, 4, Ct.byref(o),
                                    None, Ct.byref(h))
        if rc == 0:
            lib.bamg_free(h)
        return rc

    assert setup(ci, grids, off) == 0
    assert setup(ci_bad, grids, off) == B.EINVAL
    bad_grids = grids.copy()
    bad_grids[1, 0] += 1
    assert setup(ci, bad_grids, off) == B.EINVAL
    # two chains whose coarsest grid side exceeds 64
    big = [C.tandem_queue(127), C.tandem_queue(8)]
    with pytest.raises(B.BamgError) as e:
        B.BatchedHierarchy(big, 4, B.default_options(levels=1))
    assert e.value.code == B.EUNSUPPORTED


def test_cycle_graph_replays_match_eager_and_oracle():
    # the cycle is captured once and replayed; replays separated by other
    # work on the stream (a full solve) must give the same vector each time
    ch = C.tandem_queue(40)
    levels = 3
    h = B.Hierarchy.from_chain(ch, 12, B.default_options(levels=levels, cycle_mode=2))
    lvls = []
    plan = O.level_plan(_grid(ch), levels)
    for l in range(levels):
        lv = O.Level(plan[l], _csr(h, l, "B"), None)
        if l < levels - 1:
            Pg, _ = _p_from_ell(h, l, plan[l + 1].n)
            lv.P, lv.Q = Pg, O.averaging_q(Pg)
        lvls.append(lv)
    ho = O.Hierarchy(lvls, O.Options(levels=levels), O.coarsest_pinv(lvls[-1].B.toarray()), None, [], None)
    f0 = np.random.default_rng(5).random(ch.n)
    f0 -= f0.mean()
    want = O.vcycle(ho, f0)
    f = torch.tensor(f0, device="cuda")
    outs = []
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    for rep in range(3):
        e = torch.empty_like(f)
        h.apply_vcycle(f, e)
        outs.append(e.cpu().numpy())
        h.solve(x, 1e-10, 100)           # eager work and more replays in between
        torch.cuda.synchronize()
    for rep in range(3):
        assert np.array_equal(outs[rep], outs[0]), rep
        assert np.abs(outs[rep] - want).max() <= 1e-9 * np.abs(want).max(), rep
    assert h.stats().cycle_graph == 1
    # eager launches of the same cycle give the same vector
    he = B.Hierarchy.from_chain(ch, 12, B.default_options(levels=levels, cycle_mode=1))
    e = torch.empty_like(f)
    he.apply_vcycle(f, e)
    assert np.array_equal(e.cpu().numpy(), outs[0])
    assert he.stats().cycle_graph == 0


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_cycle_modes_give_the_same_solve(mode):
    chains = _mix()
    h = B.BatchedHierarchy(chains, R, B.default_options(levels=0, coarse_max=COARSE_MAX, cycle_mode=mode))
    x = torch.empty(h.n, dtype=torch.float64, device="cuda")
    info, status, _ = h.solve_batched(x, tol=1e-12, max_cycles=300)
    assert info.converged
    h1 = B.BatchedHierarchy(chains, R, B.default_options(levels=0, coarse_max=COARSE_MAX, cycle_mode=1))
    x1 = torch.empty(h.n, dtype=torch.float64, device="cuda")
    info1, _, _ = h1.solve_batched(x1, tol=1e-12, max_cycles=300)
    assert info.cycles == info1.cycles
    assert torch.equal(x, x1)
    st = h.stats()
    if mode == 0:
        assert st.cycle_gpu_us > 0 and st.cycle_host_us > 0


@pytest.mark.parametrize("precision", [B.FP64, B.MIXED])
def test_no_read_of_unwritten_memory(precision, monkeypatch):
    # with BAMG_POISON=1 every floating-point allocation starts as NaN: a
    # kernel that reads memory nothing wrote would change (or NaN) the result
    chains = _mix()
    opts = B.default_options(levels=0, coarse_max=COARSE_MAX, precision=precision)
    outs = []
    for poison in ("0", "1"):
        monkeypatch.setenv("BAMG_POISON", poison)
        h = B.BatchedHierarchy(chains, R, opts)
        x = torch.empty(h.n, dtype=torch.float64, device="cuda")
        info, status, _ = h.solve_batched(x, tol=1e-13, max_cycles=300)
        e = torch.empty_like(x)
        h.apply_vcycle(x, e)
        outs.append((x.cpu().numpy(), e.cpu().numpy(), info.cycles))
        h.close()
    assert outs[0][2] == outs[1][2]
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_batched_vcycle_is_per_chain_vcycle():
    # one cycle of the batched handle acts on each chain's block exactly as
    # the single-chain cycle (caller's chain order in and out)
    chains = _mix()
    opts = B.default_options(levels=0, coarse_max=COARSE_MAX)
    h = B.BatchedHierarchy(chains, R, opts)
    rng = np.random.default_rng(11)
    f0 = np.concatenate([rng.random(ch.n) - 0.5 for ch in chains])
    e = torch.empty(h.n, dtype=torch.float64, device="cuda")
    h.apply_vcycle(torch.tensor(f0, device="cuda"), e)
    eb = _blocks(e.cpu().numpy(), h.offsets)
    fb = _blocks(f0, h.offsets)
    for c, ch in enumerate(chains):
        h1 = B.Hierarchy.from_chain(ch, R, opts)
        e1 = torch.empty(ch.n, dtype=torch.float64, device="cuda")
        h1.apply_vcycle(torch.tensor(fb[c], device="cuda"), e1)
        want = e1.cpu().numpy()
        assert np.abs(eb[c] - want).max() <= 1e-14 * np.abs(want).max(), c
        h1.close()


def test_trim_returns_cached_memory_and_handles_still_work():
    ch = C.tandem_queue(32)
    h = B.Hierarchy.from_chain(ch, R, B.default_options(levels=3))
    h2 = B.Hierarchy.from_chain(ch, R, B.default_options(levels=3))
    h2.close()
    B.trim()                             # h2's buffers go back to HIP, h keeps its own
    x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    info = h.solve(x, 1e-12, 100)
    assert info.converged
    h3 = B.Hierarchy.from_chain(ch, R, B.default_options(levels=3))
    x3 = torch.empty(ch.n, dtype=torch.float64, device="cuda")
    h3.solve(x3, 1e-12, 100)
    assert torch.equal(x, x3)


@pytest.mark.parametrize("variant", ["1,128", "2,256", "3,128", "4,512", "6,256", "12,128", "2,256,2", "4,512,2"])
def test_sweep_variants_give_the_same_bits(variant, monkeypatch):
    # every launch shape the autotuner may pick computes the same numbers;
    # with two row pieces per thread the 1681 x 3 pieces leave the last
    # thread's second piece past the end
    ch = C.tandem_queue(40)
    opts = B.default_options(levels=3, stop_after=1)
    monkeypatch.setenv("BAMG_SWEEP_VARIANT", "1,256")
    ref = B.Hierarchy.from_chain(ch, 12, opts).export(0, B.X_U)
    monkeypatch.setenv("BAMG_SWEEP_VARIANT", variant)
    h = B.Hierarchy.from_chain(ch, 12, opts)
    assert np.array_equal(h.export(0, B.X_U), ref)
    vw, bs, *rp = map(int, variant.split(","))
    st = h.stats()
    assert st.sweep_ell == 1
    assert (st.sweep_vw, st.sweep_bs, st.sweep_rp) == (vw, bs, rp[0] if rp else 1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_ell_copies_give_the_same_bits(precision, monkeypatch):
    # the ELL-4 copy of B_0 (written by the pass that builds B_0 from A, with
    # its FP64 values for the outer products in the mixed form) and the ELL-9
    # copies of the coarse grid levels add the same terms in the same order
    # as the CSR forms: the test vectors, the operators and the solution agree
    # bit for bit with BAMG_SWEEP_ELL=0
    ch = C.tandem_queue(40)
    opts = B.default_options(levels=3, precision=B.MIXED if precision == "mixed" else B.FP64)
    out = {}
    for ell in ("0", "1"):
        monkeypatch.setenv("BAMG_SWEEP_ELL", ell)
        h = B.Hierarchy.from_chain(ch, 12, opts)
        x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
        info = h.solve(x, 1e-12, 100)
        assert info.converged
        out[ell] = (h.stats().sweep_ell, x.cpu().numpy(), h.export(0, B.X_U),
                    [h.export(l, it) for l in (0, 1, 2) for it in (B.X_B_COL, B.X_B_VAL)])
        h.close()
    assert (out["0"][0], out["1"][0]) == (0, 1)
    for a, b in zip(out["0"][1:3], out["1"][1:3]):
        assert np.array_equal(a, b)
    for a, b in zip(out["0"][3], out["1"][3]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("rows", ["14", "56"])
def test_galerkin_rows_per_workgroup_give_the_same_bits(rows, monkeypatch):
    # the fused Galerkin launch shapes the autotuner chooses from (14, 28 or
    # 56 coarse rows per workgroup) compute the same operators, level 0
    # (T_0 = I, ELL-4 B_0) and the coarser levels (ELL-9 B_l and T_l)
    ch = C.tandem_queue(40)
    opts = B.default_options(levels=4, stop_after=1)
    items = (B.X_B_COL, B.X_B_VAL, B.X_T_COL, B.X_T_VAL)
    monkeypatch.setenv("BAMG_GAL_ROWS", "28")
    h = B.Hierarchy.from_chain(ch, 12, opts)
    ref = [[h.export(l, it) for it in items] for l in (1, 2, 3)]
    h.close()
    monkeypatch.setenv("BAMG_GAL_ROWS", rows)
    h = B.Hierarchy.from_chain(ch, 12, opts)
    for l, want in zip((1, 2, 3), ref):
        for it, w in zip(items, want):
            assert np.array_equal(h.export(l, it), w), (l, it)
    h.close()


def test_tune_cache_file_is_written_and_reused(tmp_path):
    # a chain large enough that both tuners run (level-0 sweep: n R >= 2^20;
    # Galerkin: level 1 with >= 2^16 coarse rows); a second process reads the
    # choices from the cache file and times nothing
    import json
    import subprocess
    import sys
    cache = tmp_path / "tune.json"
    code = (
        "import sys, json; sys.path.insert(0, %r)\n"
        "import torch\n"
        "from paper_1004_1451_amd import bamg as B, chains as C\n"
        "ch = C.tandem_queue(512)\n"
        "h = B.Hierarchy.from_chain(ch, 12, B.default_options(levels=4, stop_after=1))\n"
        "st = h.stats()\n"
        "print(json.dumps({'tune_ms': st.tune_ms, 'vw': st.sweep_vw, 'bs': st.sweep_bs, 'rp': st.sweep_rp}))\n"
    ) % str(__import__("pathlib").Path(__file__).resolve().parents[1])
    env = dict(__import__("os").environ, BAMG_TUNE_CACHE=str(cache))
    env.pop("BAMG_SWEEP_VARIANT", None)
    env.pop("BAMG_GAL_ROWS", None)
    runs = []
    for _ in range(2):
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        assert out.returncode == 0, out.stderr[-2000:]
        runs.append(json.loads(out.stdout.strip().splitlines()[-1]))
    entries = json.loads(cache.read_text())
    kinds = {k.split("|")[1] for k in entries}
    assert {"sweep", "galerkin"} <= kinds, entries
    assert runs[0]["tune_ms"] > 0 and runs[1]["tune_ms"] == 0
    assert (runs[0]["vw"], runs[0]["bs"], runs[0]["rp"]) == (runs[1]["vw"], runs[1]["bs"], runs[1]["rp"])
