"""Benchmark: setup + solve seconds to ||Bx||_1/||x||_1 <= 1e-10 on the
n = 4,194,304 tandem queue (N = 2047, r = 12 test vectors, 6 levels), one
MI355X.  Prints one JSON line.

A step is one whole pass of the method over the resident input: bamg_setup
(relaxation, LS interpolation, Galerkin products, coarsest eigensolve,
up-leg, recomputation) + bamg_solve (V-cycle-preconditioned FGMRES to the
tolerance) + bamg_free.  The roofline object reports the level-0 test-vector
sweep: algorithmic bytes per launch / mean launch time (HIP events recorded
by the library on its own stream during the timed steps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def _traffic_from_profiles(name: str):
    """HBM bytes per launch measured by rocprofv3 counters, if a summary for
    this kernel and workload is committed (profiles/<name>_traffic.txt with
    lines 'bytes_per_launch: <value>' and 'source_hash: <sha>'), else None.
    None too when the kernel source changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.txt")
    if not os.path.exists(path):
        return None
    import hashlib
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_1004_1451_amd", "csrc", "k_sweep.h")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if vals.get("source_hash") != h:
        return None          # kernel changed since the counters were taken
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _host_cpu():
    """Cores this process may run on, and the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return avail, os.cpu_count() or avail, model


def _oracle_run(ch, args, threads):
    from threadpoolctl import threadpool_limits
    from oracle import bamg_oracle as O
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        x, info, h = O.stationary(ch.to_scipy(), O.Grid(ch.nx, ch.ny, ch.periodic), args.r,
                                  O.Options(levels=args.levels), tol=args.tol, max_cycles=200)
        return time.perf_counter() - t0, x, info, h


def cpu_baseline(args):
    """The oracle, untuned, on a bounded sample of the workload: the whole
    method (same kind of chain, r, levels, tolerance) on a chain of half the
    side (a quarter of the states: tandem N = 1023, or the 512^2 lattice),
    once with its BLAS/LAPACK on one thread and once on every core this
    process may use; the one-thread time is scaled to the benchmarked chain
    by the ratio of state counts (the work per level is linear in n; the
    coarsest SVD grows faster, so the scaled figure understates the
    oracle)."""
    from paper_1004_1451_amd import chains as C
    if args.workload == "lattice":
        ch, full, name = C.weighted_lattice(args.M // 2, seed=1), args.M * args.M, f"periodic lattice {args.M // 2}^2"
    else:
        ch, full, name = C.tandem_queue((args.N + 1) // 2 - 1), (args.N + 1) ** 2, f"tandem N={(args.N + 1) // 2 - 1}"
    avail, total, model = _host_cpu()
    dt1, _, info1, _ = _oracle_run(ch, args, 1)
    dtn, _, _, _ = _oracle_run(ch, args, avail)
    scale = full / ch.n
    return {"value": round(dt1 * scale, 3), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup+solve on {name} (n={ch.n:,}, {args.levels} levels, r={args.r}, "
                      f"tol={args.tol:g}, {info1.cycles} cycles): {dt1:.2f} s on 1 thread, scaled by the n ratio "
                      f"{scale:.0f}; {dtn:.2f} s with {avail} threads",
            "all_cores": {"threads": avail, "seconds_sample": round(dtn, 3),
                          "value_scaled": round(dtn * scale, 3)},
            "host": {"nproc": total, "available": avail, "cpu_model": model},
            "converged": bool(info1.converged)}


def oracle_full(args, x_by_form, stats_by_form, h_by_form):
    """The oracle on the benchmarked chain itself (N = 2047, one thread), and
    how far each GPU form is from it: ||x - x_oracle||_1, per level
    ||B_l - B_l^oracle||_F / ||B_l^oracle||_F and the rows whose P pattern
    differs.  Minutes of CPU time: only with --oracle-full."""
    from oracle import bamg_oracle as O
    from paper_1004_1451_amd import chains as C
    ch = C.tandem_queue(args.N)
    avail, total, model = _host_cpu()
    t0 = time.perf_counter()
    O.PROGRESS = lambda msg: print(f"oracle: {msg} ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    try:
        dt, xo, info, ho = _oracle_run(ch, args, 1)
    finally:
        O.PROGRESS = None
    out = {"oracle_seconds_1_thread": round(dt, 2), "oracle_cycles": info.cycles,
           "oracle_residual_l1": info.residual_l1, "host": {"nproc": total, "cpu_model": model}, "forms": {}}
    for form, x in x_by_form.items():
        h = h_by_form[form]
        levels = []
        for l, lv in enumerate(ho.levels):
            Bg = h["B"][l]
            Bo = lv.B.tocsr()
            rel = float(np.sqrt(((Bg - Bo).multiply(Bg - Bo)).sum() / (Bo.multiply(Bo)).sum()))
            ent = {"n": int(Bo.shape[0]), "B_rel_fro": rel}
            if l < len(ho.levels) - 1:
                Pg, Po = h["P"][l].tocsr(), lv.P.tocsr()
                Pg.sort_indices(); Po.sort_indices()
                same = np.array_equal(Pg.indptr, Po.indptr) and np.array_equal(Pg.indices, Po.indices)
                if same:
                    bad = 0
                else:
                    rows_g = np.split(Pg.indices, Pg.indptr[1:-1])
                    rows_o = np.split(Po.indices, Po.indptr[1:-1])
                    bad = int(sum(not np.array_equal(a, b) for a, b in zip(rows_g, rows_o)))
                ent["P_pattern_rows_differing"] = bad
            levels.append(ent)
        out["forms"][form] = {"l1_vs_oracle": float(np.abs(x - xo).sum()), "gpu_cycles": stats_by_form[form],
                              "levels": levels}
    return out


def cpu_baseline_batch(chains, args, budget_s=15.0):
    """The oracle on a bounded sample of the batch: chains in the batch's own
    order until about budget_s seconds of single-thread work, scaled to the
    whole batch by the ratio of state counts."""
    from threadpoolctl import threadpool_limits
    from oracle import bamg_oracle as O
    done_n, dt, k, conv = 0, 0.0, 0, True
    with threadpool_limits(limits=1):
        for ch in chains:
            if dt > budget_s:
                break
            t0 = time.perf_counter()
            _, info, _ = O.stationary(ch.to_scipy(), O.Grid(ch.nx, ch.ny, ch.periodic), args.r,
                                      O.Options(levels=0, coarse_max=1024), tol=args.tol, max_cycles=200)
            dt += time.perf_counter() - t0
            done_n += ch.n
            k += 1
            conv &= bool(info.converged)
    total = sum(ch.n for ch in chains)
    scale = total / done_n
    return {"value": dt * scale, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup+solve on the first {k} of {len(chains)} chains ({done_n:,} of {total:,} states) "
                      f"took {dt:.2f} s on 1 thread; scaled by n ratio {scale:.1f}",
            "converged": conv}


def cpu_baseline_upg(ch, args, budget_s=20.0):
    """The oracle, untuned, on the same unstructured planar graph (whole
    method, one thread), repeated while under budget_s; graphs above 16384
    points are sampled by the graph of 16384 points scaled by the ratio of
    point counts."""
    from threadpoolctl import threadpool_limits
    from oracle import bamg_oracle as O
    from paper_1004_1451_amd import chains as C
    sample = ch if ch.n <= 16384 else C.upg(16384, seed=0)
    reps, dt = 0, 0.0
    with threadpool_limits(limits=1):
        while reps == 0 or (dt < budget_s / 4 and reps < 5):
            t0 = time.perf_counter()
            _, info, _ = O.stationary(sample.to_scipy(), None, args.r, O.Options(levels=args.levels), tol=args.tol,
                                      max_cycles=200)
            dt += time.perf_counter() - t0
            reps += 1
    per = dt / reps
    scale = ch.n / sample.n
    return {"value": per * scale, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup+solve on the Delaunay graph of {sample.n} points ({args.levels} levels, r={args.r}, "
                      f"tol={args.tol:g}, {info.cycles} cycles), mean of {reps} run(s) on 1 thread: {per:.3f} s"
                      + (f"; scaled by point ratio {scale:.1f} (linear: the oracle's dense coarsest SVD grows "
                         f"faster, so this understates the oracle)" if scale != 1 else ""),
            "converged": bool(info.converged)}


PEAK_FP64_TFLOPS = 78.6


def _roofline_dense(stats):
    """Rank-64 updates of the dense coarsest Gauss-Jordan inverse: flops / HIP
    event time of those launches (FP64 vector FMAs) against the FP64 peak."""
    ms = sum(s.dense_update_ms for s in stats)
    n = sum(s.dense_update_launches for s in stats)
    flops = sum(s.dense_update_flops for s in stats)
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
            "kernel": "k_gj_update (rank-64 update of the dense coarsest inverse, FP64)",
            "flops_per_launch": round(flops / max(1, n)), "mean_launch_us": round(ms * 1e3 / max(1, n), 2)}


def _roofline(stats, traffic):
    sweep_ms = sum(s.sweep_ms for s in stats) / max(1, sum(s.sweep_launches for s in stats))
    sweep_bytes = stats[-1].sweep_bytes
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    st = stats[-1]
    return sweep_ms, {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                      "kernel": "%s<VW=%d,BS=%d%s> (level-0 test-vector sweep%s)" % (
                          "k_sweep_ve" if st.sweep_ell else "k_sweep_v", st.sweep_vw, st.sweep_bs,
                          ",RP=%d" % st.sweep_rp if st.sweep_ell else "",
                          ", ELL-4 copy of B_0" if st.sweep_ell else ""),
                      "bytes_per_launch": int(sweep_bytes), "mean_launch_us": round(sweep_ms * 1e3, 2)}


def _per_launch(stats, ms_field, n_field, bytes_field):
    """Mean HIP-event time of one launch kind (us) and its algorithmic GB/s
    (the bytes of that same launch over its own time)."""
    ms = sum(getattr(s, ms_field) for s in stats)
    n = sum(getattr(s, n_field) for s in stats)
    if n == 0 or ms <= 0:
        return None
    us = ms * 1e3 / n
    b = getattr(stats[-1], bytes_field)
    return {"us": round(us, 2), "bytes": int(b), "GBps": round(b / (us * 1e-6) / 1e9, 1),
            "frac_of_peak": round(b / (us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4), "launches": n}


def _kernel_detail(stats):
    return {
        "setup_ms": round(float(np.mean([s.t_setup_ms for s in stats])), 3),
        "solve_ms": round(float(np.mean([s.t_solve_ms for s in stats])), 3),
        "op_complexity": round(stats[-1].op_complexity, 4),
        # level 0, one entry per launch kind: both Galerkin products
        # (B_1, T_1) in one launch, their copy into CSR, LS fit of each pass
        "galerkin_BT": _per_launch(stats, "galerkin_ms", "galerkin_launches", "galerkin_bytes"),
        "galerkin_csr": _per_launch(stats, "gal_csr_ms", "gal_csr_launches", "gal_csr_bytes"),
        "lsfit_first_pass": _per_launch(stats, "lsfit_ms", "lsfit_launches", "lsfit_bytes"),
        "lsfit_recompute_pass": _per_launch(stats, "lsfit2_ms", "lsfit2_launches", "lsfit2_bytes"),
        "coarsest_min_pivot": stats[-1].coarsest_min_pivot,
        "coarsest_arnoldi_steps": stats[-1].arnoldi_steps,
        "cycle_graph": stats[-1].cycle_graph,
        "sweep_tune_ms_total": round(stats[-1].tune_ms, 2),
    }


def _timed(step, args):
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res.append(step())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / args.steps, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["tandem", "lattice", "batch64", "learned", "upg"], default="tandem",
                    help="tandem: one tandem queue (default N=2047, n=4.2M); batch64: 64 mixed chains in one handle; "
                         "learned: train the interpolation network on 32 jittered tandems (untimed), then time the "
                         "learned form on the tandem queue against the plain forms")
    ap.add_argument("--train-chains", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--N", type=int, default=2047, help="tandem queue capacity (side N+1)")
    ap.add_argument("--M", type=int, default=1024, help="lattice workload: side of the periodic lattice")
    ap.add_argument("--levels", type=int, default=None, help="6 (tandem, learned), 3 (upg)")
    ap.add_argument("--r", type=int, default=None, help="test vectors: 12, or 6 for upg (Table 4)")
    ap.add_argument("--tol", type=float, default=None, help="1e-10, or 1e-8 for upg (Table 4)")
    ap.add_argument("--upg-n", type=int, default=65536,
                    help="upg workload: points of the Delaunay triangulation (Table 4 goes to 2048; 65536 fills "
                         "the GPU better)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed",
                    help="mixed (default): FP32 relaxation, Galerkin products and cycle, FP64 coarsest level, norms "
                         "and outer iteration; fp64: every step in FP64")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip the untimed FP64 run that the mixed result is compared with")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-full", action="store_true",
                    help="tandem workload: also run the oracle on the benchmarked chain itself (minutes of CPU time) "
                         "and report each GPU form's distance from it")
    ap.add_argument("--solver", choices=["fgmres", "parnoldi", "mle"], default="fgmres",
                    help="tandem workload: FGMRES (Section 4.2), preconditioned Arnoldi (Section 4.3) or the "
                         "stand-alone MLE iteration (Section 4.1)")
    ap.add_argument("--mu", type=int, choices=[1, 2], default=1, help="setup cycle index (1 = V, 2 = W)")
    ap.add_argument("--caliber", type=int, default=4,
                    help="most coarse points an F point interpolates from (Algorithm 2; the paper's tables use 2)")
    ap.add_argument("--relax", choices=["jacobi", "mcgs"], default="jacobi",
                    help="tandem workload: omega-Jacobi (the paper's) or multicolour Gauss-Seidel sweeps")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three plain device copies of MIB MiB (the reference kernel whose FETCH_SIZE / "
                         "WRITE_SIZE counters scale the traffic figures) and exit")
    args = ap.parse_args()
    upg = args.workload == "upg"
    if args.levels is None:
        args.levels = 3 if upg else (5 if args.workload == "lattice" else 6)
    if args.r is None:
        args.r = 6 if upg else 12
    if args.tol is None:
        args.tol = 1e-8 if upg else 1e-10
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is described "
              f"in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 8, "copies": 3}))
        return
    from paper_1004_1451_amd import bamg as B
    from paper_1004_1451_amd import chains as C

    prec = B.FP64 if args.precision == "fp64" else B.MIXED
    def traffic_of(stats):
        # counters of the sweep form that ran (ELL-4 copy or CSR)
        form = "k_sweep_ve" if stats[-1].sweep_ell else "k_sweep_v"
        return _traffic_from_profiles(f"{form}_{args.workload}_{args.precision}")
    if args.workload in ("tandem", "lattice"):
        lattice = args.workload == "lattice"
        # the weighted periodic lattice with seed 1 (its stationary vector is
        # the weighted degree, known in closed form) or the tandem queue
        ch = C.weighted_lattice(args.M, seed=1) if lattice else C.tandem_queue(args.N)
        rp, ci, v = B.device_csr(ch)
        x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
        relax = B.RELAX_MCGS if args.relax == "mcgs" else B.RELAX_JACOBI
        opts = B.default_options(levels=args.levels, precision=prec, profile=1, relax=relax, mu=args.mu,
                                 caliber=args.caliber)

        def step():
            h = B.Hierarchy(ch.n, rp, ci, v, (ch.nx, ch.ny, int(ch.periodic)), args.r, opts)
            if args.solver == "mle":
                info = h.mle_iterate(x, args.tol, 200)
            else:
                info = h.solve(x, args.tol, 200, parnoldi=args.solver == "parnoldi")
            st = h.stats()
            h.close()
            return info, st

        sec, res = _timed(step, args)
        infos = [a for a, _ in res]
        stats = [b for _, b in res]
        sweep_ms, roof = _roofline(stats, traffic_of(stats) if args.relax == "jacobi" else None)
        roof["kernel"] += ", R=%d" % args.r
        if args.relax == "mcgs":
            roof["kernel"] = "k_mcgs_tv<VW=%d> x colours (level-0 test-vector Gauss-Seidel sweep), R=%d" % (
                stats[-1].sweep_vw, args.r)
        detail = _kernel_detail(stats)
        detail.update({"cycles": [i.cycles for i in infos],
                       "history": [float("%.3e" % v) for v in list(infos[-1].history)[: infos[-1].history_len]],
                       "residual_l1": max(i.residual_l1 for i in infos),
                       "converged": all(i.converged for i in infos)})
        if ch.exact is not None:
            detail["l1_error_vs_closed_form"] = float(np.abs(x.cpu().numpy() - ch.exact).sum())
        if prec == B.MIXED and not args.no_fp64_compare:
            # outside the timed region: the plain FP64 form, its time per step
            # and how far the mixed solution is from it
            x_mixed = x.clone()
            opts = B.default_options(levels=args.levels, precision=B.FP64, profile=1, relax=relax, mu=args.mu,
                                     caliber=args.caliber)
            sec64, res64 = _timed(step, argparse.Namespace(warmup=1, steps=max(1, min(args.steps, 3))))
            detail["fp64_ms_per_step"] = round(sec64 * 1e3, 3)
            detail["fp64_cycles"] = res64[-1][0].cycles
            detail["l1_diff_vs_fp64_path"] = float((x - x_mixed).abs().sum().item())
            if ch.exact is not None:
                detail["fp64_l1_error_vs_closed_form"] = float(np.abs(x.cpu().numpy() - ch.exact).sum())
        out = {
            "metric": ("setup+solve seconds to ||Bx||_1/||x||_1<=1e-10 on the 1024^2 weighted lattice" if lattice
                       else "setup+solve seconds to ||Bx||_1/||x||_1<=1e-10 at n=4.2M; sweep HBM GB/s"),
            "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prec == B.FP64 else "f32+f64", "data": "synthetic",
            "config": {"workload": (f"weighted periodic lattice {args.M}x{args.M} (n={ch.n:,}), w~U[0.1,1], "
                                    f"r={args.r}, {args.levels} levels, tol {args.tol:g}") if lattice else
                                   (f"tandem queue N={args.N} (n={ch.n:,}), rates 11/31,10/31,10/31, r={args.r}, "
                                    f"{args.levels} levels, tol {args.tol:g}"), "precision": args.precision,
                       **({"relax": "multicolour Gauss-Seidel"} if args.relax == "mcgs" else {}),
                       **({"solver": {"parnoldi": "preconditioned Arnoldi", "mle": "MLE iteration"}[args.solver]}
                          if args.solver != "fgmres" else {}),
                       **({"setup_cycle": "W"} if args.mu == 2 else {}),
                       **({"caliber": args.caliber} if args.caliber != 4 else {})},
            "roofline": roof, "detail": detail,
        }
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args)
        if args.oracle_full and not lattice:
            import scipy.sparse as sps
            xs, cyc, hs = {}, {}, {}
            for form, pr in (("mixed", B.MIXED), ("fp64", B.FP64)):
                hh = B.Hierarchy(ch.n, rp, ci, v, (ch.nx, ch.ny, int(ch.periodic)), args.r,
                                 B.default_options(levels=args.levels, precision=pr))
                info = hh.solve(x, args.tol, 200)
                xs[form], cyc[form] = x.cpu().numpy().copy(), info.cycles
                Bs, Ps = [], []
                for l in range(args.levels):
                    li = hh.level_info(l)
                    Bs.append(sps.csr_matrix((hh.export(l, B.X_B_VAL), hh.export(l, B.X_B_COL),
                                              hh.export(l, B.X_B_ROWPTR)), shape=(li.n, li.n)))
                    if l + 1 < args.levels:
                        nc = hh.level_info(l + 1).n
                        pc = hh.export(l, B.X_P_COL).reshape(-1, 4)
                        pv = hh.export(l, B.X_P_VAL).reshape(-1, 4)
                        ok = pc >= 0
                        rows = np.repeat(np.arange(li.n), 4).reshape(-1, 4)[ok]
                        Ps.append(sps.csr_matrix((pv[ok], (rows, pc[ok])), shape=(li.n, nc)))
                hs[form] = {"B": Bs, "P": Ps}
                hh.close()
            out["oracle_full"] = oracle_full(args, xs, cyc, hs)
    elif upg:
        ch = C.upg(args.upg_n, seed=0)
        rp, ci, v = B.device_csr(ch)
        x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
        opts = B.default_options(levels=args.levels, precision=prec, profile=1)
        sizes = []

        def step():
            h = B.Hierarchy(ch.n, rp, ci, v, (0, 0, 0), args.r, opts)
            info = h.solve(x, args.tol, 200)
            st = h.stats()
            if not sizes:
                sizes.extend((h.level_info(l).n, h.level_info(l).cr_rounds) for l in range(st.n_levels))
            h.close()
            return info, st

        sec, res = _timed(step, args)
        infos = [a for a, _ in res]
        stats = [b for _, b in res]
        sweep_ms, roof = _roofline(stats, None)
        roof["kernel"] += ", R=%d" % args.r
        gj_ms = sum(s.dense_update_ms for s in stats)
        sweep_tot = sum(s.sweep_ms for s in stats)
        if gj_ms > sweep_tot:
            # the dense coarsest inverse dominates: report its rank-64 updates
            roof = _roofline_dense(stats)
        detail = _kernel_detail(stats)
        detail.update({"cycles": [i.cycles for i in infos], "residual_l1": max(i.residual_l1 for i in infos),
                       "converged": all(i.converged for i in infos),
                       "l1_error_vs_closed_form": float(np.abs(x.cpu().numpy() - ch.exact).sum()),
                       "level_sizes": [a for a, _ in sizes], "cr_rounds": [b for _, b in sizes]})
        out = {
            "metric": "setup+solve seconds to ||Bx||_1/||x||_1<=tol on an unstructured planar graph",
            "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prec == B.FP64 else "f32+f64", "data": "synthetic",
            "config": {"workload": f"unstructured planar graph: Delaunay of N={args.upg_n} random points "
                                   f"(nnz={ch.nnz:,}), compatible-relaxation coarsening, r={args.r}, "
                                   f"{args.levels} levels, tol {args.tol:g}", "precision": args.precision},
            "roofline": roof, "detail": detail,
        }
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_upg(ch, args)
    elif args.workload == "learned":
        from paper_1004_1451_amd import learned as LRN
        t0 = time.perf_counter()
        # the library builds the training chains, collects the pairs and trains
        params, tinfo = LRN.train(n_chains=args.train_chains, n_val=4, r=args.r, levels=args.levels,
                                  epochs=args.epochs)
        train_s = time.perf_counter() - t0
        ch = C.tandem_queue(args.N)
        rp, ci, v = B.device_csr(ch)
        x = torch.empty(ch.n, dtype=torch.float64, device="cuda")
        forms = {
            "plain_fp64": dict(precision=B.FP64),
            "mixed_ls": dict(precision=B.MIXED),
            "mixed_ls_1pass": dict(precision=B.MIXED, setup_passes=1),
            "mixed_learned_1pass": dict(precision=B.MIXED, interp=B.INTERP_MLP, mlp_weights=params.data_ptr(),
                                        setup_passes=1),
            "mixed_learned": dict(precision=B.MIXED, interp=B.INTERP_MLP, mlp_weights=params.data_ptr()),
        }
        res = {}
        for name, kw in forms.items():
            opts = B.default_options(levels=args.levels, profile=1, **kw)

            def step():
                h = B.Hierarchy(ch.n, rp, ci, v, (ch.nx, ch.ny, 0), args.r, opts)
                info = h.solve(x, args.tol, 300)
                st = h.stats()
                h.close()
                return info, st

            sec_f, rr = _timed(step, args)
            info, st = rr[-1]
            res[name] = {"ms_per_step": round(sec_f * 1e3, 3), "cycles": info.cycles,
                         "residual_l1": info.residual_l1, "converged": bool(info.converged),
                         "setup_ms": round(st.t_setup_ms, 3), "solve_ms": round(st.t_solve_ms, 3)}
            if kw.get("interp") == B.INTERP_MLP:
                res[name]["fallback_fraction"] = round(st.mlp_fallback / max(1, st.mlp_points), 4)
            if name == "mixed_learned_1pass":
                sec, stats = sec_f, [b for _, b in rr]
        sweep_ms, roof = _roofline(stats, traffic_of(stats) if args.precision == "mixed" else None)
        roof["kernel"] += ", R=%d" % args.r
        out = {
            "metric": "setup+solve seconds to ||Bx||_1/||x||_1<=1e-10 at n=4.2M, learned + mixed form",
            "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64+bf16", "data": "synthetic",
            "config": {"workload": f"tandem queue N={args.N} (n={ch.n:,}), r={args.r}, {args.levels} levels, "
                                   f"tol {args.tol:g}; network trained on {args.train_chains} jittered tandems "
                                   f"N in [255,1023]", "precision": "mixed+learned"},
            "roofline": roof,
            "detail": {"forms": res, "train_s": round(train_s, 2),
                       "train_steps": tinfo.steps, "train_ms": round(tinfo.ms, 1),
                       "val_loss_first": tinfo.val_loss_first, "val_loss_last": tinfo.val_loss_last,
                       "learned_vs_plain_fp64": round(res["plain_fp64"]["ms_per_step"] /
                                                      res["mixed_learned_1pass"]["ms_per_step"], 3),
                       "learned_vs_mixed_ls_1pass": round(res["mixed_ls_1pass"]["ms_per_step"] /
                                                          res["mixed_learned_1pass"]["ms_per_step"], 3)},
        }
    else:
        chains = C.batch_mix(64)
        db = B.DeviceBatch(chains)
        x = torch.empty(db.n, dtype=torch.float64, device="cuda")
        opts = B.default_options(levels=0, coarse_max=1024, precision=prec, profile=1)

        def step():
            h = B.BatchedHierarchy(db, args.r, opts)
            info, status, resid = h.solve_batched(x, args.tol, 200)
            st = h.stats()
            h.close()
            return info, status, resid, st

        sec, res = _timed(step, args)
        stats = [r[3] for r in res]
        sweep_ms, roof = _roofline(stats, traffic_of(stats))
        roof["kernel"] += ", R=%d, all 64 chains" % args.r
        detail = _kernel_detail(stats)
        detail.update({"chains_per_s": round(64 / sec, 2), "cycles": [r[0].cycles for r in res],
                       "worst_chain_residual": float(max(r[2].max() for r in res)),
                       "all_chains_converged": bool(all(r[1].all() for r in res)),
                       "levels_max": stats[-1].n_levels})
        out = {
            "metric": "batched setup+solve seconds, 64 chains, every chain to ||Bx||_1/||x||_1<=1e-10",
            "value": round(sec, 6), "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if prec == B.FP64 else "f32+f64", "data": "synthetic",
            "config": {"workload": f"64 chains (tandem N in [31,511] jittered, periodic lattices side in [32,512]), "
                                   f"n={db.n:,}, r={args.r}, coarsen to <=1024, tol {args.tol:g}",
                       "precision": args.precision},
            "roofline": roof, "detail": detail,
        }
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_batch(chains, args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
