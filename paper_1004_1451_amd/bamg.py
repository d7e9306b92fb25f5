"""Python binding of the C ABI in include/bamg.h (argument marshalling only).

Every numerical step runs in the HIP library ``libbamg.so`` built in this
directory; PyTorch only provides device memory and the stream.  Importing this
module does not need a GPU; calling a function that launches kernels does.
There is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbamg.so")

OK, EINVAL, ENOTSTOCH, EZERODIAG, EUNSUPPORTED, ENOMEM, EDEVICE, ENOCONV, ESINGULAR = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, MIXED = 0, 1
INTERP_LS, INTERP_MLP = 0, 1
RELAX_JACOBI, RELAX_MCGS = 0, 1
USE_GUESS = 1
PARNOLDI = 2

X_B_ROWPTR, X_B_COL, X_B_VAL, X_T_ROWPTR, X_T_COL, X_T_VAL = 1, 2, 3, 4, 5, 6
X_P_COL, X_P_VAL, X_U, X_V, X_LAMBDA, X_VKIND, X_X0, X_W, X_Y, X_U0 = 7, 8, 9, 10, 11, 12, 13, 14, 15, 16
X_FEATURES, X_SLOTW, X_SLOTW0, X_CMAP, X_CR_RHO = 17, 18, 19, 20, 21
MLP_NPARAM = 6020

ERROR_NAMES = {EINVAL: "EINVAL", ENOTSTOCH: "ENOTSTOCH", EZERODIAG: "EZERODIAG", EUNSUPPORTED: "EUNSUPPORTED",
               ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOCONV: "ENOCONV", ESINGULAR: "ESINGULAR"}

# every symbol include/bamg.h declares
EXPORTS = ["bamg_options_default", "bamg_setup", "bamg_solve", "bamg_free", "bamg_last_error", "bamg_get_stats",
           "bamg_level_info_get", "bamg_export", "bamg_apply_vcycle", "bamg_relax", "bamg_setup_batched",
           "bamg_solve_batched", "bamg_trim", "bamg_mlp_init", "bamg_mlp_forward", "bamg_mlp_loss_grad",
           "bamg_mlp_train", "bamg_mle_iterate", "bamg_mlp_forward_noalloc", "bamg_mlp_collect",
           "bamg_train_spec_default", "bamg_mlp_train_spec"]


class BamgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("levels", C.c_int32), ("coarse_max", C.c_int32), ("nu_setup", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("omega", C.c_double),
                ("caliber", C.c_int32), ("n_eig", C.c_int32), ("arnoldi_m", C.c_int32),
                ("gmres_m", C.c_int32), ("precision", C.c_int32), ("interp", C.c_int32),
                ("mlp_weights", C.c_void_p), ("seed", C.c_uint64), ("mem_budget", C.c_size_t),
                ("profile", C.c_int32), ("stop_after", C.c_int32), ("cycle_mode", C.c_int32),
                ("setup_passes", C.c_int32), ("collect", C.c_int32), ("mlp_judge", C.c_float),
                ("relax", C.c_int32), ("gs_omega", C.c_double), ("mu", C.c_int32),
                ("cr_theta", C.c_double), ("cr_nu", C.c_int32), ("cr_rounds", C.c_int32),
                ("nbr_dist", C.c_int32), ("mlp_weights_path", C.c_char_p)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("history_len", C.c_int32), ("residual_l1", C.c_double), ("clamped_mass", C.c_double),
                ("history", C.c_double * 256)]


class Stats(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_v", C.c_int32), ("op_complexity", C.c_double),
                ("coarsest_min_pivot", C.c_double), ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("sweep_ms", C.c_double), ("galerkin_ms", C.c_double), ("lsfit_ms", C.c_double),
                ("sweep_launches", C.c_int32), ("galerkin_launches", C.c_int32), ("lsfit_launches", C.c_int32),
                ("sweep_bytes", C.c_int64), ("galerkin_bytes", C.c_int64), ("lsfit_bytes", C.c_int64),
                ("cycle_graph", C.c_int32), ("cycle_host_us", C.c_double), ("cycle_gpu_us", C.c_double),
                ("sweep_vw", C.c_int32), ("sweep_bs", C.c_int32), ("tune_ms", C.c_double),
                ("mlp_points", C.c_int64), ("mlp_fallback", C.c_int64), ("dense_update_ms", C.c_double),
                ("dense_update_launches", C.c_int32), ("dense_update_flops", C.c_double),
                ("sweep_ell", C.c_int32), ("gal_csr_ms", C.c_double), ("lsfit2_ms", C.c_double),
                ("gal_csr_launches", C.c_int32), ("lsfit2_launches", C.c_int32), ("gal_csr_bytes", C.c_int64),
                ("lsfit2_bytes", C.c_int64), ("sweep_rp", C.c_int32), ("arnoldi_steps", C.c_int32)]


class MlpTrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class MlpTrainInfo(C.Structure):
    _fields_ = [("steps", C.c_int32), ("train_loss_first", C.c_double), ("train_loss_last", C.c_double),
                ("val_loss_first", C.c_double), ("val_loss_last", C.c_double), ("ms", C.c_double),
                ("val_len", C.c_int32), ("val_history", C.c_double * 64)]


class TrainSpec(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_val", C.c_int32), ("side_min", C.c_int32), ("side_max", C.c_int32),
                ("jitter", C.c_double), ("seed", C.c_uint64), ("r", C.c_int32), ("levels", C.c_int32),
                ("init_seed", C.c_uint64), ("train", MlpTrainOpts)]


class LevelInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nx", C.c_int32), ("ny", C.c_int32), ("periodic", C.c_int32),
                ("nnz_b", C.c_int64), ("nnz_t", C.c_int64), ("nnz_p", C.c_int64), ("r", C.c_int32),
                ("n_v", C.c_int32), ("cr_rounds", C.c_int32)]


_lib = None


def load():
    """Load libbamg.so (built by build_lib.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() or paper_1004_1451_amd/build_lib.py")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.bamg_options_default.argtypes = [C.POINTER(Options)]
    lib.bamg_options_default.restype = None
    lib.bamg_setup.argtypes = [i64, vp, vp, vp, Grid, i32, C.POINTER(Options), vp, C.POINTER(vp)]
    lib.bamg_setup.restype = C.c_int
    lib.bamg_solve.argtypes = [vp, vp, dbl, i32, C.c_uint32, C.POINTER(SolveInfo)]
    lib.bamg_solve.restype = C.c_int
    lib.bamg_mle_iterate.argtypes = [vp, vp, dbl, i32, C.POINTER(SolveInfo)]
    lib.bamg_mle_iterate.restype = C.c_int
    lib.bamg_free.argtypes = [vp]
    lib.bamg_free.restype = C.c_int
    lib.bamg_last_error.argtypes = []
    lib.bamg_last_error.restype = C.c_char_p
    lib.bamg_get_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.bamg_get_stats.restype = C.c_int
    lib.bamg_level_info_get.argtypes = [vp, i32, C.POINTER(LevelInfo)]
    lib.bamg_level_info_get.restype = C.c_int
    lib.bamg_export.argtypes = [vp, i32, i32, vp, C.c_size_t]
    lib.bamg_export.restype = C.c_int
    lib.bamg_apply_vcycle.argtypes = [vp, vp, vp]
    lib.bamg_apply_vcycle.restype = C.c_int
    lib.bamg_relax.argtypes = [i64, vp, vp, vp, vp, vp, i32, dbl, i32, vp]
    lib.bamg_relax.restype = C.c_int
    lib.bamg_setup_batched.argtypes = [i32, vp, vp, vp, vp, vp, i32, C.POINTER(Options), vp, C.POINTER(vp)]
    lib.bamg_setup_batched.restype = C.c_int
    lib.bamg_solve_batched.argtypes = [vp, vp, dbl, i32, C.c_uint32, vp, vp, C.POINTER(SolveInfo)]
    lib.bamg_solve_batched.restype = C.c_int
    lib.bamg_trim.argtypes = []
    lib.bamg_trim.restype = C.c_int
    lib.bamg_mlp_init.argtypes = [C.c_uint64, vp, vp]
    lib.bamg_mlp_init.restype = C.c_int
    lib.bamg_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    lib.bamg_mlp_forward.restype = C.c_int
    lib.bamg_mlp_forward_noalloc.argtypes = [vp, i64, vp, vp, vp]
    lib.bamg_mlp_forward_noalloc.restype = C.c_int
    lib.bamg_mlp_loss_grad.argtypes = [vp, vp, i64, vp, vp, C.POINTER(C.c_double), vp]
    lib.bamg_mlp_loss_grad.restype = C.c_int
    lib.bamg_mlp_train.argtypes = [vp, vp, i64, vp, vp, i64, vp, C.POINTER(MlpTrainOpts), C.POINTER(MlpTrainInfo), vp]
    lib.bamg_mlp_train.restype = C.c_int
    lib.bamg_mlp_collect.argtypes = [vp, vp, vp, i64, C.POINTER(C.c_int64)]
    lib.bamg_mlp_collect.restype = C.c_int
    lib.bamg_train_spec_default.argtypes = [C.POINTER(TrainSpec)]
    lib.bamg_train_spec_default.restype = None
    lib.bamg_mlp_train_spec.argtypes = [C.POINTER(TrainSpec), C.c_char_p, vp, C.POINTER(MlpTrainInfo), vp]
    lib.bamg_mlp_train_spec.restype = C.c_int
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise BamgError(rc, load().bamg_last_error().decode())
    return rc


def default_options(**kw) -> Options:
    o = Options()
    load().bamg_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def device_csr(chain, device="cuda"):
    """Upload a chain's CSR arrays (row_ptr, col_idx, val) to the device."""
    import torch
    rp = torch.as_tensor(np.ascontiguousarray(chain.row_ptr, dtype=np.int32), device=device)
    ci = torch.as_tensor(np.ascontiguousarray(chain.col_idx, dtype=np.int32), device=device)
    v = torch.as_tensor(np.ascontiguousarray(chain.val, dtype=np.float64), device=device)
    return rp, ci, v


class Hierarchy:
    """Owns a bamg_handle (the setup of bamg_setup)."""

    def __init__(self, n, row_ptr, col_idx, val, grid, r, options: Options | None = None, stream=None):
        lib = load()
        self._h = C.c_void_p()
        self.n = int(n)
        opts = options if options is not None else default_options()
        g = Grid(int(grid[0]), int(grid[1]), int(bool(grid[2])))
        _check(lib.bamg_setup(self.n, C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col_idx.data_ptr()),
                              C.c_void_p(val.data_ptr()), g, int(r), C.byref(opts), _stream_ptr(stream),
                              C.byref(self._h)))

    @classmethod
    def from_chain(cls, chain, r, options=None, stream=None):
        rp, ci, v = device_csr(chain)
        return cls(chain.n, rp, ci, v, (chain.nx, chain.ny, chain.periodic), r, options, stream)

    def solve(self, x, tol=1e-10, max_cycles=200, use_guess=False, parnoldi=False):
        info = SolveInfo()
        flags = (USE_GUESS if use_guess else 0) | (PARNOLDI if parnoldi else 0)
        rc = load().bamg_solve(self._h, C.c_void_p(x.data_ptr()), float(tol), int(max_cycles), flags, C.byref(info))
        _check(rc, allow=(ENOCONV,))
        return info

    def mle_iterate(self, x, tol=1e-10, max_cycles=50):
        """Stand-alone MLE iteration on this handle (bamg_mle_iterate)."""
        info = SolveInfo()
        rc = load().bamg_mle_iterate(self._h, C.c_void_p(x.data_ptr()), float(tol), int(max_cycles), C.byref(info))
        _check(rc, allow=(ENOCONV,))
        return info

    def stats(self) -> Stats:
        st = Stats()
        _check(load().bamg_get_stats(self._h, C.byref(st)))
        return st

    def level_info(self, l: int) -> LevelInfo:
        li = LevelInfo()
        _check(load().bamg_level_info_get(self._h, int(l), C.byref(li)))
        return li

    def export(self, l: int, what: int) -> np.ndarray:
        li = self.level_info(l)
        n = int(li.n)
        sizes = {X_B_ROWPTR: (n + 1, np.int32), X_B_COL: (li.nnz_b, np.int32), X_B_VAL: (li.nnz_b, np.float64),
                 X_T_ROWPTR: (n + 1, np.int32), X_T_COL: (li.nnz_t, np.int32), X_T_VAL: (li.nnz_t, np.float64),
                 X_P_COL: (4 * n, np.int32), X_P_VAL: (4 * n, np.float64), X_U: (n * li.r, np.float64),
                 X_V: (n * li.n_v, np.float64), X_LAMBDA: (2 * li.n_v, np.float64), X_VKIND: (li.n_v, np.int32),
                 X_X0: (n, np.float64), X_W: (n * n, np.float64), X_Y: (n, np.float64),
                 X_U0: (n * li.r, np.float64), X_FEATURES: (n * 24, np.float32), X_SLOTW: (n * 4, np.float32),
                 X_SLOTW0: (n * 4, np.float32), X_CMAP: (n, np.int32), X_CR_RHO: (li.cr_rounds, np.float64)}
        cnt, dt = sizes[what]
        out = np.empty(int(cnt), dtype=dt)
        _check(load().bamg_export(self._h, int(l), int(what), out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def apply_vcycle(self, f, e):
        _check(load().bamg_apply_vcycle(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(e.data_ptr())))

    def close(self):
        if self._h:
            _check(load().bamg_free(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def concat_chains(chains):
    """Block-diagonal concatenation: (row offsets, row_ptr, col_idx, val, grids) as numpy arrays."""
    off = np.zeros(len(chains) + 1, dtype=np.int64)
    for c, ch in enumerate(chains):
        off[c + 1] = off[c] + ch.n
    nnz = np.cumsum([0] + [len(ch.col_idx) for ch in chains])
    rp = np.concatenate([np.asarray(ch.row_ptr[:-1], dtype=np.int64) + nnz[c] for c, ch in enumerate(chains)]
                        + [np.array([nnz[-1]], dtype=np.int64)]).astype(np.int32)
    ci = np.concatenate([np.asarray(ch.col_idx, dtype=np.int64) + off[c] for c, ch in enumerate(chains)]).astype(np.int32)
    v = np.concatenate([np.asarray(ch.val, dtype=np.float64) for ch in chains])
    grids = np.array([(ch.nx, ch.ny, int(bool(ch.periodic))) for ch in chains], dtype=np.int32)
    return off, rp, ci, v, grids


class DeviceBatch:
    """Concatenated chains resident on the device (inputs of bamg_setup_batched)."""

    def __init__(self, chains, device="cuda"):
        import torch
        off, rp, ci, v, grids = concat_chains(chains)
        self.nchains = len(chains)
        self.offsets = off
        self.n = int(off[-1])
        self.row_ptr = torch.as_tensor(rp, device=device)
        self.col_idx = torch.as_tensor(ci, device=device)
        self.val = torch.as_tensor(v, device=device)
        self.grids = (Grid * self.nchains)(*[Grid(int(a), int(b), int(c)) for a, b, c in grids])


class BatchedHierarchy(Hierarchy):
    """Owns a bamg_handle made by bamg_setup_batched (several chains, one handle).
    `chains` is a list of Chain objects or a DeviceBatch already on the device."""

    def __init__(self, chains, r, options: Options | None = None, stream=None):
        lib = load()
        self._h = C.c_void_p()
        db = chains if isinstance(chains, DeviceBatch) else DeviceBatch(chains)
        self.nchains = db.nchains
        self.offsets = db.offsets
        self.n = db.n
        opts = options if options is not None else default_options()
        _check(lib.bamg_setup_batched(self.nchains, db.offsets.ctypes.data_as(C.c_void_p),
                                      C.c_void_p(db.row_ptr.data_ptr()), C.c_void_p(db.col_idx.data_ptr()),
                                      C.c_void_p(db.val.data_ptr()), db.grids, int(r), C.byref(opts),
                                      _stream_ptr(stream), C.byref(self._h)))

    def solve_batched(self, x, tol=1e-10, max_cycles=200, use_guess=False, parnoldi=False):
        """Returns (info, per-chain status int32 array, per-chain residual array)."""
        info = SolveInfo()
        status = np.zeros(self.nchains, dtype=np.int32)
        resid = np.zeros(self.nchains, dtype=np.float64)
        flags = (USE_GUESS if use_guess else 0) | (PARNOLDI if parnoldi else 0)
        rc = load().bamg_solve_batched(self._h, C.c_void_p(x.data_ptr()), float(tol), int(max_cycles),
                                       flags, status.ctypes.data_as(C.c_void_p),
                                       resid.ctypes.data_as(C.c_void_p), C.byref(info))
        _check(rc, allow=(ENOCONV,))
        return info, status, resid


def mlp_init(seed, stream=None):
    """Fresh network parameters (device FP32 tensor of MLP_NPARAM values)."""
    import torch
    th = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    _check(load().bamg_mlp_init(int(seed), C.c_void_p(th.data_ptr()), _stream_ptr(stream)))
    return th


def mlp_forward(feat, params, stream=None):
    import torch
    n = feat.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    _check(load().bamg_mlp_forward(C.c_void_p(feat.data_ptr()), n, C.c_void_p(params.data_ptr()),
                                   C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def mlp_forward_noalloc(feat, params, out, stream=None):
    """The allocation-free inference call: out (n x 4, FP32, device) is the
    caller's; the library stages through its static scratch."""
    _check(load().bamg_mlp_forward_noalloc(C.c_void_p(feat.data_ptr()), feat.shape[0], C.c_void_p(params.data_ptr()),
                                           C.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def mlp_loss_grad(feat, tgt, params, stream=None):
    import torch
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = C.c_double()
    _check(load().bamg_mlp_loss_grad(C.c_void_p(feat.data_ptr()), C.c_void_p(tgt.data_ptr()), feat.shape[0],
                                     C.c_void_p(params.data_ptr()), C.c_void_p(g.data_ptr()), C.byref(loss),
                                     _stream_ptr(stream)))
    return loss.value, g


def mlp_train(feat, tgt, params, vfeat=None, vtgt=None, epochs=8, batch=4096, lr=1e-3, seed=6, stream=None):
    """Adam on params (in place); returns the MlpTrainInfo."""
    o = MlpTrainOpts(int(epochs), int(batch), float(lr), 0.9, 0.999, 1e-8, int(seed))
    info = MlpTrainInfo()
    nv = 0 if vfeat is None else vfeat.shape[0]
    _check(load().bamg_mlp_train(C.c_void_p(feat.data_ptr()), C.c_void_p(tgt.data_ptr()), feat.shape[0],
                                 C.c_void_p(vfeat.data_ptr()) if nv else None,
                                 C.c_void_p(vtgt.data_ptr()) if nv else None, nv, C.c_void_p(params.data_ptr()),
                                 C.byref(o), C.byref(info), _stream_ptr(stream)))
    return info


def trim():
    """Return the library's cached device buffers to HIP."""
    _check(load().bamg_trim())


def relax(row_ptr, col_idx, val, X, R, omega=0.7, nu=1, F=None, stream=None):
    """nu omega-Jacobi sweeps on X (n x R, in place) for B = I - A."""
    n = row_ptr.numel() - 1
    _check(load().bamg_relax(n, C.c_void_p(row_ptr.data_ptr()), C.c_void_p(col_idx.data_ptr()),
                             C.c_void_p(val.data_ptr()), C.c_void_p(X.data_ptr()),
                             C.c_void_p(F.data_ptr()) if F is not None else None, int(R), float(omega), int(nu),
                             _stream_ptr(stream)))


def stationary(chain, r, tol=1e-10, max_cycles=200, parnoldi=False, **opts):
    """Setup + solve for a chain; returns (x as a CPU numpy array, solve info, hierarchy)."""
    import torch
    h = Hierarchy.from_chain(chain, r, default_options(**opts))
    x = torch.empty(chain.n, dtype=torch.float64, device="cuda")
    info = h.solve(x, tol, max_cycles, parnoldi=parnoldi)
    return x.cpu().numpy(), info, h


def mlp_collect(h):
    """Training pairs of a handle set up with options.collect (bamg_mlp_collect):
    (features n x 24, targets n x 4) as device FP32 tensors."""
    import torch
    lib = load()
    cnt = C.c_int64()
    _check(lib.bamg_mlp_collect(h._h, None, None, 0, C.byref(cnt)))
    n = int(cnt.value)
    f = torch.empty((max(n, 1), 24), dtype=torch.float32, device="cuda")
    t = torch.empty((max(n, 1), 4), dtype=torch.float32, device="cuda")
    _check(lib.bamg_mlp_collect(h._h, C.c_void_p(f.data_ptr()), C.c_void_p(t.data_ptr()), n, C.byref(cnt)))
    return f[:n], t[:n]


def train_spec(**kw) -> TrainSpec:
    sp = TrainSpec()
    load().bamg_train_spec_default(C.byref(sp))
    for k, v in kw.items():
        if k in ("epochs", "batch", "lr", "beta1", "beta2", "eps") or k == "shuffle_seed":
            setattr(sp.train, "seed" if k == "shuffle_seed" else k, v)
        elif hasattr(sp, k):
            setattr(sp, k, v)
        else:
            raise KeyError(k)
    return sp


def mlp_train_spec(spec: TrainSpec, out_path=None, stream=None):
    """bamg_mlp_train_spec: the library builds the training chains, collects
    the pairs and trains; returns (params (device FP32), MlpTrainInfo)."""
    import torch
    params = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    info = MlpTrainInfo()
    _check(load().bamg_mlp_train_spec(C.byref(spec), out_path.encode() if out_path else None,
                                      C.c_void_p(params.data_ptr()), C.byref(info), _stream_ptr(stream)))
    return params, info
