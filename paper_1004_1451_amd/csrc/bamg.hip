// Host orchestration and C ABI of the Bootstrap AMG library (see bamg.h).
//
// One handle = one hierarchy on one HIP stream.  Every numerical step runs in
// the kernels of k_sparse.h / k_dense.h / k_solve.h; the host plans levels,
// allocates, launches, and reads back a few scalars (error flags, the number
// of coarsest eigenvector columns, convergence estimates).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bamg.h"
#include "common.h"
#include "k_dense.h"
#include "k_solve.h"
#include "k_sparse.h"

namespace {

thread_local std::string g_last_error;

struct BamgError : std::runtime_error {
    int code;
    BamgError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw BamgError(code, buf);
}

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) fail(BAMG_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH(kern, grid, block, s, ...)                           \
    do {                                                            \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__); \
        HIPCHK(hipGetLastError());                                  \
    } while (0)

inline int nblk(long long n) { return (int)std::max<long long>(1, (n + BAMG_BLK - 1) / BAMG_BLK); }
constexpr int RED_PARTS = 1024;       // fixed partition of every FP64 reduction
constexpr int MDOT_BLOCKS = 1024;     // fixed row partition of the GMRES multi-dots

struct GridH {
    int nx, ny, periodic;
    long long n() const { return (long long)nx * ny; }
    GridH coarse() const { return {(nx + 1) / 2, (ny + 1) / 2, periodic}; }
    bool can_coarsen() const {
        if (periodic) return nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= 3 && ny / 2 >= 3;
        return n() > 1;
    }
    GridDev dev() const { return GridDev{nx, ny, periodic, FastDiv((uint32_t)ny)}; }
};

// Levels 0..L: "levels" counts the finest; 0 = coarsen while n > coarse_max.
std::vector<GridH> level_plan(GridH g, int levels, int coarse_max) {
    std::vector<GridH> plan{g};
    for (;;) {
        GridH c = plan.back();
        if (levels > 0 && (int)plan.size() >= levels) break;
        if (levels == 0 && c.n() <= coarse_max) break;
        if (!c.can_coarsen()) {
            if (levels > 0) fail(BAMG_EUNSUPPORTED, "grid %dx%d cannot be coarsened to %d levels", g.nx, g.ny, levels);
            break;
        }
        plan.push_back(c.coarse());
    }
    return plan;
}

// ------------------------------------------------------------------ memory
struct Arena {
    hipStream_t s = nullptr;
    size_t bytes = 0, budget = 0;
    std::vector<void*> ptrs;
    template <typename X>
    X* alloc(size_t count) {
        size_t b = std::max<size_t>(count, 1) * sizeof(X);
        b = (b + 255) & ~size_t(255);
        if (budget && bytes + b > budget) fail(BAMG_ENOMEM, "memory budget of %zu bytes exceeded", budget);
        void* p = nullptr;
        if (hipMallocAsync(&p, b, s) != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(BAMG_ENOMEM, "device allocation of %zu bytes failed", b);
        }
        bytes += b;
        ptrs.push_back(p);
        return (X*)p;
    }
    void release() {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
        ptrs.clear();
        bytes = 0;
    }
};

template <typename T>
struct Csr {
    int n = 0, cap = 0;
    int* rp = nullptr;
    int* ci = nullptr;
    T* v = nullptr;
};

template <typename T>
struct Level {
    GridH g{};
    int n = 0;
    Csr<T> B, Tm;           // Tm.rp == nullptr: T = I (finest level)
    T* dinv = nullptr;
    int* pc = nullptr;      // P: n x 4 (ELL)
    T* pv = nullptr;
    int* qc = nullptr;      // Q: n_{l+1} x 9 (ELL)
    T* qv = nullptr;
    T* U = nullptr;         // n x r relaxed test vectors
    T* V = nullptr;         // n x nv eigenvector approximations
    T *e = nullptr, *e2 = nullptr, *f = nullptr, *r = nullptr;   // cycle vectors
    unsigned short* mask = nullptr;
    int* cnt = nullptr;
};

}  // namespace

// ------------------------------------------------------------------ context
struct bamg_ctx {
    virtual ~bamg_ctx() {}
    virtual void setup(const int32_t* rp, const int32_t* ci, const double* val) = 0;
    virtual int solve(double* x, double tol, int max_cycles, uint32_t flags, bamg_solve_info* info) = 0;
    virtual void level_info(int l, bamg_level_info* out) = 0;
    virtual void export_item(int l, int what, void* dst, size_t bytes) = 0;
    virtual void vcycle_apply(const double* f, double* e) = 0;
    hipStream_t s = nullptr;
    bamg_options o{};
    bamg_stats st{};
    int r = 0;
    long long n = 0;
    GridH grid{};
};

namespace {

template <typename T>
struct Engine : bamg_ctx {
    Arena A;
    std::vector<GridH> plan;
    std::vector<Level<T>> L;
    // finest level in FP64 for the outer iteration
    int* b0rp = nullptr;
    int* b0ci = nullptr;
    double* b0v = nullptr;
    int nnz0 = 0;
    // coarsest level
    int nL = 0;
    double* W = nullptr;     // B_L^+ (n_L x n_L)
    float* Wf = nullptr;     // FP32 copy for the mixed cycle
    double* y = nullptr;     // null vector
    double* cvec = nullptr;  // T_L^T 1
    double* bcol = nullptr;
    double* tmpL = nullptr;  // n_L scratch vectors
    double* tmpL2 = nullptr;
    double* fL = nullptr;    // FP64 coarse right-hand side / solution
    double* eL = nullptr;
    // eigen tables (device): lam[2*8], kind[8], ent_col[8]
    double* lam = nullptr;
    int* kind = nullptr;
    int* ent_col = nullptr;
    int nv = 0, nent = 0;
    double* x0 = nullptr;
    // reductions
    double* part = nullptr;
    double* sc = nullptr;   // 64 device scalars
    double* wts = nullptr;  // TV weights (<= 64)
    int* err = nullptr;
    int* itmp = nullptr;    // scan scratch
    int* bsum = nullptr;
    int* total = nullptr;
    // FGMRES
    double *Vk = nullptr, *Zk = nullptr, *wk = nullptr, *Hg = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
           *ysol = nullptr, *hbuf = nullptr, *rvec = nullptr;
    double *v64 = nullptr, *z64 = nullptr;   // V-cycle entry/exit in FP64
    // Arnoldi
    double *Vb = nullptr, *Hh = nullptr, *Hrow = nullptr, *sel_lam = nullptr, *sel_s = nullptr, *ritz_re = nullptr,
           *ritz_im = nullptr;
    int* nsel = nullptr;
    double* ah = nullptr;   // Gram-Schmidt coefficients of one Arnoldi step
    // profiling
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_sweep, ev_gal, ev_ls;

    static constexpr bool MIXED = sizeof(T) == 4;

    ~Engine() override {
        for (auto* v : {&ev_sweep, &ev_gal, &ev_ls})
            for (auto& p : *v) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
        A.release();
        (void)hipStreamSynchronize(s);
    }

    // -------------------------------------------------------------- helpers
    void sync() { HIPCHK(hipStreamSynchronize(s)); }
    template <typename X>
    X get1(const X* p) {
        X v;
        HIPCHK(hipMemcpyAsync(&v, p, sizeof(X), hipMemcpyDeviceToHost, s));
        sync();
        return v;
    }
    void zero(void* p, size_t bytes) { HIPCHK(hipMemsetAsync(p, 0, bytes, s)); }

    void scan(int n, const int* cnt, int* out) {
        int nb = nblk(n);
        LAUNCH(k_scan_block, nb, BAMG_BLK, s, n, cnt, out, bsum);
        LAUNCH(k_scan_sums, 1, BAMG_BLK, s, nb, bsum, total);
        LAUNCH(k_scan_add, nb, BAMG_BLK, s, n, out, bsum, total);
    }

    // reductions into device scalar *out
    template <int OP>
    void reduce(long long n, const double* a, const double* b, double* out) {
        LAUNCH(k_reduce_partial<OP>, RED_PARTS, BAMG_BLK, s, n, a, b, part);
        LAUNCH(k_reduce_final, 1, BAMG_BLK, s, RED_PARTS, part, out);
    }

    std::pair<hipEvent_t, hipEvent_t> ev_begin() {
        std::pair<hipEvent_t, hipEvent_t> p;
        HIPCHK(hipEventCreate(&p.first));
        HIPCHK(hipEventCreate(&p.second));
        HIPCHK(hipEventRecord(p.first, s));
        return p;
    }
    void ev_end(std::pair<hipEvent_t, hipEvent_t> p, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
        HIPCHK(hipEventRecord(p.second, s));
        v.push_back(p);
    }

    // -------------------------------------------------------------- setup
    void allocate(int nnzA) {
        const int nl = (int)plan.size();
        const int kmax = std::max(1, o.n_eig) + 1;      // columns of V (a pair may add one)
        L.resize(nl);
        for (int l = 0; l < nl; ++l) {
            auto& lv = L[l];
            lv.g = plan[l];
            lv.n = (int)plan[l].n();
            if (l == 0) {
                lv.B.cap = nnzA + lv.n;
            } else {
                lv.B.cap = 9 * lv.n;
                lv.Tm.cap = 9 * lv.n;
                lv.Tm.rp = A.alloc<int>(lv.n + 1);
                lv.Tm.ci = A.alloc<int>(lv.Tm.cap);
                lv.Tm.v = A.alloc<T>(lv.Tm.cap);
            }
            lv.B.n = lv.n;
            lv.B.rp = A.alloc<int>(lv.n + 1);
            lv.B.ci = A.alloc<int>(lv.B.cap);
            lv.B.v = A.alloc<T>(lv.B.cap);
            lv.dinv = A.alloc<T>(lv.n);
            lv.U = A.alloc<T>((size_t)lv.n * r);
            lv.V = A.alloc<T>((size_t)lv.n * kmax);
            lv.e = A.alloc<T>(lv.n);
            lv.e2 = A.alloc<T>(lv.n);
            lv.f = A.alloc<T>(lv.n);
            lv.r = A.alloc<T>(lv.n);
            if (l + 1 < nl) {
                int nc = (int)plan[l + 1].n();
                lv.pc = A.alloc<int>((size_t)lv.n * 4);
                lv.pv = A.alloc<T>((size_t)lv.n * 4);
                lv.qc = A.alloc<int>((size_t)nc * 9);
                lv.qv = A.alloc<T>((size_t)nc * 9);
                lv.mask = A.alloc<unsigned short>(nc);
                lv.cnt = A.alloc<int>(nc);
            }
        }
        if (MIXED) {
            b0rp = A.alloc<int>(n + 1);
            b0ci = A.alloc<int>(L[0].B.cap);
            b0v = A.alloc<double>(L[0].B.cap);
        } else {
            b0rp = L[0].B.rp;
            b0ci = L[0].B.ci;
            b0v = (double*)L[0].B.v;
        }
        nL = L.back().n;
        W = A.alloc<double>((size_t)nL * nL);
        if (MIXED) Wf = A.alloc<float>((size_t)nL * nL);
        y = A.alloc<double>(nL);
        cvec = A.alloc<double>(nL);
        bcol = A.alloc<double>(nL);
        tmpL = A.alloc<double>(nL);
        tmpL2 = A.alloc<double>(nL);
        fL = A.alloc<double>(nL);
        eL = A.alloc<double>(nL);
        lam = A.alloc<double>(2 * 16);
        kind = A.alloc<int>(16);
        ent_col = A.alloc<int>(16);
        x0 = A.alloc<double>(n);
        {
            size_t need = std::max<size_t>((size_t)RED_PARTS * 2 * 64 + 4096,
                                           (size_t)MDOT_BLOCKS * (BAMG_BLK / BAMG_WAVE) * (o.gmres_m + 2));
            need = std::max<size_t>(need, (size_t)ceil_div(nL, GT_ROWS) * nL);
            part = A.alloc<double>(need);
        }
        sc = A.alloc<double>(64);
        wts = A.alloc<double>(64);
        err = A.alloc<int>(4);
        itmp = A.alloc<int>(n + 1);
        bsum = A.alloc<int>(nblk(n) + 1);
        total = A.alloc<int>(4);
        const int am = std::max(1, std::min({o.arnoldi_m, nL - 1, HQR_MAXM}));
        Vb = A.alloc<double>((size_t)nL * (am + 1));
        Hh = A.alloc<double>((size_t)(am + 1) * am);
        Hrow = A.alloc<double>((size_t)am * am);
        sel_lam = A.alloc<double>(2 * 16);
        sel_s = A.alloc<double>((size_t)16 * 2 * am);
        ritz_re = A.alloc<double>(nL);
        ritz_im = A.alloc<double>(nL);
        nsel = A.alloc<int>(4);
        ah = A.alloc<double>(HQR_MAXM + 8);
    }

    void build_b0(const int32_t* rp, const int32_t* ci, const double* val, int nnzA) {
        auto& lv = L[0];
        GridDev gd = lv.g.dev();
        double* colsum = A.alloc<double>(n);
        zero(colsum, sizeof(double) * n);
        zero(err, sizeof(int) * 4);
        LAUNCH(k_check_a, nblk(n), BAMG_BLK, s, (int)n, rp, ci, val, gd, nnzA, colsum, itmp, err);
        LAUNCH(k_check_colsum, nblk(n), BAMG_BLK, s, (int)n, colsum, err);
        int e = get1(err);
        if (e & ERR_RANGE) fail(BAMG_EINVAL, "CSR of A: row_ptr not monotone, column out of range, or columns not strictly ascending");
        if (e & ERR_NEG) fail(BAMG_ENOTSTOCH, "A has a negative, non-finite or > 1 entry");
        if (e & ERR_COLSUM) fail(BAMG_ENOTSTOCH, "a column of A does not sum to 1 within 1e-12");
        if (e & ERR_WIDE) fail(BAMG_EUNSUPPORTED, "A joins states farther apart than the 3x3 grid box");
        scan((int)n, itmp, b0rp);
        int nnzB = get1(b0rp + n);
        nnz0 = nnzB;
        T* lo = MIXED ? lv.B.v : nullptr;
        T* dlo = MIXED ? lv.dinv : nullptr;
        double* dinv64 = MIXED ? A.alloc<double>(n) : (double*)lv.dinv;
        LAUNCH(k_build_b<T>, nblk(n), BAMG_BLK, s, (int)n, rp, ci, val, b0rp, b0ci, b0v, lo, o.omega, dinv64, dlo, err);
        if (MIXED) {
            HIPCHK(hipMemcpyAsync(lv.B.rp, b0rp, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
            HIPCHK(hipMemcpyAsync(lv.B.ci, b0ci, sizeof(int) * nnzB, hipMemcpyDeviceToDevice, s));
        }
        e = get1(err);
        if (e & ERR_ZERODIAG) fail(BAMG_EZERODIAG, "b_ii <= 0 on the finest level");
    }

    void sweeps(int l, T* X, int R, int nu, bool profile) {
        auto& lv = L[l];
        T* a = X;
        T* b = sweep_tmp;
        FastDiv dR((uint32_t)R);
        long long tot = (long long)lv.n * R;
        for (int k = 0; k < nu; ++k) {
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (profile) ev = ev_begin();
            LAUNCH((k_sweep<T, T>), nblk(tot), BAMG_BLK, s, lv.n, R, dR, lv.B.rp, lv.B.ci, lv.B.v, lv.dinv, a,
                   (const T*)nullptr, b);
            if (profile) ev_end(ev, ev_sweep);
            std::swap(a, b);
        }
        if (a != X) HIPCHK(hipMemcpyAsync(X, a, sizeof(T) * tot, hipMemcpyDeviceToDevice, s));
    }
    T* sweep_tmp = nullptr;

    void tv_weights(int l, int Ru, int Rv, const T* U, const T* V) {
        auto& lv = L[l];
        int R = Ru + Rv;
        int bs = R * (BAMG_BLK / R);
        int grid = RED_PARTS;
        LAUNCH((k_colnorm_partial<T, T>), grid, bs, s, lv.n, Ru, Rv, FastDiv((uint32_t)R), lv.B.rp, lv.B.ci, lv.B.v,
               U, V, part);
        LAUNCH(k_colnorm_final, R, BAMG_BLK, s, grid, R, part, wts, (double*)nullptr);
    }

    void galerkin(int l, bool profile) {
        auto& f = L[l];
        auto& c = L[l + 1];
        GridH cg = c.g;
        FastDiv dcy((uint32_t)cg.ny);
        int nc = c.n;
        // B_{l+1} = Q (B P)
        for (int which = 0; which < 2; ++which) {
            Csr<T>& M = which == 0 ? f.B : f.Tm;
            Csr<T>& C = which == 0 ? c.B : c.Tm;
            const int* mrp = M.rp;
            const int gb = ceil_div(nc, GAL_ROWS);
            LAUNCH(k_galerkin_symbolic, gb, GAL_THREADS, s, nc, dcy, cg.nx, cg.ny, cg.periodic, f.qc, mrp, M.ci,
                   f.pc, f.cnt, f.mask);
            scan(nc, f.cnt, C.rp);
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (profile) ev = ev_begin();
            LAUNCH(k_galerkin_numeric<T>, gb, GAL_THREADS, s, nc, dcy, cg.nx, cg.ny, cg.periodic, f.qc,
                   (const T*)f.qv, mrp, M.ci, (const T*)M.v, f.pc, (const T*)f.pv, f.mask, C.rp, C.ci, C.v);
            if (profile) ev_end(ev, ev_gal);
        }
        zero(err, sizeof(int) * 4);
        LAUNCH(k_dinv<T>, nblk(nc), BAMG_BLK, s, nc, c.B.rp, c.B.ci, c.B.v, o.omega, c.dinv, err);
    }

    void build_level(int l, int Ru, int Rv, const T* U, const T* V, T* inject, bool profile) {
        auto& lv = L[l];
        auto& c = L[l + 1];
        tv_weights(l, Ru, Rv, U, V);
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (profile) ev = ev_begin();
        LAUNCH((k_ls_fit<T, T>), nblk(lv.n), BAMG_BLK, s, lv.n, lv.g.dev(), c.g.ny, Ru, Rv, U, V, (const double*)wts,
               o.caliber, lv.pc, lv.pv, inject, (int*)nullptr);
        if (profile) ev_end(ev, ev_ls);
        LAUNCH(k_build_q<T>, nblk(c.n), BAMG_BLK, s, c.n, lv.g.dev(), FastDiv((uint32_t)c.g.ny), c.g.ny, lv.pc, lv.qc,
               lv.qv);
        galerkin(l, profile);
    }

    // Inverse of the padded coarsest operator [[B_11, 0], [0, 1]] into W by
    // block LU of its block-tridiagonal (+ periodic corner) structure; the
    // dense B_L is in W on entry.  Grid rows give blocks of b = ny <= 64.
    double* btbuf = nullptr;
    void block_tridiagonal_inverse(const GridH& g) {
        const int nx = g.nx, b = g.ny, K = nx - 1, bb = b * b;
        const bool arrow = g.periodic && nx >= 3;
        if (!btbuf) btbuf = A.alloc<double>((size_t)5 * nx * bb);
        double* Dk = btbuf;
        double* Up = Dk + (size_t)nx * bb;
        double* Lo = Up + (size_t)nx * bb;
        double* Cl = Lo + (size_t)nx * bb;
        double* Rw = Cl + (size_t)nx * bb;
        {
            dim3 grid(ceil_div(bb, BAMG_BLK), nx, arrow ? 5 : 3);
            hipLaunchKernelGGL(k_bt_extract, grid, dim3(BAMG_BLK), 0, s, nx, b, (const double*)W, Dk, Up, Lo, Cl, Rw);
            HIPCHK(hipGetLastError());
        }
        auto blk = [&](double* base, int k) { return base + (size_t)k * bb; };
        auto inv = [&](int k) {
            LAUNCH(k_gj_diag, 1, BAMG_BLK, s, b, 0, b, blk(Dk, k), (const double*)(sc + 10), sc + 11);
        };
        for (int k = 0; k < K; ++k) {
            inv(k);
            BlkOps g1{}, g2{};
            if (k + 1 < K) {
                int q = 0;
                g1.A[q] = blk(Lo, k + 1); g1.B[q] = blk(Dk, k); g1.C[q] = blk(Lo, k + 1); g1.mode[q++] = 0;
                if (arrow) { g1.A[q] = blk(Rw, k); g1.B[q] = blk(Dk, k); g1.C[q] = blk(Rw, k); g1.mode[q++] = 0; }
                LAUNCH(k_blk_gemm, q, BAMG_BLK, s, b, g1);
                q = 0;
                g2.A[q] = blk(Lo, k + 1); g2.B[q] = blk(Up, k); g2.C[q] = blk(Dk, k + 1); g2.mode[q++] = 1;
                if (arrow) {
                    double* colK = (k + 1 < K - 1) ? blk(Cl, k + 1) : blk(Up, k + 1);
                    double* rowK = (k + 1 < K - 1) ? blk(Rw, k + 1) : blk(Lo, K);
                    g2.A[q] = blk(Lo, k + 1); g2.B[q] = blk(Cl, k); g2.C[q] = colK; g2.mode[q++] = 1;
                    g2.A[q] = blk(Rw, k); g2.B[q] = blk(Up, k); g2.C[q] = rowK; g2.mode[q++] = 1;
                    g2.A[q] = blk(Rw, k); g2.B[q] = blk(Cl, k); g2.C[q] = blk(Dk, K); g2.mode[q++] = 1;
                }
                LAUNCH(k_blk_gemm, q, BAMG_BLK, s, b, g2);
            } else {
                g1.A[0] = blk(Lo, K); g1.B[0] = blk(Dk, k); g1.C[0] = blk(Lo, K); g1.mode[0] = 0;
                LAUNCH(k_blk_gemm, 1, BAMG_BLK, s, b, g1);
                g2.A[0] = blk(Lo, K); g2.B[0] = blk(Up, k); g2.C[0] = blk(Dk, K); g2.mode[0] = 1;
                LAUNCH(k_blk_gemm, 1, BAMG_BLK, s, b, g2);
            }
        }
        inv(K);
        // forward substitution on the identity: W[k] = E_k - sum L_kj W[j]
        const long long nn = (long long)nL * nL;
        LAUNCH(k_identity, nblk(nn), BAMG_BLK, s, nn, nL, W);
        const int ct = ceil_div(nL, 64);
        for (int k = 1; k < K; ++k)
            LAUNCH(k_bt_strip, ct, BAMG_BLK, s, b, nL, W, k, (const double*)blk(Lo, k), k - 1, (const double*)nullptr,
                   0, (const double*)nullptr);
        if (K >= 1) {
            if (arrow)
                for (int j = 0; j < K - 1; j += 2) {
                    const double* A2 = j + 1 < K - 1 ? blk(Rw, j + 1) : nullptr;
                    LAUNCH(k_bt_strip, ct, BAMG_BLK, s, b, nL, W, K, (const double*)blk(Rw, j), j, A2, j + 1,
                           (const double*)nullptr);
                }
            LAUNCH(k_bt_strip, ct, BAMG_BLK, s, b, nL, W, K, (const double*)blk(Lo, K), K - 1, (const double*)nullptr,
                   0, (const double*)nullptr);
        }
        // back substitution: W[k] = Dinv_k (W[k] - U_k W[k+1] - C_k W[K])
        LAUNCH(k_bt_strip, ct, BAMG_BLK, s, b, nL, W, K, (const double*)nullptr, 0, (const double*)nullptr, 0,
               (const double*)blk(Dk, K));
        for (int k = K - 1; k >= 0; --k) {
            const double* A2 = (arrow && k < K - 1) ? blk(Cl, k) : nullptr;
            LAUNCH(k_bt_strip, ct, BAMG_BLK, s, b, nL, W, k, (const double*)blk(Up, k), k + 1, A2, K,
                   (const double*)blk(Dk, k));
        }
    }

    // Dense pseudo-inverse of the coarsest operator into W, null vector y.
    void coarsest_inverse() {
        auto& cl = L.back();
        const int m = nL - 1;
        const long long nn = (long long)nL * nL;
        LAUNCH(k_fill, nblk(nn), BAMG_BLK, s, nn, 0.0, W);
        LAUNCH(k_densify_cast<T>, nblk(nL), BAMG_BLK, s, nL, cl.B.rp, cl.B.ci, cl.B.v, W);
        LAUNCH(k_get_col, nblk(nL), BAMG_BLK, s, nL, nL, nL - 1, W, bcol);
        LAUNCH(k_absmax_partial, 64, BAMG_BLK, s, nn, W, part);
        LAUNCH(k_absmax_partial, 1, BAMG_BLK, s, 64LL, part, sc + 10);
        double big = 1e300;
        HIPCHK(hipMemcpyAsync(sc + 11, &big, sizeof(double), hipMemcpyHostToDevice, s));
        if (m > 0) {
            if (cl.g.ny <= GJ_NB) {
                block_tridiagonal_inverse(cl.g);
            } else {
                const int tiles = ceil_div(m, 64);
                const int ut = ceil_div(m, GJ_T);
                for (int k0 = 0; k0 < m; k0 += GJ_NB) {
                    int nb = std::min(GJ_NB, m - k0);
                    LAUNCH(k_gj_diag, 1, BAMG_BLK, s, nL, k0, nb, W, (const double*)(sc + 10), sc + 11);
                    LAUNCH(k_gj_rowpanel, tiles, BAMG_BLK, s, m, nL, k0, nb, W);
                    LAUNCH(k_gj_update, ut * ut, BAMG_BLK, s, m, nL, k0, nb, W);
                    LAUNCH(k_gj_colpanel, tiles, BAMG_BLK, s, m, nL, k0, nb, W);
                }
            }
        }
        LAUNCH(k_zero_border, nblk(nL), BAMG_BLK, s, nL, W);
        // y = [-Binv b_col; 1]
        if (m > 0) LAUNCH(k_gemv, ceil_div(m, 4), BAMG_BLK, s, m, m, nL, (const double*)W, (const double*)bcol, tmpL);
        LAUNCH(k_null_finish, nblk(nL), BAMG_BLK, s, nL, (const double*)tmpL, y);
        // projections: s = W 1, u = y^T W, sc0 = y^T s, sc1 = y^T y
        LAUNCH(k_fill, nblk(nL), BAMG_BLK, s, (long long)nL, 1.0, tmpL2);
        LAUNCH(k_gemv, ceil_div(nL, 4), BAMG_BLK, s, nL, nL, nL, (const double*)W, (const double*)tmpL2, tmpL);
        {
            dim3 gt(nblk(nL), ceil_div(nL, GT_ROWS));
            hipLaunchKernelGGL(k_gemv_t_partial, gt, dim3(BAMG_BLK), 0, s, nL, nL, nL, (const double*)W,
                               (const double*)y, part);
            HIPCHK(hipGetLastError());
            LAUNCH(k_gemv_t_final, nblk(nL), BAMG_BLK, s, (int)gt.y, nL, (const double*)part, tmpL2);
        }
        LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)y, (const double*)tmpL, sc + 0);
        LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)y, (const double*)y, sc + 1);
        LAUNCH(k_project_w, nblk(nn), BAMG_BLK, s, nL, W, (const double*)tmpL, (const double*)tmpL2, (const double*)y,
               (const double*)sc);
        // c = T^T 1, cy = c^T y
        LAUNCH(k_colsum_box<T>, nblk(nL), BAMG_BLK, s, nL, FastDiv((uint32_t)cl.g.ny), cl.g.nx, cl.g.ny,
               cl.g.periodic, cl.Tm.rp, cl.Tm.ci, (const T*)cl.Tm.v, cvec);
        LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)cvec, (const double*)y, sc + 2);
        st.coarsest_min_pivot = get1(sc + 11);
        if (m > 0 && !(st.coarsest_min_pivot > 1e-12))
            fail(BAMG_ESINGULAR, "coarsest pivot %.3e below 1e-12 of max |B_L|", st.coarsest_min_pivot);
        if (MIXED) LAUNCH((k_cast<double, float>), nblk(nn), BAMG_BLK, s, nn, (const double*)W, Wf);
    }

    // Coarsest eigenpairs (Algorithm 3, l = L) by Arnoldi on the shift-invert
    // operator; fills V_L, lam, kind, ent_col and nv.
    void coarsest_eigs() {
        auto& cl = L.back();
        const int want = o.n_eig - 1;
        int am = std::min({o.arnoldi_m, nL - 1, HQR_MAXM});
        int ne = 0, ncols = 0;
        if (want > 0 && am >= 1) {
            zero(Hh, sizeof(double) * (am + 1) * am);
            LAUNCH(k_rand_vec, nblk(nL), BAMG_BLK, s, nL, o.seed, Vb);
            LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)cvec, (const double*)Vb, sc + 3);
            LAUNCH(k_project_domain, nblk(nL), BAMG_BLK, s, nL, (const double*)y, (const double*)(sc + 3),
                   (const double*)(sc + 2), Vb);
            LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)Vb, (const double*)Vb, sc + 4);
            LAUNCH(k_normalize_into, nblk(nL), BAMG_BLK, s, nL, (const double*)Vb, (const double*)(sc + 4), Vb, sc + 5);
            for (int j = 0; j < am; ++j) {
                double* vj = Vb + (size_t)j * nL;
                // w = T v_j
                if (cl.Tm.rp) {
                    LAUNCH(k_spmv<T>, nblk(nL), BAMG_BLK, s, nL, cl.Tm.rp, cl.Tm.ci, (const T*)cl.Tm.v,
                           (const double*)vj, 1.0, tmpL);
                } else {
                    LAUNCH(k_copy, nblk(nL), BAMG_BLK, s, (long long)nL, (const double*)vj, tmpL);
                }
                double* u = Vb + (size_t)(j + 1) * nL;
                LAUNCH(k_gemv, ceil_div(nL, 4), BAMG_BLK, s, nL, nL, nL, (const double*)W, (const double*)tmpL, u);
                LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)cvec, (const double*)u, sc + 3);
                LAUNCH(k_project_domain, nblk(nL), BAMG_BLK, s, nL, (const double*)y, (const double*)(sc + 3),
                       (const double*)(sc + 2), u);
                double* hcol = Hh + (size_t)j * (am + 1);
                for (int pass = 0; pass < 2; ++pass) {
                    LAUNCH(k_mdot, j + 1, BAMG_BLK, s, nL, j + 1, (const double*)Vb, (const double*)u, ah);
                    LAUNCH(k_mupdate, nblk(nL), BAMG_BLK, s, nL, j + 1, (const double*)Vb, (const double*)ah, u,
                           hcol);
                }
                LAUNCH(k_dot1, 1, BAMG_BLK, s, nL, (const double*)u, (const double*)u, sc + 4);
                LAUNCH(k_normalize_into, nblk(nL), BAMG_BLK, s, nL, (const double*)u, (const double*)(sc + 4), u,
                       hcol + j + 1);
            }
            LAUNCH(k_hessenberg_eig, 1, BAMG_WAVE, s, am, want, (const double*)Hh, Hrow, nsel, sel_lam, sel_s);
            int h[4];
            HIPCHK(hipMemcpyAsync(h, nsel, sizeof(int) * 3, hipMemcpyDeviceToHost, s));
            sync();
            if (h[2]) fail(BAMG_EDEVICE, "Hessenberg QR of the coarsest Arnoldi matrix did not converge");
            ne = h[0];
            ncols = h[1];
        }
        nv = 1 + ncols;
        nent = 1 + ne;
        // V_L: column 0 = y / (c^T y), then normalised Ritz vectors
        double* VL = MIXED ? A.alloc<double>((size_t)nL * nv) : (double*)cl.V;
        LAUNCH(k_scale_into_col, nblk(nL), BAMG_BLK, s, nL, (const double*)y, (const double*)(sc + 2), VL, nv, 0);
        std::vector<double> hl(2 * 16);
        int col = 1;
        if (ne > 0) {
            HIPCHK(hipMemcpyAsync(hl.data(), sel_lam, sizeof(double) * 2 * ne, hipMemcpyDeviceToHost, s));
            sync();
        }
        for (int e = 0; e < ne; ++e) {
            bool pair = hl[2 * e + 1] != 0.0;
            LAUNCH(k_ritz, nblk(nL), BAMG_BLK, s, nL, am, (const double*)Vb, (const double*)(sel_s + (size_t)e * 2 * am),
                   ritz_re, ritz_im);
            LAUNCH(k_eigvec_normalise, 1, BAMG_BLK, s, nL, (const double*)ritz_re, (const double*)ritz_im, pair ? 1 : 0,
                   VL, nv, col);
            col += pair ? 2 : 1;
        }
        LAUNCH(k_eig_tables, 1, 64, s, (const int*)nsel, (const double*)sel_lam, lam, kind, ent_col);
        if (ne == 0) {
            // no nonzero eigenpairs requested or available: only the null vector
            std::vector<double> z(4, 0.0);
            std::vector<int> kz(2, 0);
            HIPCHK(hipMemcpyAsync(lam, z.data(), sizeof(double) * 2, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(kind, kz.data(), sizeof(int), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(ent_col, kz.data(), sizeof(int), hipMemcpyHostToDevice, s));
        }
        if (MIXED) LAUNCH((k_cast<double, float>), nblk((long long)nL * nv), BAMG_BLK, s, (long long)nL * nv,
                          (const double*)VL, (float*)cl.V);
    }

    void upleg() {
        for (int l = (int)L.size() - 2; l >= 0; --l) {
            auto& lv = L[l];
            auto& c = L[l + 1];
            long long tot = (long long)lv.n * nv;
            FastDiv dR((uint32_t)nv);
            LAUNCH((k_interp<T, T>), nblk(tot), BAMG_BLK, s, lv.n, nv, dR, lv.pc, (const T*)lv.pv, (const T*)c.V, lv.V);
            T* a = lv.V;
            T* b = sweep_tmp;
            for (int k = 0; k < o.nu_setup; ++k) {
                LAUNCH((k_eig_relax<T, T>), nblk(lv.n), BAMG_BLK, s, lv.n, nv, lv.B.rp, lv.B.ci, (const T*)lv.B.v,
                       lv.Tm.rp, lv.Tm.ci, (const T*)lv.Tm.v, (const double*)lam, (const int*)kind, o.omega,
                       (const T*)a, b);
                std::swap(a, b);
            }
            if (a != lv.V) HIPCHK(hipMemcpyAsync(lv.V, a, sizeof(T) * tot, hipMemcpyDeviceToDevice, s));
            if (nent > 1) {
                const int grid = 256;
                LAUNCH((k_rayleigh_partial<T, T>), grid, BAMG_BLK, s, lv.n, nv, nent, (const int*)ent_col,
                       (const int*)kind, lv.B.rp, lv.B.ci, (const T*)lv.B.v, lv.Tm.rp, lv.Tm.ci, (const T*)lv.Tm.v,
                       (const T*)lv.V, part);
                LAUNCH(k_rayleigh_final, nent, BAMG_BLK, s, grid, nent, (const int*)ent_col, (const int*)kind,
                       (const double*)part, lam);
            }
        }
        // x0 = V_0[:, 0] / sum
        auto& l0 = L[0];
        extract_col0(l0.V, nv, x0);
        reduce<RED_SUM>(n, x0, nullptr, sc + 7);
        LAUNCH(k_scale, nblk(n), BAMG_BLK, s, (int)n, (const double*)x0, (const double*)nullptr,
               (const double*)(sc + 7), 0, x0);
    }

    void extract_col0(const T* V, int R, double* out) {
        LAUNCH((k_get_col_t<T>), nblk(n), BAMG_BLK, s, (int)n, R, 0, V, out);
    }

    void setup(const int32_t* rp, const int32_t* ci, const double* val) override {
        auto t0 = std::chrono::steady_clock::now();
        A.s = s;
        A.budget = o.mem_budget;
        plan = level_plan(grid, o.levels, o.coarse_max);
        int hr[2];
        HIPCHK(hipMemcpyAsync(&hr[0], rp, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hr[1], rp + n, sizeof(int), hipMemcpyDeviceToHost, s));
        sync();
        if (hr[0] != 0 || hr[1] < 0) fail(BAMG_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] >= 0");
        const int nnzA = hr[1];
        allocate(nnzA);
        const int kmax = std::max(1, o.n_eig) + 1;
        sweep_tmp = A.alloc<T>((size_t)n * std::max(r, kmax));
        build_b0(rp, ci, val, nnzA);
        const bool prof = o.profile != 0;
        // initial test vectors
        LAUNCH(k_tv_init<T>, nblk((long long)n * r), BAMG_BLK, s, (long long)n * r, o.seed, L[0].U);
        // down-leg: relax, fit, Galerkin, inject
        const int nl = (int)L.size();
        for (int l = 0; l + 1 < nl; ++l) {
            sweeps(l, L[l].U, r, o.nu_setup, prof && l == 0);
            build_level(l, r, 0, L[l].U, nullptr, L[l + 1].U, prof && l == 0);
        }
        if (o.stop_after == 1) { finish_setup(t0); return; }
        coarsest_inverse();
        coarsest_eigs();
        if (o.stop_after == 2) { finish_setup(t0); return; }
        upleg();
        if (o.stop_after == 3) { finish_setup(t0); return; }
        // recompute every P, B, T from U u V
        for (int l = 0; l + 1 < nl; ++l) build_level(l, r, nv, L[l].U, L[l].V, nullptr, prof && l == 0);
        coarsest_inverse();
        finish_setup(t0);
    }

    void finish_setup(std::chrono::steady_clock::time_point t0) {
        sync();
        st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st.n_levels = (int)L.size();
        st.n_v = nv;
        long long tot = 0;
        for (auto& lv : L) {
            int z;
            HIPCHK(hipMemcpyAsync(&z, lv.B.rp + lv.n, sizeof(int), hipMemcpyDeviceToHost, s));
            sync();
            tot += z;
        }
        st.op_complexity = nnz0 > 0 ? (double)tot / nnz0 : 0.0;
        auto acc = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& ms, int& cnt) {
            ms = 0; cnt = 0;
            for (auto& p : v) {
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, p.first, p.second));
                ms += t; ++cnt;
                (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second);
            }
            v.clear();
        };
        acc(ev_sweep, st.sweep_ms, st.sweep_launches);
        acc(ev_gal, st.galerkin_ms, st.galerkin_launches);
        acc(ev_ls, st.lsfit_ms, st.lsfit_launches);
        // algorithmic bytes of one level-0 launch
        const long long n0 = L[0].n;
        const int vb = sizeof(T);
        st.sweep_bytes = (long long)(n0 + 1) * 4 + (long long)nnz0 * (4 + vb) + n0 * vb + 2LL * n0 * r * vb;
        if (L.size() > 1) {
            long long nc = L[1].n;
            // numeric Galerkin of B: Q (9 per coarse row), B, P read; C written
            st.galerkin_bytes = nc * 9 * (4 + vb) + (long long)(n0 + 1) * 4 + (long long)nnz0 * (4 + vb) +
                                n0 * 4 * (4 + vb) + (nc + 1) * 4 + nc * 9 * (4 + vb);
            st.lsfit_bytes = n0 * (long long)(r + nv) * vb + n0 * 4 * (4 + vb);
        }
    }

    // -------------------------------------------------------------- cycle
    // e_l = C f_l on level l (vectors in the level's cycle buffers, type T);
    // result left in lv.e.
    void vcycle(int l) {
        auto& lv = L[l];
        if (l == (int)L.size() - 1) {
            if (MIXED) {
                LAUNCH(k_gemv_f32, ceil_div(nL, 4), BAMG_BLK, s, nL, nL, nL, (const float*)Wf, (const float*)lv.f,
                       (float*)lv.e);
            } else {
                LAUNCH(k_gemv, ceil_div(nL, 4), BAMG_BLK, s, nL, nL, nL, (const double*)W, (const double*)lv.f,
                       (double*)lv.e);
            }
            return;
        }
        auto& c = L[l + 1];
        FastDiv d1(1u);
        T* cur = lv.e;
        T* oth = lv.e2;
        int nb = nblk(lv.n);
        if (o.nu_pre > 0) {
            LAUNCH((k_jacobi_zero<T, T>), nb, BAMG_BLK, s, lv.n, (const T*)lv.dinv, (const T*)lv.f, cur);
            for (int k = 1; k < o.nu_pre; ++k) {
                LAUNCH((k_sweep<T, T>), nb, BAMG_BLK, s, lv.n, 1, d1, lv.B.rp, lv.B.ci, (const T*)lv.B.v,
                       (const T*)lv.dinv, (const T*)cur, (const T*)lv.f, oth);
                std::swap(cur, oth);
            }
        } else {
            zero(cur, sizeof(T) * lv.n);
        }
        LAUNCH((k_residual<T, T>), nb, BAMG_BLK, s, lv.n, lv.B.rp, lv.B.ci, (const T*)lv.B.v, (const T*)cur,
               (const T*)lv.f, lv.r);
        LAUNCH((k_restrict<T, T>), nblk(c.n), BAMG_BLK, s, c.n, lv.qc, (const T*)lv.qv, (const T*)lv.r, c.f);
        vcycle(l + 1);
        LAUNCH((k_prolong_add<T, T>), nb, BAMG_BLK, s, lv.n, lv.pc, (const T*)lv.pv, (const T*)c.e, cur);
        for (int k = 0; k < o.nu_post; ++k) {
            LAUNCH((k_sweep<T, T>), nb, BAMG_BLK, s, lv.n, 1, d1, lv.B.rp, lv.B.ci, (const T*)lv.B.v,
                   (const T*)lv.dinv, (const T*)cur, (const T*)lv.f, oth);
            std::swap(cur, oth);
        }
        if (cur != lv.e) std::swap(lv.e, lv.e2);   // keep the result in lv.e
    }

    // z = C v for FP64 level-0 vectors.
    void precondition(const double* v, double* z);

    void vcycle_apply(const double* f, double* e) override {
        precondition(f, e);
        sync();
    }

    // -------------------------------------------------------------- solve
    int solve(double* x, double tol, int max_cycles, uint32_t flags, bamg_solve_info* info) override {
        auto t0 = std::chrono::steady_clock::now();
        const int m = std::max(1, o.gmres_m);
        const int N = (int)n;
        if (!Vk) {
            Vk = A.alloc<double>((size_t)(m + 1) * N);
            Zk = A.alloc<double>((size_t)m * N);
            wk = A.alloc<double>(N);
            rvec = A.alloc<double>(N);
            Hg = A.alloc<double>((size_t)(m + 1) * m);
            cs = A.alloc<double>(m + 1);
            sn = A.alloc<double>(m + 1);
            g = A.alloc<double>(m + 2);
            ysol = A.alloc<double>(m + 1);
            hbuf = A.alloc<double>(m + 2);
        }
        bamg_solve_info inf{};
        if (!(flags & BAMG_USE_GUESS)) HIPCHK(hipMemcpyAsync(x, x0, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        auto normalise = [&]() {
            reduce<RED_SUM>(N, x, nullptr, sc + 20);
            LAUNCH(k_scale, nblk(N), BAMG_BLK, s, N, (const double*)x, (const double*)nullptr, (const double*)(sc + 20),
                   0, x);
        };
        normalise();
        const int nb = nblk(N);
        for (;;) {
            // r = -B x; relative 1-norm residual
            LAUNCH(k_spmv<double>, nb, BAMG_BLK, s, N, b0rp, b0ci, (const double*)b0v, (const double*)x, -1.0, rvec);
            reduce<RED_ABS>(N, rvec, nullptr, sc + 21);
            reduce<RED_ABS>(N, x, nullptr, sc + 22);
            reduce<RED_DOT>(N, rvec, rvec, sc + 23);
            double h3[3];
            HIPCHK(hipMemcpyAsync(h3, sc + 21, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
            sync();
            double rel = h3[0] / h3[1];
            inf.residual_l1 = rel;
            if (inf.history_len < 256) inf.history[inf.history_len++] = rel;
            if (rel <= tol) { inf.converged = 1; break; }
            if (inf.cycles >= max_cycles || !(rel == rel)) break;
            double beta = std::sqrt(h3[2]);
            double inner_tol = 0.5 * tol * h3[1] * beta / h3[0];
            zero(Hg, sizeof(double) * (m + 1) * m);
            LAUNCH(k_gmres_init, 1, 64, s, m, (const double*)(sc + 23), g);
            LAUNCH(k_scale, nb, BAMG_BLK, s, N, (const double*)rvec, (const double*)nullptr, (const double*)(sc + 23),
                   1, Vk);
            int kdone = 0;
            for (int j = 0; j < m && inf.cycles < max_cycles; ++j) {
                double* vj = Vk + (size_t)j * N;
                double* zj = Zk + (size_t)j * N;
                precondition(vj, zj);
                ++inf.cycles;
                LAUNCH(k_spmv<double>, nb, BAMG_BLK, s, N, b0rp, b0ci, (const double*)b0v, (const double*)zj, 1.0, wk);
                double* hcol = Hg + (size_t)j * (m + 1);
                for (int pass = 0; pass < 2; ++pass) {
                    LAUNCH(k_mdot_partial, MDOT_BLOCKS, BAMG_BLK, s, N, j + 1, (const double*)Vk, (const double*)wk,
                           part);
                    LAUNCH(k_mdot_final, j + 1, BAMG_BLK, s, MDOT_BLOCKS * (BAMG_BLK / BAMG_WAVE), j + 1,
                           (const double*)part, hbuf, hcol);
                    LAUNCH(k_vupdate, nb, BAMG_BLK, s, N, j + 1, (const double*)Vk, (const double*)hbuf, wk);
                }
                reduce<RED_DOT>(N, wk, wk, sc + 24);
                LAUNCH(k_scale, nb, BAMG_BLK, s, N, (const double*)wk, (const double*)nullptr, (const double*)(sc + 24),
                       1, Vk + (size_t)(j + 1) * N);
                LAUNCH(k_givens, 1, 64, s, j, m + 1, Hg, (const double*)(sc + 24), cs, sn, g, sc + 26);
                double h3b[3];
                HIPCHK(hipMemcpyAsync(h3b, sc + 24, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
                sync();
                double hn = std::sqrt(h3b[0]), est = h3b[2];
                kdone = j + 1;
                if (est <= inner_tol || hn == 0.0) break;
            }
            if (kdone > 0) {
                LAUNCH(k_gmres_y, 1, 64, s, kdone, m + 1, (const double*)Hg, (const double*)g, ysol);
                LAUNCH(k_xupdate, nb, BAMG_BLK, s, N, kdone, (const double*)Zk, (const double*)ysol, x);
            }
            normalise();
            ++inf.restarts;
        }
        // x >= 0, sum 1
        reduce<RED_NEGSUM>(N, x, nullptr, sc + 27);
        LAUNCH(k_clamp, nb, BAMG_BLK, s, N, x);
        normalise();
        LAUNCH(k_spmv<double>, nb, BAMG_BLK, s, N, b0rp, b0ci, (const double*)b0v, (const double*)x, -1.0, rvec);
        reduce<RED_ABS>(N, rvec, nullptr, sc + 21);
        reduce<RED_ABS>(N, x, nullptr, sc + 22);
        double h4[7];
        HIPCHK(hipMemcpyAsync(h4, sc + 21, sizeof(double) * 7, hipMemcpyDeviceToHost, s));
        sync();
        inf.residual_l1 = h4[0] / h4[1];
        inf.clamped_mass = h4[6];
        inf.converged = inf.residual_l1 <= tol;
        st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return inf.converged ? BAMG_OK : BAMG_ENOCONV;
    }

    // -------------------------------------------------------------- inspection
    void level_info(int l, bamg_level_info* out) override {
        if (l < 0 || l >= (int)L.size()) fail(BAMG_EINVAL, "level %d out of range", l);
        auto& lv = L[l];
        memset(out, 0, sizeof *out);
        out->n = lv.n;
        out->nx = lv.g.nx; out->ny = lv.g.ny; out->periodic = lv.g.periodic;
        int z = 0;
        HIPCHK(hipMemcpyAsync(&z, lv.B.rp + lv.n, sizeof(int), hipMemcpyDeviceToHost, s));
        sync();
        out->nnz_b = z;
        if (lv.Tm.rp) {
            HIPCHK(hipMemcpyAsync(&z, lv.Tm.rp + lv.n, sizeof(int), hipMemcpyDeviceToHost, s));
            sync();
            out->nnz_t = z;
        }
        if (lv.pc) out->nnz_p = 4LL * lv.n;
        out->r = r;
        out->n_v = nv;
    }

    template <typename X>
    void copy_out(const X* src, size_t count, void* dst, size_t bytes) {
        if (bytes < count * sizeof(X)) fail(BAMG_EINVAL, "export buffer too small (%zu < %zu)", bytes, count * sizeof(X));
        HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(X), hipMemcpyDeviceToHost, s));
        sync();
    }
    void copy_out_T(const T* src, size_t count, void* dst, size_t bytes) {
        if (bytes < count * sizeof(double)) fail(BAMG_EINVAL, "export buffer too small");
        if (!MIXED) { copy_out((const double*)src, count, dst, bytes); return; }
        std::vector<T> h(count);
        HIPCHK(hipMemcpyAsync(h.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s));
        sync();
        for (size_t i = 0; i < count; ++i) ((double*)dst)[i] = (double)h[i];
    }

    void export_item(int l, int what, void* dst, size_t bytes) override {
        if (l < 0 || l >= (int)L.size()) fail(BAMG_EINVAL, "level %d out of range", l);
        auto& lv = L[l];
        sync();
        int nnzb = 0, nnzt = 0;
        HIPCHK(hipMemcpyAsync(&nnzb, lv.B.rp + lv.n, sizeof(int), hipMemcpyDeviceToHost, s));
        if (lv.Tm.rp) HIPCHK(hipMemcpyAsync(&nnzt, lv.Tm.rp + lv.n, sizeof(int), hipMemcpyDeviceToHost, s));
        sync();
        const bool last = l == (int)L.size() - 1;
        switch (what) {
            case BAMG_X_B_ROWPTR: copy_out(lv.B.rp, lv.n + 1, dst, bytes); break;
            case BAMG_X_B_COL: copy_out(lv.B.ci, nnzb, dst, bytes); break;
            case BAMG_X_B_VAL:
                if (l == 0) copy_out((const double*)b0v, nnzb, dst, bytes);
                else copy_out_T(lv.B.v, nnzb, dst, bytes);
                break;
            case BAMG_X_T_ROWPTR: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out(lv.Tm.rp, lv.n + 1, dst, bytes); break;
            case BAMG_X_T_COL: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out(lv.Tm.ci, nnzt, dst, bytes); break;
            case BAMG_X_T_VAL: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out_T(lv.Tm.v, nnzt, dst, bytes); break;
            case BAMG_X_P_COL: if (!lv.pc) fail(BAMG_EINVAL, "no P on the coarsest level"); copy_out(lv.pc, (size_t)lv.n * 4, dst, bytes); break;
            case BAMG_X_P_VAL: if (!lv.pc) fail(BAMG_EINVAL, "no P on the coarsest level"); copy_out_T(lv.pv, (size_t)lv.n * 4, dst, bytes); break;
            case BAMG_X_U: copy_out_T(lv.U, (size_t)lv.n * r, dst, bytes); break;
            case BAMG_X_V: copy_out_T(lv.V, (size_t)lv.n * nv, dst, bytes); break;
            case BAMG_X_LAMBDA: copy_out(lam, 2 * (size_t)nv, dst, bytes); break;
            case BAMG_X_VKIND: copy_out(kind, nv, dst, bytes); break;
            case BAMG_X_X0: if (l != 0) fail(BAMG_EINVAL, "x0 lives on level 0"); copy_out(x0, lv.n, dst, bytes); break;
            case BAMG_X_W: if (!last) fail(BAMG_EINVAL, "W lives on the coarsest level"); copy_out(W, (size_t)nL * nL, dst, bytes); break;
            case BAMG_X_Y: if (!last) fail(BAMG_EINVAL, "y lives on the coarsest level"); copy_out(y, nL, dst, bytes); break;
            case BAMG_X_U0: {
                if (l != 0) fail(BAMG_EINVAL, "U0 lives on level 0");
                T* tmp = sweep_tmp;
                LAUNCH(k_tv_init<T>, nblk((long long)n * r), BAMG_BLK, s, (long long)n * r, o.seed, tmp);
                copy_out_T(tmp, (size_t)n * r, dst, bytes);
                break;
            }
            default: fail(BAMG_EINVAL, "unknown export item %d", what);
        }
    }
};

template <>
void Engine<double>::precondition(const double* v, double* z) {
    auto& l0 = L[0];
    HIPCHK(hipMemcpyAsync(l0.f, v, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    vcycle(0);
    HIPCHK(hipMemcpyAsync(z, l0.e, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
}
template <>
void Engine<float>::precondition(const double* v, double* z) {
    auto& l0 = L[0];
    LAUNCH(k_d2f, nblk(n), BAMG_BLK, s, (int)n, v, l0.f);
    vcycle(0);
    LAUNCH(k_f2d, nblk(n), BAMG_BLK, s, (int)n, (const float*)l0.e, z);
}

}  // namespace

// ------------------------------------------------------------------ C ABI
namespace {
int run_guarded(const std::function<void()>& fn) {
    try {
        fn();
        g_last_error.clear();
        return BAMG_OK;
    } catch (const BamgError& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return BAMG_EDEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return BAMG_EDEVICE;
    }
}
}  // namespace

extern "C" {

void bamg_options_default(bamg_options* opt) {
    if (!opt) return;
    memset(opt, 0, sizeof *opt);
    opt->levels = 0;
    opt->coarse_max = 1024;
    opt->nu_setup = 4;
    opt->nu_pre = 2;
    opt->nu_post = 2;
    opt->omega = 0.7;
    opt->caliber = 4;
    opt->n_eig = 6;
    opt->arnoldi_m = 64;
    opt->gmres_m = 50;
    opt->precision = BAMG_FP64;
    opt->interp = BAMG_INTERP_LS;
    opt->seed = 0;
}

const char* bamg_last_error(void) { return g_last_error.c_str(); }

int bamg_setup(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* val, bamg_grid grid,
               int32_t r, const bamg_options* opt, void* stream, bamg_handle* out) {
    bamg_ctx* ctx = nullptr;
    int rc = run_guarded([&] {
        if (!out) fail(BAMG_EINVAL, "out is NULL");
        *out = nullptr;
        if (!row_ptr || !col_idx || !val) fail(BAMG_EINVAL, "CSR pointer is NULL");
        if (n < 1 || n > (1LL << 30)) fail(BAMG_EINVAL, "n = %lld out of range", (long long)n);
        if (r < 1 || r > 32) fail(BAMG_EINVAL, "r = %d out of range [1, 32]", r);
        if (grid.nx < 1 || grid.ny < 1 || (long long)grid.nx * grid.ny != n)
            fail(BAMG_EINVAL, "grid %dx%d does not match n = %lld", grid.nx, grid.ny, (long long)n);
        if (grid.periodic && (grid.nx < 3 || grid.ny < 3)) fail(BAMG_EUNSUPPORTED, "periodic sides must be >= 3");
        bamg_options o;
        if (opt) o = *opt; else bamg_options_default(&o);
        if (o.nu_setup < 0 || o.nu_pre < 0 || o.nu_post < 0 || !(o.omega > 0) || o.caliber < 1 || o.n_eig < 1 ||
            o.n_eig > 8 || o.gmres_m < 1 || o.gmres_m > 200 || o.arnoldi_m < 1 || o.levels < 0 || o.coarse_max < 1)
            fail(BAMG_EINVAL, "invalid options");
        if (o.interp != BAMG_INTERP_LS) fail(BAMG_EUNSUPPORTED, "interpolation mode %d not available", o.interp);
        if (o.precision == BAMG_FP64) ctx = new Engine<double>();
        else if (o.precision == BAMG_MIXED) ctx = new Engine<float>();
        else fail(BAMG_EINVAL, "unknown precision %d", o.precision);
        ctx->s = (hipStream_t)stream;
        ctx->o = o;
        ctx->r = r;
        ctx->n = n;
        ctx->grid = GridH{grid.nx, grid.ny, grid.periodic ? 1 : 0};
        ctx->setup(row_ptr, col_idx, val);
        *out = ctx;
    });
    if (rc != BAMG_OK) delete ctx;
    return rc;
}

int bamg_solve(bamg_handle h, double* x, double tol, int32_t max_cycles, uint32_t flags, bamg_solve_info* info) {
    int code = BAMG_OK;
    int rc = run_guarded([&] {
        if (!h || !x) fail(BAMG_EINVAL, "NULL handle or x");
        if (!(tol > 0) || max_cycles < 0) fail(BAMG_EINVAL, "invalid tol or max_cycles");
        code = h->solve(x, tol, max_cycles, flags, info);
        if (code == BAMG_ENOCONV) g_last_error = "tolerance not reached";
    });
    if (rc != BAMG_OK) return rc;
    if (code == BAMG_ENOCONV) g_last_error = "tolerance not reached within max_cycles";
    return code;
}

int bamg_free(bamg_handle h) {
    return run_guarded([&] { delete h; });
}

int bamg_get_stats(bamg_handle h, bamg_stats* st) {
    return run_guarded([&] {
        if (!h || !st) fail(BAMG_EINVAL, "NULL argument");
        *st = h->st;
    });
}

int bamg_level_info_get(bamg_handle h, int32_t l, bamg_level_info* out) {
    return run_guarded([&] {
        if (!h || !out) fail(BAMG_EINVAL, "NULL argument");
        h->level_info(l, out);
    });
}

int bamg_export(bamg_handle h, int32_t l, int32_t what, void* dst, size_t bytes) {
    return run_guarded([&] {
        if (!h || !dst) fail(BAMG_EINVAL, "NULL argument");
        h->export_item(l, what, dst, bytes);
    });
}

int bamg_apply_vcycle(bamg_handle h, const double* f, double* e) {
    return run_guarded([&] {
        if (!h || !f || !e) fail(BAMG_EINVAL, "NULL argument");
        h->vcycle_apply(f, e);
    });
}

int bamg_relax(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* val, double* X,
               const double* F, int32_t R, double omega, int32_t nu, void* stream) {
    return run_guarded([&] {
        if (!row_ptr || !col_idx || !val || !X) fail(BAMG_EINVAL, "NULL argument");
        if (n < 1 || R < 1 || (long long)n * R >= (1LL << 31) || nu < 0 || !(omega > 0)) fail(BAMG_EINVAL, "bad sizes");
        hipStream_t s = (hipStream_t)stream;
        Arena A;
        A.s = s;
        struct Rel {
            Arena& A;
            ~Rel() { A.release(); (void)hipStreamSynchronize(A.s); }
        } rel{A};
        int hr[2];
        HIPCHK(hipMemcpyAsync(&hr[0], row_ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hr[1], row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hr[0] != 0 || hr[1] < 0) fail(BAMG_EINVAL, "row_ptr[0] must be 0");
        int N = (int)n;
        // validate as a 1 x n grid would reject wide stencils; relaxation itself
        // needs no grid, so use a grid of one row of n states (every offset is
        // then a b-offset) with the 3x3-box test disabled through n x 1.
        GridDev gd{N, 1, 0, FastDiv(1u)};
        double* colsum = A.alloc<double>(N);
        int* cnt = A.alloc<int>(N);
        int* brp = A.alloc<int>(N + 1);
        int* err = A.alloc<int>(4);
        int* bsum = A.alloc<int>(nblk(N) + 1);
        int* total = A.alloc<int>(2);
        HIPCHK(hipMemsetAsync(colsum, 0, sizeof(double) * N, s));
        HIPCHK(hipMemsetAsync(err, 0, sizeof(int) * 4, s));
        LAUNCH(k_check_a, nblk(N), BAMG_BLK, s, N, row_ptr, col_idx, val, gd, hr[1], colsum, cnt, err);
        LAUNCH(k_check_colsum, nblk(N), BAMG_BLK, s, N, colsum, err);
        int e = 0;
        HIPCHK(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        e &= ~ERR_WIDE;
        if (e & ERR_RANGE) fail(BAMG_EINVAL, "bad CSR");
        if (e & (ERR_NEG | ERR_COLSUM)) fail(BAMG_ENOTSTOCH, "A is not column stochastic");
        int nb = nblk(N);
        LAUNCH(k_scan_block, nb, BAMG_BLK, s, N, (const int*)cnt, brp, bsum);
        LAUNCH(k_scan_sums, 1, BAMG_BLK, s, nb, bsum, total);
        LAUNCH(k_scan_add, nb, BAMG_BLK, s, N, brp, (const int*)bsum, (const int*)total);
        int nnzB = 0;
        HIPCHK(hipMemcpyAsync(&nnzB, brp + N, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int* bci = A.alloc<int>(nnzB);
        double* bv = A.alloc<double>(nnzB);
        double* dinv = A.alloc<double>(N);
        LAUNCH(k_build_b<double>, nb, BAMG_BLK, s, N, row_ptr, col_idx, val, (const int*)brp, bci, bv,
               (double*)nullptr, omega, dinv, (double*)nullptr, err);
        HIPCHK(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (e & ERR_ZERODIAG) fail(BAMG_EZERODIAG, "b_ii <= 0");
        double* tmp = A.alloc<double>((size_t)N * R);
        double* a = X;
        double* b = tmp;
        FastDiv dR((uint32_t)R);
        for (int k = 0; k < nu; ++k) {
            LAUNCH((k_sweep<double, double>), nblk((long long)N * R), BAMG_BLK, s, N, R, dR, (const int*)brp,
                   (const int*)bci, (const double*)bv, (const double*)dinv, (const double*)a, F, b);
            std::swap(a, b);
        }
        if (a != X) HIPCHK(hipMemcpyAsync(X, a, sizeof(double) * N * R, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    });
}

}  // extern "C"
