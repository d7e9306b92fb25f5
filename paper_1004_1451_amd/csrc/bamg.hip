// Host orchestration and C ABI of the Bootstrap AMG library (see bamg.h).
//
// One handle = one hierarchy of one or more chains on one HIP stream.  Several
// chains form one block-diagonal system: on every level the rows of each
// chain are contiguous, the chains ordered by depth (deepest first) so that
// the chains that continue to the next level are always a row prefix.  Every
// phase of the setup and of the cycle is one launch over all chains; the
// per-chain small work (coarsest level, Arnoldi, GMRES scalars) is batched
// over the chains inside its kernels.  The host plans levels, allocates,
// launches, and reads back a few scalars (error flags, the number of coarsest
// eigenvector columns, convergence estimates).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <tuple>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bamg.h"
#include "common.h"
#include "k_coarse.h"
#include "k_cr.h"
#include "k_dense.h"
#include "k_learn.h"
#include "k_mcgs.h"
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

#define LAUNCH(kern, grid, block, s, ...)                                    \
    do {                                                                     \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, __VA_ARGS__); \
        HIPCHK(hipGetLastError());                                           \
    } while (0)

inline int nblk(long long n) { return (int)std::max<long long>(1, (n + BAMG_BLK - 1) / BAMG_BLK); }
// Per-chain reductions split each chain into chunks of SEG_ROWS rows, so that
// a large chain fills the chip and a chain's summation order does not depend
// on the other chains of its batch.
constexpr int SEG_ROWS = 1024;
// The coarsest Arnoldi process stops after ARN_CHECK1 or ARN_CHECK2 steps
// when every wanted Ritz pair's relative residual is at most ARN_TOL there
// (otherwise it runs all its steps).
constexpr int ARN_CHECK1 = 20, ARN_CHECK2 = 30;
constexpr double ARN_TOL = 1e-9;
// Coarse grid levels of at most this many rows take the prolongation and the
// first post-smoothing sweep of the cycle in one pass (measured on the
// hierarchy of the 2048 x 2048 tandem queue: 5.5-5.8 us against 8.0-8.3 us
// for the two launches at 16K and 66K rows, but 11.7 against 8.6 us at 263K
// rows).
constexpr int FUSE_ROWS = 1 << 17;
// The TV-weight and Rayleigh partials do a sparse product per (row, column)
// on top of the sum: shorter chunks keep many workgroups in flight.
constexpr int CN_ROWS = 256;
// Pad (doubles) after each Krylov basis vector.
constexpr int GS_PAD_DEFAULT = 640;   // 5 KiB

// Row stride of the Krylov bases: n rounded up to 256 bytes, plus a pad so
// that the vectors do not all start at the same offset modulo a large power
// of two (the passes read 20 to 50 of them at the same row index, and equal
// offsets fall on the same HBM channel).  BAMG_GS_PAD overrides the pad (in
// doubles, rounded up to a multiple of 32).
static int basis_stride(int n) {
    static const int pad = [] {
        const char* e = std::getenv("BAMG_GS_PAD");
        const int p = e ? std::max(0, std::atoi(e)) : GS_PAD_DEFAULT;
        return (p + 31) / 32 * 32;
    }();
    return (n + 31) / 32 * 32 + pad;
}

// Calls f(std::integral_constant<int, EF>) for the storage a setup kernel
// reads B_l from (EF_CSR, EF_ELL4 or EF_ELL9).
template <typename F>
static void ef_dispatch(int ef, F&& f) {
    if (ef == EF_ELL4) f(std::integral_constant<int, EF_ELL4>{});
    else if (ef == EF_ELL9) f(std::integral_constant<int, EF_ELL9>{});
    else f(std::integral_constant<int, EF_CSR>{});
}

// Calls f(std::integral_constant<int, K>) with K = 1, 2, 4 or the multiple
// of 8 (8 .. 64), the smallest that covers nb finished basis vectors: the
// register width of the Gram-Schmidt passes (their sums do not depend on K).
template <typename F>
static void gs_dispatch(int nb, F&& f) {
    if (nb <= 1) { f(std::integral_constant<int, 1>{}); return; }
    if (nb <= 2) { f(std::integral_constant<int, 2>{}); return; }
    if (nb <= 4) { f(std::integral_constant<int, 4>{}); return; }
    switch ((nb + 7) / 8) {
        case 1: f(std::integral_constant<int, 8>{}); break;
        case 2: f(std::integral_constant<int, 16>{}); break;
        case 3: f(std::integral_constant<int, 24>{}); break;
        case 4: f(std::integral_constant<int, 32>{}); break;
        case 5: f(std::integral_constant<int, 40>{}); break;
        case 6: f(std::integral_constant<int, 48>{}); break;
        case 7: f(std::integral_constant<int, 56>{}); break;
        case 8: f(std::integral_constant<int, 64>{}); break;
        default: throw std::logic_error("Gram-Schmidt basis wider than 64");
    }
}
constexpr int WS = 64;            // stride of the per-chain TV weights
constexpr int KV = 16;            // stride of the per-chain eigen tables
constexpr int SCS = 16;           // stride of the per-chain scalars
constexpr int NS = 4, LSS = 32;   // strides of the Hessenberg selection outputs
constexpr int GT_RCH = 128;       // row chunk of the y^T W partials

struct GridH {
    int nx, ny, periodic;
    long long n() const { return (long long)nx * ny; }
    GridH coarse() const { return {grid_coarse_side(nx, periodic), grid_coarse_side(ny, periodic), periodic}; }
    bool can_coarsen() const {
        if (periodic) return nx % 2 == 0 && ny % 2 == 0 && nx / 2 >= 3 && ny / 2 >= 3;
        return coarse().n() < n();   // a side of one or two points keeps them all
    }
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
// BAMG_POISON=1 in the environment: floating-point allocations start as NaN
// (all bits set) and integer ones as zero, so that a read of memory no kernel
// has written shows up in the results instead of depending on what the
// allocator hands out.
bool poison_enabled() {
    const char* e = getenv("BAMG_POISON");
    return e && e[0] == '1';
}

// Process-wide cache of device buffers, per device, in size classes of a
// sixteenth of an octave (at most 6.25% rounding).  A handle's buffers go
// back to the cache when it is freed (after its stream has drained) and are
// handed to the next request of the same class, so repeated setups make no
// runtime allocation calls.  bamg_trim() returns cached buffers to HIP.
struct DeviceCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void*>> idle;
    static size_t size_class(size_t b) {
        if (b <= 4096) return 4096;
        const int lg = 63 - __builtin_clzll(b);
        const size_t g = size_t(1) << (lg - 4);
        return (b + g - 1) / g * g;
    }
    void* get(int dev, size_t cls) {
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = idle.find({dev, cls});
            if (it != idle.end() && !it->second.empty()) {
                void* p = it->second.back();
                it->second.pop_back();
                return p;
            }
        }
        void* p = nullptr;
        if (hipMalloc(&p, cls) == hipSuccess && p) return p;
        (void)hipGetLastError();
        trim(dev);                                    // give cached memory back and retry once
        p = nullptr;
        if (hipMalloc(&p, cls) == hipSuccess && p) return p;
        (void)hipGetLastError();
        return nullptr;
    }
    void put(int dev, size_t cls, void* p) {
        std::lock_guard<std::mutex> lk(mu);
        idle[{dev, cls}].push_back(p);
    }
    void trim(int dev) {                              // dev < 0: every device
        std::lock_guard<std::mutex> lk(mu);
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto& kv : idle) {
            if (dev >= 0 && kv.first.first != dev) continue;
            if (kv.first.first != cur) (void)hipSetDevice(kv.first.first);
            for (void* p : kv.second) (void)hipFree(p);
            kv.second.clear();
        }
        (void)hipSetDevice(cur);
    }
};

DeviceCache& device_cache() {
    static DeviceCache* c = new DeviceCache();        // lives until the process ends
    return *c;
}

// Autotuned launch shape of the multi-vector sweep: a thread owns VW adjacent
// columns of a row, workgroups of BS threads.  Every variant computes the same
// bits; the fastest for a (device, rows, R, nnz, type) shape is found once per
// process by timing each candidate on the real operator, then reused.
// On an ELL-4 operator a thread may also take two row pieces (rp = 2).
// BAMG_SWEEP_VARIANT="VW,BS[,RP]" in the environment forces a variant.
struct SweepShape { int vw = 1, bs = 256, rp = 1; };

// The tuner also picks the coarse rows per workgroup of the fused Galerkin
// launch (14, 28 or 56) per (device, coarse rows, operator forms, type).
// With BAMG_TUNE_CACHE=<path> the choices persist across processes as one
// JSON object, {"<arch>|<kernel>|<shape ...>": [choice ...], ...}: read at the
// first tuner use, rewritten (through a temporary file) after each new choice.
struct SweepTuner {
    std::mutex mu;
    std::map<std::tuple<int, int, int, int, int>, SweepShape> best;
    std::map<std::tuple<int, int, int, int, int>, int> gal_rows;
    std::map<std::string, std::vector<int>> file;     // entries of the cache file
    bool file_read = false;
    double tune_ms = 0;
};

SweepTuner& sweep_tuner() {
    static SweepTuner* t = new SweepTuner();
    return *t;
}

const char* tune_cache_path() {
    const char* e = getenv("BAMG_TUNE_CACHE");
    return e && *e ? e : nullptr;
}

std::string device_arch(int dev) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Entries of the cache file into tu.file (once per process; caller holds tu.mu).
void tune_cache_read(SweepTuner& tu) {
    if (tu.file_read) return;
    tu.file_read = true;
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = fopen(path, "rb");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, k);
    fclose(f);
    size_t pos = 0;
    while (true) {
        const size_t q0 = txt.find('"', pos);
        if (q0 == std::string::npos) break;
        const size_t q1 = txt.find('"', q0 + 1);
        const size_t b0 = q1 == std::string::npos ? q1 : txt.find('[', q1);
        const size_t b1 = b0 == std::string::npos ? b0 : txt.find(']', b0);
        if (b1 == std::string::npos) break;
        std::vector<int> v;
        const char* p = txt.c_str() + b0 + 1;
        const char* end = txt.c_str() + b1;
        while (p < end) {
            char* nx = nullptr;
            const long x = strtol(p, &nx, 10);
            if (nx == p) { ++p; continue; }
            v.push_back((int)x);
            p = nx;
        }
        tu.file[txt.substr(q0 + 1, q1 - q0 - 1)] = v;
        pos = b1 + 1;
    }
}

// Rewrite the cache file with tu.file (caller holds tu.mu); failures to
// write only lose the cache.
void tune_cache_write(const SweepTuner& tu) {
    const char* path = tune_cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    fputs("{", f);
    bool first = true;
    for (const auto& kv : tu.file) {
        fprintf(f, "%s\n  \"%s\": [", first ? "" : ",", kv.first.c_str());
        for (size_t i = 0; i < kv.second.size(); ++i) fprintf(f, "%s%d", i ? ", " : "", kv.second[i]);
        fputs("]", f);
        first = false;
    }
    fputs("\n}\n", f);
    const bool ok = fclose(f) == 0;
    if (ok) (void)rename(tmp.c_str(), path);
}

std::string tune_key(int dev, const char* kernel, std::initializer_list<long long> shape) {
    std::string k = device_arch(dev) + "|" + kernel;
    for (long long x : shape) k += "|" + std::to_string(x);
    return k;
}

bool forced_sweep_shape(int R, SweepShape& out) {
    const char* e = getenv("BAMG_SWEEP_VARIANT");
    if (!e || !*e) return false;
    int vw = 0, bs = 0, rp = 1;
    if (sscanf(e, "%d,%d,%d", &vw, &bs, &rp) < 2) return false;
    if ((vw != 1 && vw != 2 && vw != 3 && vw != 4 && vw != 6 && vw != 12) || (bs != 128 && bs != 256 && bs != 512) ||
        ((vw == 3 || vw > 4) && bs > 256) || R % vw || (rp != 1 && rp != 2) ||
        (rp == 2 && ((vw != 2 && vw != 4) || bs == 128)))
        return false;
    out.vw = vw;
    out.bs = bs;
    out.rp = rp;
    return true;
}

// HIP events are reused process-wide (per device): creating one costs host
// time that would otherwise show as idle GPU time between launches.
struct EventPool {
    std::mutex mu;
    std::map<int, std::vector<hipEvent_t>> free;
    hipEvent_t get() {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        {
            std::lock_guard<std::mutex> lk(mu);
            auto& v = free[dev];
            if (!v.empty()) {
                hipEvent_t e = v.back();
                v.pop_back();
                return e;
            }
        }
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        return e;
    }
    void put(hipEvent_t e) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) { (void)hipEventDestroy(e); return; }
        std::lock_guard<std::mutex> lk(mu);
        free[dev].push_back(e);
    }
};
EventPool& event_pool() {
    static EventPool* p = new EventPool();   // never destroyed: outlives every handle
    return *p;
}

struct Arena {
    hipStream_t s = nullptr;
    size_t bytes = 0, budget = 0;
    bool poison = poison_enabled();
    int dev = -1;
    struct Buf { void* p; size_t cls; };
    std::vector<Buf> bufs;
    template <typename X>
    X* alloc(size_t count) {
        if (dev < 0) HIPCHK(hipGetDevice(&dev));
        const size_t cls = DeviceCache::size_class(std::max<size_t>(count, 1) * sizeof(X));
        if (budget && bytes + cls > budget) fail(BAMG_ENOMEM, "memory budget of %zu bytes exceeded", budget);
        void* p = device_cache().get(dev, cls);
        if (!p) fail(BAMG_ENOMEM, "device allocation of %zu bytes failed", cls);
        bytes += cls;
        bufs.push_back({p, cls});
        if (poison) HIPCHK(hipMemsetAsync(p, std::is_floating_point<X>::value ? 0xFF : 0x00, cls, s));
        return (X*)p;
    }
    template <typename X>
    X* upload(const std::vector<X>& v) {
        X* p = alloc<X>(v.size());
        if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), sizeof(X) * v.size(), hipMemcpyHostToDevice, s));
        return p;
    }
    // Drain the stream, then hand every buffer back to the cache.
    void release() {
        if (!bufs.empty()) (void)hipStreamSynchronize(s);
        for (auto& b : bufs) device_cache().put(dev, b.cls, b.p);
        bufs.clear();
        bytes = 0;
    }
};

template <typename T>
struct Csr {
    int cap = 0;
    int* rp = nullptr;
    int* ci = nullptr;
    T* v = nullptr;
    int* eci = nullptr;              // ELL-4 copy (rows of at most 4 entries), or null
    T* ev = nullptr;
    int* cci = nullptr;              // column-major ELL-9 copy (coarse grid levels) the kernels
    T* cv = nullptr;                 // read, or null (BAMG_SWEEP_ELL=0)
    int cld = 0;                     // its stride (the level's rows)
    int* gci = nullptr;              // the ELL-9 arrays the Galerkin product writes
    T* gv = nullptr;                 // (coarse grid levels; cci / cv alias them)
};

// Rows of one level: all present chains, continuing chains first.
template <typename T>
struct Level {
    int nch = 0, ncont = 0;          // present chains, chains with a next level
    int segp = 1;                    // reduction chunks of its largest chain
    int cnp = 1;                     // CN_ROWS chunks of its largest chain
    int rows = 0, cont_rows = 0;     // all rows, rows of continuing chains
    std::vector<ChainGeo> geo;       // host copy
    ChainGeo* dgeo = nullptr;        // device copy
    Csr<T> B, Tm;                    // Tm.rp == nullptr: T = I (finest level)
    T* dinv = nullptr;
    int* pc = nullptr;               // P: cont_rows x 4 (ELL)
    T* pv = nullptr;
    int* qc = nullptr;               // Q: next level rows x 9 (ELL)
    T* qv = nullptr;
    T* U = nullptr;                  // rows x r relaxed test vectors
    T* V = nullptr;                  // rows x VS eigenvector approximations
    T *e = nullptr, *e2 = nullptr, *f = nullptr, *r = nullptr;   // cycle vectors
    unsigned short* qmask = nullptr; // Q's box slots per next-level row (cycle restriction)
    unsigned char* jcnt = nullptr;   // |J_i| per continuing row
    float* feat = nullptr;           // collected first-pass features (rows x 24)
    float* slotw = nullptr;          // collected final slot weights (rows x 4)
    float* slotw0 = nullptr;         // collected first-pass slot weights (rows x 4)
    int* cnt = nullptr;
    int* cnt2 = nullptr;             // entries per coarse row of T_{l+1} (grid levels)
    bool zero_into_e2 = false;       // first smoothing sweep target (fixed buffers)
    // levels without a grid (compatible relaxation)
    bool decided = false;            // coarsening fixed (on the first pass)
    int* cmap = nullptr;             // coarse index per row, -1 on F
    int *qrp = nullptr, *qci = nullptr;   // Q: CSR over the next level's rows
    T* qvv = nullptr;
    int cr_rounds = 0;
    std::vector<double> cr_rho;      // CR estimate of every relaxation round
};

struct ChainH {
    int uidx = 0;                    // caller's index
    long long uoff = 0, n = 0;       // caller's row offset and size
    GridH grid{};
    std::vector<GridH> plan;
};

}  // namespace

// ------------------------------------------------------------------ context
// ------------------------------------------------------------------ network files
// The learned form's parameters on disk: the 8 bytes "BAMGMLP1", the count
// (int32, BAMG_MLP_NPARAM), then the FP32 values in parameter order.
constexpr float MLP_FEATURE_CAP = 16.0f, MLP_TARGET_CAP = 1.0f;

void write_mlp_file(const char* path, const std::vector<float>& p) {
    FILE* f = std::fopen(path, "wb");
    if (!f) fail(BAMG_EINVAL, "cannot open %s for writing", path);
    const int32_t cnt = (int32_t)p.size();
    bool ok = std::fwrite("BAMGMLP1", 1, 8, f) == 8 && std::fwrite(&cnt, sizeof(cnt), 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) fail(BAMG_EINVAL, "writing %s failed", path);
}

std::vector<float> read_mlp_file(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) fail(BAMG_EINVAL, "cannot open network file %s", path);
    char magic[8];
    int32_t cnt = 0;
    std::vector<float> p(MLP_NPARAM);
    const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "BAMGMLP1", 8) == 0 &&
                    std::fread(&cnt, sizeof(cnt), 1, f) == 1 && cnt == MLP_NPARAM &&
                    std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    std::fclose(f);
    if (!ok) fail(BAMG_EINVAL, "%s is not a network file of %d parameters", path, MLP_NPARAM);
    return p;
}

struct bamg_ctx {
    virtual ~bamg_ctx() {}
    virtual void setup(const int32_t* rp, const int32_t* ci, const double* val) = 0;
    virtual int solve(double* x, double tol, int max_cycles, uint32_t flags, int32_t* status, double* resid,
                      bamg_solve_info* info) = 0;
    virtual void level_info(int l, bamg_level_info* out) = 0;
    virtual void export_item(int l, int what, void* dst, size_t bytes) = 0;
    virtual void vcycle_apply(const double* f, double* e) = 0;
    virtual int mle_iterate(double* x, double tol, int max_cycles, bamg_solve_info* info) = 0;
    virtual long long collect_pairs(float* F, float* Tg, long long cap, float fcap, float tcap) = 0;
    hipStream_t s = nullptr;
    bamg_options o{};
    bamg_stats st{};
    int r = 0;
    int nch = 1;
    long long n = 0;
    std::vector<ChainH> chains;      // internal (depth-sorted) order
};

namespace {

template <typename T>
struct Engine : bamg_ctx {
    static constexpr bool MIXED = sizeof(T) == 4;
    Arena A;
    std::vector<Level<T>> L;
    int VS = 8;                      // row stride of the eigenvector blocks (a multiple of 4)
    int ncol = 4;                    // colours of the multicolour Gauss-Seidel sweeps
    bool mcgs = false;
    bool unstructured = false;       // no grid: compatible relaxation coarsens every level
    // compatible-relaxation work arrays (level-0 sized)
    int *cr_st = nullptr, *cr_isc = nullptr, *cr_cand = nullptr, *cr_pos = nullptr, *cr_flag = nullptr;
    double *cr_u0 = nullptr, *cr_ua = nullptr, *cr_ub = nullptr, *cr_part = nullptr, *cr_out = nullptr;
    Csr<T> Wt;                       // M P of the Galerkin products without a grid
    // finest level in FP64 for the outer iteration
    int* b0rp = nullptr;
    int* b0ci = nullptr;
    double* b0v = nullptr;
    double* b0ev = nullptr;          // FP64 values of the ELL-4 copy of B_0 (columns in L[0].B.eci)
    int nnz0 = 0;
    bool reordered = false;
    int *perm_src = nullptr, *perm_dst = nullptr, *perm_len = nullptr;   // caller -> internal
    // coarsest levels (one per chain)
    std::vector<CoarseDesc> cdh;
    CoarseDesc* cd = nullptr;
    // Descriptors the block path runs on: cdh, except that the coarsest grid
    // of a single chain with rows of GJ_NB + 1 points (bordered) is replaced
    // by its main part (k_bd_* in k_coarse.h).
    std::vector<CoarseDesc> cdsh;
    CoarseDesc* cds = nullptr;
    bool bordered = false;
    double *bdZ = nullptr, *bdY = nullptr, *bdG = nullptr, *bdH = nullptr, *bdS = nullptr;
    int NVt = 0;                     // sum of coarsest sizes
    int AMmax = 0, maxnL = 0, nxmax = 0;
    double *Wp = nullptr, *Fp = nullptr, *ypool = nullptr, *cpool = nullptr, *bcolp = nullptr, *t1 = nullptr,
           *t2 = nullptr, *rre = nullptr, *rim = nullptr, *gtpart = nullptr;
    float* Wfp = nullptr;
    double *dcP = nullptr, *dcR = nullptr, *dcmp = nullptr, *apart = nullptr, *arn_u = nullptr;
    double *scale = nullptr, *minpiv = nullptr, *cy = nullptr, *csc = nullptr, *dots = nullptr, *vyb = nullptr,
           *npart = nullptr;
    double *Vb = nullptr, *Hh = nullptr, *sel_lam = nullptr, *sel_s = nullptr;
    int* nsel = nullptr;
    int HS = 1, SS = 1, DS = 1;
    bool dense_fallback = false;
    // eigen tables
    double* lam = nullptr;
    int *kind = nullptr, *ent_col = nullptr, *nvc = nullptr, *nentc = nullptr;
    std::vector<int> nvc_h;
    int nvmax = 1;
    double* x0 = nullptr;
    // reductions / scalars
    double* part = nullptr;
    double* sc = nullptr;            // nch x SCS per-chain scalars
    double* wts = nullptr;           // nch x WS TV weights
    int* err = nullptr;
    int* derr = nullptr;             // error flags checked once, at the end of the setup
    int* gath = nullptr;             // scalars gathered for one read-back
    int *itmp = nullptr, *bsum = nullptr, *total = nullptr;
    T* sweep_tmp = nullptr;
    // FGMRES
    int m_alloc = 0;
    double *hbuf2 = nullptr, *gsaux = nullptr, *gscoef = nullptr;
    int vld = 0;   // row stride of the Krylov bases Vk, Zk (n rounded up, plus a pad)
    double *Vk = nullptr, *Zk = nullptr, *wk = nullptr, *Hg = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
           *ysol = nullptr, *hbuf = nullptr, *rvec = nullptr, *est = nullptr, *xperm = nullptr;
    int *act = nullptr, *kd = nullptr;
    int* cmask = nullptr;            // chains the cycle works on (all ones outside solve)
    int* hfail = nullptr;
    double *vin = nullptr, *vout = nullptr;   // permuted vectors of bamg_apply_vcycle
    // graph of one cycle on fixed buffers
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_s = nullptr;     // capture needs a stream other than the legacy default one
    bool pivot_pending = false;      // the last coarsest inverse's pivot not yet checked
    int arn_used = 1 << 30;          // Arnoldi steps the last coarsest eigenpairs came from (cap)
    bool cycle_decided = false, use_graph = false;
    // learned form
    MlpPack* mlp_pk = nullptr;
    float* learn_part = nullptr;
    double* learn_acc = nullptr;
    int learn_grid = 0;
    // profiling
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_sweep, ev_gal, ev_ls, ev_gj, ev_gal_csr, ev_ls2;
    double gj_flops = 0;             // flops of the profiled dense updates
    // FGMRES: chain flags after each Arnoldi step, read by the host one step
    // late (pinned, two slots), the events that mark them, the inner
    // tolerances on the device, and a row of ones to restore the cycle mask
    int* hflag = nullptr;
    hipEvent_t fev[2] = {nullptr, nullptr};
    double* itol_d = nullptr;
    int* ones_d = nullptr;

    ~Engine() override {
        if (hflag) (void)hipHostFree(hflag);
        for (hipEvent_t e : fev)
            if (e) event_pool().put(e);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_s) (void)hipStreamDestroy(cap_s);
        for (auto* v : {&ev_sweep, &ev_gal, &ev_ls, &ev_gj, &ev_gal_csr, &ev_ls2})
            for (auto& p : *v) { event_pool().put(p.first); event_pool().put(p.second); }
        A.release();
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
    template <typename X>
    std::vector<X> getn(const X* p, size_t cnt) {
        std::vector<X> v(cnt);
        if (cnt) HIPCHK(hipMemcpyAsync(v.data(), p, sizeof(X) * cnt, hipMemcpyDeviceToHost, s));
        sync();
        return v;
    }
    void zero(void* p, size_t bytes) { HIPCHK(hipMemsetAsync(p, 0, bytes, s)); }

    void scan(int cnt_n, const int* cnt, int* out) {
        int nb = nblk(cnt_n);
        LAUNCH(k_scan_block, nb, BAMG_BLK, s, cnt_n, cnt, out, bsum);
        LAUNCH(k_scan_sums, 1, BAMG_BLK, s, nb, bsum, total);
        LAUNCH(k_scan_add, nb, BAMG_BLK, s, cnt_n, out, bsum, total);
    }

    // per-chain reduction over the finest rows -> out[c * SCS]
    template <int OP>
    void seg_reduce(const double* a, const double* b, double* out) {
        const int P = L[0].segp;
        dim3 grid(P, nch);
        hipLaunchKernelGGL(k_seg_reduce_partial<OP>, grid, dim3(BAMG_BLK), 0, s, (const ChainGeo*)L[0].dgeo, SEG_ROWS,
                           a, b, part);
        HIPCHK(hipGetLastError());
        LAUNCH(k_seg_reduce_final, nch, BAMG_BLK, s, (const ChainGeo*)L[0].dgeo, SEG_ROWS, P, (const double*)part,
               out, SCS);
    }

    std::pair<hipEvent_t, hipEvent_t> ev_begin() {
        std::pair<hipEvent_t, hipEvent_t> p;
        p.first = event_pool().get();
        p.second = event_pool().get();
        HIPCHK(hipEventRecord(p.first, s));
        return p;
    }
    void ev_end(std::pair<hipEvent_t, hipEvent_t> p, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
        HIPCHK(hipEventRecord(p.second, s));
        v.push_back(p);
    }

    // -------------------------------------------------------------- planning
    void plan_levels() {
        int depth = 0;
        for (auto& c : chains) depth = std::max(depth, (int)c.plan.size());
        L.resize(depth);
        for (int l = 0; l < depth; ++l) {
            auto& lv = L[l];
            int off = 0;
            for (int c = 0; c < nch; ++c) {
                auto& ch = chains[c];
                if ((int)ch.plan.size() <= l) break;     // depth-sorted: the rest are shorter
                ChainGeo gg{};
                const GridH& gh = ch.plan[l];
                gg.off = off; gg.n = (int)gh.n();
                gg.nx = gh.nx; gg.ny = gh.ny; gg.periodic = gh.periodic; gg.dy = FastDiv((uint32_t)gh.ny);
                if (unstructured) { gg.nx = 0; gg.ny = 1; gg.dy = FastDiv(1u); }     // no grid
                if ((int)ch.plan.size() > l + 1) {
                    const GridH& gc = ch.plan[l + 1];
                    gg.cn = (int)gc.n(); gg.ncx = gc.nx; gg.ncy = gc.ny; gg.dcy = FastDiv((uint32_t)gc.ny);
                    ++lv.ncont;
                } else {
                    gg.cn = 0; gg.ncx = 1; gg.ncy = 1; gg.dcy = FastDiv(1u);
                }
                lv.geo.push_back(gg);
                off += gg.n;
            }
            lv.nch = (int)lv.geo.size();
            for (auto& gg : lv.geo) {
                lv.segp = std::max(lv.segp, ceil_div(gg.n, SEG_ROWS));
                lv.cnp = std::max(lv.cnp, ceil_div(gg.n, CN_ROWS));
            }
            lv.rows = off;
            lv.cont_rows = lv.ncont < lv.nch ? lv.geo[lv.ncont].off : off;
        }
        for (int l = 0; l + 1 < depth; ++l)
            for (int c = 0; c < L[l].ncont; ++c) L[l].geo[c].coff = L[l + 1].geo[c].off;
        mcgs = o.relax == BAMG_RELAX_MCGS;
        ncol = 1;
        for (auto& lv : L)
            for (auto& gg : lv.geo) ncol = std::max(ncol, dir_colours(gg.nx, gg.periodic) * dir_colours(gg.ny, gg.periodic));
        // fixed buffers of the cycle: the first smoothing sweep writes where the
        // parity of the remaining sweeps leaves the result in e
        for (auto& lv : L) {
            int flips = std::max(0, o.nu_pre - 1) + o.nu_post;
            lv.zero_into_e2 = (flips % 2) == 1;
        }
    }

    void allocate(int nnzA) {
        const int depth = (int)L.size();
        VS = (std::max(1, o.n_eig) + 1 + 3) / 4 * 4;     // padded for 16-byte row moves
        for (int l = 0; l < depth; ++l) {
            alloc_level(l, nnzA);
            if (L[l].ncont > 0) alloc_cont(l);
        }
        alloc_globals();
        // without a grid the depth and the coarsest size are known only once
        // compatible relaxation has coarsened every level
        if (!unstructured) alloc_coarsest();
    }

    // Rows, operators (grid levels: 9 entries per row reserved; levels
    // without a grid: allocated by their Galerkin product), vectors of level l.
    void alloc_level(int l, int nnzA) {
        auto& lv = L[l];
        const int n_l = lv.rows;
        lv.dgeo = A.upload(lv.geo);
        if (l == 0) {
            lv.B.cap = nnzA + n_l;
        } else {
            lv.B.cap = unstructured ? 0 : 9 * n_l;
            lv.Tm.cap = unstructured ? 0 : 9 * n_l;
            lv.Tm.rp = A.alloc<int>(n_l + 1);
            if (lv.Tm.cap) {
                lv.Tm.ci = A.alloc<int>(lv.Tm.cap);
                lv.Tm.v = A.alloc<T>(lv.Tm.cap);
            }
        }
        lv.B.rp = A.alloc<int>(n_l + 1);
        if (lv.B.cap) {
            lv.B.ci = A.alloc<int>(lv.B.cap);
            lv.B.v = A.alloc<T>(lv.B.cap);
        }
        if (l > 0 && !unstructured) {
            for (Csr<T>* M : {&lv.B, &lv.Tm}) {
                M->gci = A.alloc<int>((size_t)n_l * 9);
                M->gv = A.alloc<T>((size_t)n_l * 9);
                M->cld = n_l;
                if (ell9_on()) { M->cci = M->gci; M->cv = M->gv; }
            }
        }
        lv.dinv = A.alloc<T>(n_l);
        lv.U = A.alloc<T>((size_t)n_l * r);
        lv.V = A.alloc<T>((size_t)n_l * VS);
        zero(lv.V, sizeof(T) * (size_t)n_l * VS);
        lv.e = A.alloc<T>(n_l);
        lv.e2 = A.alloc<T>(n_l);
        lv.f = A.alloc<T>(n_l);
        lv.r = A.alloc<T>(n_l);
    }

    // P, Q and the per-row work arrays of a level that has a next level.
    void alloc_cont(int l) {
        auto& lv = L[l];
        const int nc = L[l + 1].rows;
        lv.pc = A.alloc<int>((size_t)lv.cont_rows * 4);
        lv.pv = A.alloc<T>((size_t)lv.cont_rows * 4);
        lv.jcnt = A.alloc<unsigned char>(lv.cont_rows);
        lv.cnt = A.alloc<int>(nc + 1);
        if (unstructured) {
            lv.qrp = A.alloc<int>(nc + 1);
            lv.qci = A.alloc<int>((size_t)lv.cont_rows * 4);
            lv.qvv = A.alloc<T>((size_t)lv.cont_rows * 4);
            return;
        }
        lv.qc = A.alloc<int>((size_t)nc * 9);
        lv.qv = A.alloc<T>((size_t)nc * 9);
        lv.cnt2 = A.alloc<int>(nc + 1);
        lv.qmask = A.alloc<unsigned short>(nc);
        if (o.collect) {
            lv.feat = A.alloc<float>((size_t)lv.cont_rows * 24);
            lv.slotw = A.alloc<float>((size_t)lv.cont_rows * 4);
            lv.slotw0 = A.alloc<float>((size_t)lv.cont_rows * 4);
        }
    }

    void alloc_globals() {
        if (MIXED) {
            // the FP32 and FP64 forms of B_0 share one structure
            b0rp = L[0].B.rp;
            b0ci = L[0].B.ci;
            b0v = A.alloc<double>(L[0].B.cap);
        } else {
            b0rp = L[0].B.rp;
            b0ci = L[0].B.ci;
            b0v = (double*)L[0].B.v;
        }
        if (o.interp == BAMG_INTERP_MLP) {
            mlp_pk = A.alloc<MlpPack>(1);
            const float* wts_in = o.mlp_weights;
            if (!wts_in) wts_in = A.upload(read_mlp_file(o.mlp_weights_path));
            LAUNCH(k_mlp_pack, 16, BAMG_BLK, s, wts_in, mlp_pk);
            learn_grid = std::min(1024, nblk(L[0].cont_rows));
            learn_part = A.alloc<float>(2 * (size_t)learn_grid);
            learn_acc = A.alloc<double>(2);
            zero(learn_acc, 2 * sizeof(double));
        }
        lam = A.alloc<double>((size_t)nch * 2 * KV);
        kind = A.alloc<int>((size_t)nch * KV);
        ent_col = A.alloc<int>((size_t)nch * KV);
        nvc = A.alloc<int>(nch);
        nentc = A.alloc<int>(nch);
        zero(nvc, sizeof(int) * nch);
        zero(lam, sizeof(double) * nch * 2 * KV);
        zero(kind, sizeof(int) * nch * KV);
        zero(ent_col, sizeof(int) * nch * KV);
        x0 = A.alloc<double>(n);
        cmask = A.upload(std::vector<int>(nch, 1));
        ones_d = A.upload(std::vector<int>(nch, 1));
        {
            const size_t P = L[0].segp;
            size_t need = 4096;
            const size_t PC = L[0].cnp;
            need = std::max(need, (size_t)nch * PC * 2 * WS);
            need = std::max(need, (size_t)nch * PC * KV * 4);
            need = std::max(need, (size_t)nch * P * (BAMG_BLK / BAMG_WAVE) * (o.gmres_m + 2));
            need = std::max(need, (size_t)nch * 64);
            part = A.alloc<double>(need);
        }
        sc = A.alloc<double>((size_t)nch * SCS);
        wts = A.alloc<double>((size_t)nch * WS);
        err = A.alloc<int>(4);
        derr = A.alloc<int>(1);
        zero(derr, sizeof(int));
        gath = A.alloc<int>(72);
        itmp = A.alloc<int>(n + 1);
        bsum = A.alloc<int>(nblk(n) + 1);
        total = A.alloc<int>(4);
        sweep_tmp = A.alloc<T>((size_t)n * std::max(r, VS));
        if (unstructured) {
            for (int** p : {&cr_st, &cr_isc, &cr_cand}) *p = A.alloc<int>(n);
            cr_pos = A.alloc<int>(n + 1);
            cr_flag = A.alloc<int>(8);
            for (double** p : {&cr_u0, &cr_ua, &cr_ub}) *p = A.alloc<double>(n);
            cr_part = A.alloc<double>(2 * (size_t)CR_RED_BLOCKS);
            cr_out = A.alloc<double>(2);
            Wt.rp = A.alloc<int>(n + 1);
        }
    }

    // Coarsest descriptors (chain c's coarsest level is its last plan entry)
    // and the pools of the coarsest pseudo-inverse and eigensolve.
    void alloc_coarsest() {
        long long woff = 0, boff = 0, aoff = 0, wfoff = 0;
        int voff = 0;
        AMmax = 0; maxnL = 0; nxmax = 0;
        dense_fallback = false;
        bordered = false;
        cdh.clear();
        for (int c = 0; c < nch; ++c) {
            const auto& ch = chains[c];
            const int lc = (int)ch.plan.size() - 1;
            const GridH& gh = ch.plan[lc];
            CoarseDesc d{};
            if (unstructured) {
                // no grid: the dense inverse
                d.n = L[lc].rows; d.nx = 0; d.ny = 0; d.periodic = 0; d.dy = FastDiv(1u);
                dense_fallback = true;
            } else {
                d.n = (int)gh.n(); d.nx = gh.nx; d.ny = gh.ny; d.periodic = gh.periodic; d.dy = FastDiv((uint32_t)gh.ny);
                if (gh.ny > GJ_NB || gh.nx > CZ_MAX_NX) {
                    if (nch == 1 && !gh.periodic && gh.ny == GJ_NB + 1 && gh.nx <= GJ_NB + 1) bordered = true;
                    else dense_fallback = true;
                }
            }
            d.row0 = L[lc].geo[c].off;
            d.voff = voff;
            d.woff = woff;
            d.soff = woff;
            d.sld = d.n;
            d.bord = 0;
            d.boff = boff;
            d.aoff = aoff;
            d.wfld = (d.n + 3) & ~3;
            d.wfoff = wfoff;
            wfoff += (long long)d.n * d.wfld;
            d.am = (o.n_eig > 1) ? std::max(0, std::min({o.arnoldi_m, d.n - 1, HQR_MAXM})) : 0;
            d.brp = L[lc].B.rp; d.bci = L[lc].B.ci; d.bv = L[lc].B.v;
            d.trp = L[lc].Tm.rp; d.tci = L[lc].Tm.ci; d.tv = L[lc].Tm.v;
            voff += d.n;
            woff += (long long)d.n * d.n;
            boff += 5LL * d.nx * d.ny * d.ny;
            aoff += (long long)d.n * (d.am + 1);
            AMmax = std::max(AMmax, d.am);
            maxnL = std::max(maxnL, d.n);
            nxmax = std::max(nxmax, d.nx);
            cdh.push_back(d);
        }
        if (dense_fallback && nch > 1)
            fail(BAMG_EUNSUPPORTED, "batched chains need coarsest grids with ny <= %d and nx <= %d", GJ_NB, CZ_MAX_NX);
        NVt = voff;
        cd = A.upload(cdh);
        cdsh = cdh;
        long long wall = woff;
        if (bordered) {
            CoarseDesc& m = cdsh[0];
            m.ny = GJ_NB;
            m.n = m.nx * GJ_NB;
            m.dy = FastDiv((uint32_t)GJ_NB);
            m.woff = woff;              // A^-1 of the main part, after the chain's W
            m.bord = 1;
            wall += (long long)m.n * m.n;
            const size_t zs = (size_t)m.n * GJ_NB;
            for (double** p : {&bdZ, &bdY, &bdG, &bdH}) *p = A.alloc<double>(zs);
            bdS = A.alloc<double>((size_t)GJ_NB * GJ_NB);
        }
        cds = A.upload(cdsh);
        Wp = A.alloc<double>(wall);
        if (MIXED) Wfp = A.alloc<float>(std::max<long long>(wfoff, 1));
        Fp = A.alloc<double>(std::max<long long>(boff, 1));
        for (double** p : {&ypool, &cpool, &bcolp, &t1, &t2, &rre, &rim}) *p = A.alloc<double>(NVt);
        gtpart = A.alloc<double>((size_t)ceil_div(maxnL, GT_RCH) * NVt);
        scale = A.alloc<double>(nch);
        minpiv = A.alloc<double>(nch);
        // divide and conquer: left and right panels, pivot partials
        dcP = A.alloc<double>((size_t)NVt * 2 * GJ_NB);
        dcR = A.alloc<double>((size_t)NVt * GJ_NB);
        dcmp = A.alloc<double>((size_t)nch * DC_MP);
        cy = A.alloc<double>(nch);
        csc = A.alloc<double>((size_t)nch * SCS);
        const int am = std::max(1, AMmax);
        HS = (am + 1) * am;
        SS = 16 * 2 * am;
        DS = am + 2;
        Vb = A.alloc<double>(std::max<long long>(aoff, 1));
        Hh = A.alloc<double>((size_t)nch * HS);
        sel_lam = A.alloc<double>((size_t)nch * LSS);
        sel_s = A.alloc<double>((size_t)nch * SS);
        nsel = A.alloc<int>((size_t)nch * NS);
        dots = A.alloc<double>((size_t)nch * DS);
        vyb = A.alloc<double>((size_t)nch * DS);
        npart = A.alloc<double>((size_t)nch * nblk(std::max(1, maxnL)) * 2);
        apart = A.alloc<double>((size_t)nch * DS * nblk(std::max(1, maxnL)));
        arn_u = A.alloc<double>(std::max(1, NVt));
    }

    // The coarsest descriptors after the coarsest operators moved (a level
    // without a grid reallocates a product that outgrew its arrays).
    void refresh_coarse_desc() {
        if (cdh.empty()) return;
        for (int c = 0; c < nch; ++c) {
            const int lc = (int)chains[c].plan.size() - 1;
            auto& d = cdh[c];
            d.brp = L[lc].B.rp; d.bci = L[lc].B.ci; d.bv = L[lc].B.v;
            d.trp = L[lc].Tm.rp; d.tci = L[lc].Tm.ci; d.tv = L[lc].Tm.v;
            auto& m = cdsh[c];
            m.brp = d.brp; m.bci = d.bci; m.bv = d.bv;
            m.trp = d.trp; m.tci = d.tci; m.tv = d.tv;
        }
        HIPCHK(hipMemcpyAsync(cd, cdh.data(), sizeof(CoarseDesc) * cdh.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(cds, cdsh.data(), sizeof(CoarseDesc) * cdsh.size(), hipMemcpyHostToDevice, s));
        sync();
    }

    // Validate A and build B = I - A on the finest level.
    void build_b0(const int32_t* rp, const int32_t* ci, const double* val, int nnzA) {
        auto& lv = L[0];
        double* colsum = A.alloc<double>(n);
        zero(colsum, sizeof(double) * n);
        zero(err, sizeof(int) * 4);
        LAUNCH(k_check_a, nblk(n), BAMG_BLK, s, (int)n, rp, ci, val, (const ChainGeo*)lv.dgeo, lv.nch, nnzA, colsum,
               itmp, err);
        LAUNCH(k_check_colsum, nblk(n), BAMG_BLK, s, (int)n, colsum, err);
        // the row counts are scanned before the flags are read (a scan of
        // counts touches no memory they index), so one read-back brings both
        // the flags and nnz(B_0)
        scan((int)n, itmp, b0rp);
        LAUNCH(k_copy_int, 1, BAMG_WAVE, s, (const int*)(b0rp + n), err + 1);
        const std::vector<int> chk = getn(err, 2);
        const int e = chk[0];
        if (e & ERR_RANGE)
            fail(BAMG_EINVAL, "CSR of A: row_ptr not monotone, column out of range or outside its chain, or columns "
                              "not strictly ascending");
        if (e & ERR_NEG) fail(BAMG_ENOTSTOCH, "A has a negative, non-finite or > 1 entry");
        if (e & ERR_COLSUM) fail(BAMG_ENOTSTOCH, "a column of A does not sum to 1 within 1e-12");
        if (e & ERR_WIDE) fail(BAMG_EUNSUPPORTED, "A joins states farther apart than the 3x3 grid box");
        nnz0 = chk[1];
        // the ELL-4 copy of B_0 (and of its FP64 values in the mixed form)
        // for the level-0 sweeps, the cycle's level-0 residual and the outer
        // SpMV, written by the same pass when every row may have at most 4
        // entries (BAMG_SWEEP_ELL=0 turns it off)
        const char* ee = getenv("BAMG_SWEEP_ELL");
        const bool ell = !(ee && ee[0] == '0') && nnz0 <= 4LL * lv.rows;
        int* eci = ell ? A.alloc<int>((size_t)lv.rows * 4) : nullptr;
        T* ev = ell ? A.alloc<T>((size_t)lv.rows * 4) : nullptr;
        double* ev64 = ell ? (MIXED ? A.alloc<double>((size_t)lv.rows * 4) : (double*)ev) : nullptr;
        T* lo = MIXED ? lv.B.v : nullptr;
        T* dlo = MIXED ? lv.dinv : nullptr;
        double* dinv64 = MIXED ? A.alloc<double>(n) : (double*)lv.dinv;
        zero(err, sizeof(int) * 4);
        LAUNCH(k_build_b<T>, nblk(n), BAMG_BLK, s, (int)n, rp, ci, val, b0rp, b0ci, b0v, lo, o.omega, dinv64, dlo, eci,
               MIXED ? ev : (T*)nullptr, ev64, err);
        const int e2 = get1(err);
        if (e2 & ERR_ZERODIAG) fail(BAMG_EZERODIAG, "b_ii <= 0 on the finest level");
        if (ell && !(e2 & ERR_ELL)) {
            lv.B.eci = eci;
            lv.B.ev = ev;
            b0ev = ev64;
        }
    }

    // -------------------------------------------------------------- setup steps
    // nu homogeneous sweeps on the continuing rows of level l (R columns).
    template <int VW, int BS, int RP = 1>
    void sweep_launch(int rows, int R, const Csr<T>& Bm, const T* dinv, const T* X, const T* F, T* Y) {
        const int G = R / VW;
        const long long tot = (long long)rows * G;
        const int grid = (int)std::max<long long>(1, (tot + BS - 1) / BS);
        if (Bm.eci) {
            const long long span = (tot + RP - 1) / RP;
            hipLaunchKernelGGL((k_sweep_ve<T, T, VW, BS, RP>), dim3((int)std::max<long long>(1, (span + BS - 1) / BS)),
                               dim3(BS), 0, s, rows, G, FastDiv((uint32_t)G), (const int*)Bm.eci, (const T*)Bm.ev,
                               dinv, X, F, Y);
            HIPCHK(hipGetLastError());
            return;
        }
        if (RP != 1) fail(BAMG_EDEVICE, "two row pieces per thread need the ELL-4 operator");
        if (Bm.cci) {
            hipLaunchKernelGGL((k_sweep_v9<T, T, VW, BS>), dim3(grid), dim3(BS), 0, s, rows, G, FastDiv((uint32_t)G),
                               Bm.cld, (const int*)Bm.cci, (const T*)Bm.cv, dinv, X, F, Y);
            HIPCHK(hipGetLastError());
            return;
        }
        hipLaunchKernelGGL((k_sweep_v<T, T, VW, BS>), dim3(grid), dim3(BS), 0, s, rows, G, FastDiv((uint32_t)G),
                           (const int*)Bm.rp, (const int*)Bm.ci, (const T*)Bm.v, dinv, X, F, Y);
        HIPCHK(hipGetLastError());
    }

    void sweep_shape(const SweepShape& sh, int rows, int R, const Csr<T>& Bm, const T* dinv, const T* X, const T* F,
                     T* Y) {
        switch (sh.rp * 100000 + sh.vw * 1000 + sh.bs) {
            case 202256: sweep_launch<2, 256, 2>(rows, R, Bm, dinv, X, F, Y); break;
            case 202512: sweep_launch<2, 512, 2>(rows, R, Bm, dinv, X, F, Y); break;
            case 204256: sweep_launch<4, 256, 2>(rows, R, Bm, dinv, X, F, Y); break;
            case 204512: sweep_launch<4, 512, 2>(rows, R, Bm, dinv, X, F, Y); break;
            case 101128: sweep_launch<1, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 101256: sweep_launch<1, 256>(rows, R, Bm, dinv, X, F, Y); break;
            case 101512: sweep_launch<1, 512>(rows, R, Bm, dinv, X, F, Y); break;
            case 102128: sweep_launch<2, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 102256: sweep_launch<2, 256>(rows, R, Bm, dinv, X, F, Y); break;
            case 102512: sweep_launch<2, 512>(rows, R, Bm, dinv, X, F, Y); break;
            case 104128: sweep_launch<4, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 104256: sweep_launch<4, 256>(rows, R, Bm, dinv, X, F, Y); break;
            case 104512: sweep_launch<4, 512>(rows, R, Bm, dinv, X, F, Y); break;
            case 103128: sweep_launch<3, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 103256: sweep_launch<3, 256>(rows, R, Bm, dinv, X, F, Y); break;
            case 106128: sweep_launch<6, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 106256: sweep_launch<6, 256>(rows, R, Bm, dinv, X, F, Y); break;
            case 112128: sweep_launch<12, 128>(rows, R, Bm, dinv, X, F, Y); break;
            case 112256: sweep_launch<12, 256>(rows, R, Bm, dinv, X, F, Y); break;
            default: fail(BAMG_EDEVICE, "no sweep variant %d,%d,%d", sh.vw, sh.bs, sh.rp);
        }
    }

    // Launch shape for a sweep of this level: forced, cached, or tuned now by
    // timing every candidate once (X -> scratch, X unchanged).  Shapes below
    // 2^20 entries are not worth timing and take the plain layout.
    SweepShape pick_sweep_shape(int l, int R, const T* X, T* scratch) {
        SweepShape sh;
        if (forced_sweep_shape(R, sh)) {
            if (!L[l].B.eci) sh.rp = 1;        // two pieces per thread only on the ELL-4 operator
            return sh;
        }
        auto& lv = L[l];
        const int rows = lv.cont_rows;
        if ((long long)rows * R < (1LL << 20)) return sh;
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        // (the key only separates shapes: level 0 by its nnz, the others by
        // their rows, without a read-back)
        const int nnz = l == 0 ? nnz0 : -1;
        auto key = std::make_tuple(dev, rows, R, nnz, (int)sizeof(T));
        auto& tu = sweep_tuner();
        const std::string fkey = tune_key(dev, "sweep", {rows, R, nnz, (long long)sizeof(T), lv.B.eci ? 1 : 0});
        {
            std::lock_guard<std::mutex> lk(tu.mu);
            auto it = tu.best.find(key);
            if (it != tu.best.end()) return it->second;
            tune_cache_read(tu);
            auto ft = tu.file.find(fkey);
            if (ft != tu.file.end() && ft->second.size() == 3) {
                SweepShape c{ft->second[0], ft->second[1], ft->second[2]};
                const bool known = (c.vw == 1 || c.vw == 2 || c.vw == 3 || c.vw == 4 || c.vw == 6 || c.vw == 12) &&
                                   R % c.vw == 0 && (c.bs == 128 || c.bs == 256 || c.bs == 512) &&
                                   (c.vw <= 2 || c.vw == 4 || c.bs <= 256) &&
                                   (c.rp == 1 || (c.rp == 2 && lv.B.eci && (c.vw == 2 || c.vw == 4) && c.bs >= 256));
                if (known) { tu.best[key] = c; return c; }
            }
        }
        auto t0 = std::chrono::steady_clock::now();
        std::vector<SweepShape> cand;
        for (int vw : {1, 2, 3, 4, 6, 12})
            for (int bs : {128, 256, 512})
                if (R % vw == 0 && (vw == 1 || vw == 2 || vw == 4 || bs <= 256)) cand.push_back({vw, bs, 1});
        if (lv.B.eci)
            for (int vw : {2, 4})
                for (int bs : {256, 512})
                    if (R % vw == 0) cand.push_back({vw, bs, 2});
        hipEvent_t a, b;
        a = event_pool().get();
        b = event_pool().get();
        sweep_shape(cand[0], rows, R, lv.B, lv.dinv, X, nullptr, scratch);     // warm-up
        float bestms = 1e30f;
        for (int rep = 0; rep < 2; ++rep)       // each candidate's best of two
            for (auto& c : cand) {
                HIPCHK(hipEventRecord(a, s));
                sweep_shape(c, rows, R, lv.B, lv.dinv, X, nullptr, scratch);
                HIPCHK(hipEventRecord(b, s));
                HIPCHK(hipEventSynchronize(b));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, a, b));
                if (ms < bestms) { bestms = ms; sh = c; }
            }
        event_pool().put(a);
        event_pool().put(b);
        std::lock_guard<std::mutex> lk(tu.mu);
        tu.best[key] = sh;
        tu.file[fkey] = {sh.vw, sh.bs, sh.rp};
        tune_cache_write(tu);
        tu.tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return sh;
    }

    // nu homogeneous sweeps on the continuing rows of level l (R columns).
    // Multicolour Gauss-Seidel needs every coupling of the operators of level
    // l between points of different colours.
    void check_colours(int l) {
        auto& lv = L[l];
        if (!mcgs || lv.rows == 0) return;
        zero(err, sizeof(int) * 4);
        LAUNCH(k_check_colours, nblk(lv.rows), BAMG_BLK, s, lv.rows, (const ChainGeo*)lv.dgeo, lv.nch,
               (const int*)lv.B.rp, (const int*)lv.B.ci, err);
        if (lv.Tm.rp)
            LAUNCH(k_check_colours, nblk(lv.rows), BAMG_BLK, s, lv.rows, (const ChainGeo*)lv.dgeo, lv.nch,
                   (const int*)lv.Tm.rp, (const int*)lv.Tm.ci, err);
        if (get1(err))
            fail(BAMG_EINVAL, "multicolour Gauss-Seidel: level %d couples points of one colour "
                              "(the operator reaches beyond the 3 x 3 box)", l);
    }

    // nu multicolour Gauss-Seidel sweeps on B X = 0 for R interleaved columns.
    void mcgs_tv(int l, T* X, int R, int nu, bool profile) {
        auto& lv = L[l];
        const int rows = lv.cont_rows;
        const int vw = R % 4 == 0 ? 4 : R % 2 == 0 ? 2 : 1;
        const int G = R / vw;
        const FastDiv dG((uint32_t)G);
        const long long tot = (long long)rows * G;
        if (tot >= (1LL << 31)) fail(BAMG_EINVAL, "level %d too large for one sweep launch", l);
        auto kern = vw == 4 ? k_mcgs_tv<T, T, 4> : vw == 2 ? k_mcgs_tv<T, T, 2> : k_mcgs_tv<T, T, 1>;
        if (l == 0) { st.sweep_vw = vw; st.sweep_bs = BAMG_BLK; st.sweep_rp = 1; }
        for (int k = 0; k < nu; ++k) {
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (profile) ev = ev_begin();
            for (int c = 0; c < ncol; ++c)
                LAUNCH(kern, nblk(tot), BAMG_BLK, s, rows, (const ChainGeo*)lv.dgeo, lv.ncont, G, dG, c, o.gs_omega,
                       (const int*)lv.B.rp, (const int*)lv.B.ci, (const T*)lv.B.v, X);
            if (profile) ev_end(ev, ev_sweep);     // one sweep = every colour
        }
    }

    void sweeps(int l, T* X, int R, int nu, bool profile) {
        auto& lv = L[l];
        const int rows = lv.cont_rows;
        if (rows == 0 || nu == 0) return;
        if (mcgs) { mcgs_tv(l, X, R, nu, profile); return; }
        T* a = X;
        T* b = sweep_tmp;
        const SweepShape sh = pick_sweep_shape(l, R, X, sweep_tmp);
        if (l == 0) { st.sweep_vw = sh.vw; st.sweep_bs = sh.bs; st.sweep_rp = sh.rp; }
        long long tot = (long long)rows * R;
        for (int k = 0; k < nu; ++k) {
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (profile) ev = ev_begin();
            sweep_shape(sh, rows, R, lv.B, lv.dinv, a, nullptr, b);
            if (profile) ev_end(ev, ev_sweep);
            std::swap(a, b);
        }
        if (a != X) HIPCHK(hipMemcpyAsync(X, a, sizeof(T) * tot, hipMemcpyDeviceToDevice, s));
    }

    // The ELL copy of B_l that the setup kernels read instead of its CSR
    // arrays: row-major 4-wide on the finest level, column-major 9-wide
    // (stride = rows) on a coarse grid level, or none.
    struct EllSrc { const int* c; const T* v; int ld; int ef; };
    EllSrc ell_of(int l) const {
        const auto& lv = L[l];
        if (lv.B.eci) return {lv.B.eci, lv.B.ev, 0, EF_ELL4};
        if (lv.B.cci) return {lv.B.cci, lv.B.cv, lv.B.cld, EF_ELL9};
        return {nullptr, nullptr, 0, EF_CSR};
    }

    // TV weights of the continuing chains of level l.
    void tv_weights(int l, int use_v) {
        auto& lv = L[l];
        dim3 grid(lv.cnp, lv.ncont);
        const EllSrc es = ell_of(l);
        ef_dispatch(es.ef, [&](auto efc) {
            constexpr int EF = decltype(efc)::value;
            auto part_k = r % 4 == 0 ? k_colnorm_partial<T, T, 4, EF>
                        : r % 2 == 0 ? k_colnorm_partial<T, T, 2, EF> : k_colnorm_partial<T, T, 1, EF>;
            hipLaunchKernelGGL(part_k, grid, dim3(BAMG_BLK), 0, s, (const ChainGeo*)lv.dgeo, CN_ROWS, r, use_v,
                               (const int*)nvc, VS, lv.B.rp, lv.B.ci, (const T*)lv.B.v, es.c, es.v, es.ld,
                               (const T*)lv.U, (const T*)lv.V, WS, part);
        });
        HIPCHK(hipGetLastError());
        dim3 g2(r + (use_v ? nvmax : 0), lv.ncont);
        hipLaunchKernelGGL(k_colnorm_final, g2, dim3(BAMG_BLK), 0, s, (const ChainGeo*)lv.dgeo, CN_ROWS, lv.cnp, r,
                           use_v, (const int*)nvc, WS,
                           (const double*)part, wts);
        HIPCHK(hipGetLastError());
    }

    // BAMG_ARNOLDI_CHECK=0 in the environment: the coarsest Arnoldi process
    // always runs all its steps (no convergence check after ARN_CHECK).
    static bool arnoldi_check_on() {
        const char* e = getenv("BAMG_ARNOLDI_CHECK");
        return !(e && e[0] == '0');
    }

    // BAMG_CYCLE_FUSE=0 in the environment: the cycle takes the
    // prolongation and the first post-smoothing sweep of a small coarse grid
    // level as separate launches (the fused pass computes the same bits).
    static bool cycle_fuse_on() {
        const char* e = getenv("BAMG_CYCLE_FUSE");
        return !(e && e[0] == '0');
    }

    // BAMG_SWEEP_ELL=0 in the environment: kernels read the coarse grid
    // operators from CSR instead of their ELL-9 copies.
    static bool ell9_on() {
        const char* e = getenv("BAMG_SWEEP_ELL");
        return !(e && e[0] == '0');
    }

    // Coarse rows per workgroup of the fused Galerkin launch: forced, cached,
    // or tuned now by timing each candidate twice in place (each writes the
    // same outputs).  Below 2^16 coarse rows, and with a CSR operand, 28.
    template <typename RUN>
    int pick_gal_rows(int nc, int efb, int eft, RUN&& run) {
        if (const int g = forced_gal_rows()) return g;
        if (nc < (1 << 16) || efb == EF_CSR || eft == EF_CSR) return GAL_ROWS;
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        auto key = std::make_tuple(dev, nc, efb, eft, (int)sizeof(T));
        const std::string fkey = tune_key(dev, "galerkin", {nc, efb, eft, (long long)sizeof(T)});
        auto& tu = sweep_tuner();
        {
            std::lock_guard<std::mutex> lk(tu.mu);
            auto it = tu.gal_rows.find(key);
            if (it != tu.gal_rows.end()) return it->second;
            tune_cache_read(tu);
            auto ft = tu.file.find(fkey);
            if (ft != tu.file.end() && ft->second.size() == 1 &&
                (ft->second[0] == 14 || ft->second[0] == 28 || ft->second[0] == 56)) {
                tu.gal_rows[key] = ft->second[0];
                return ft->second[0];
            }
        }
        auto t0 = std::chrono::steady_clock::now();
        hipEvent_t a = event_pool().get(), b = event_pool().get();
        float bestms = 1e30f;
        int best = GAL_ROWS;
        for (int rep = 0; rep < 2; ++rep)
            for (int gr : {14, 28, 56}) {
                HIPCHK(hipEventRecord(a, s));
                run(gr);
                HIPCHK(hipEventRecord(b, s));
                HIPCHK(hipEventSynchronize(b));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, a, b));
                if (ms < bestms) { bestms = ms; best = gr; }
            }
        event_pool().put(a);
        event_pool().put(b);
        std::lock_guard<std::mutex> lk(tu.mu);
        tu.gal_rows[key] = best;
        tu.file[fkey] = {best};
        tune_cache_write(tu);
        tu.tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return best;
    }

    // Both Galerkin products of a grid level in one launch (ELL-9 output),
    // then their CSR forms and the next level's D^-1.
    // BAMG_GAL_ROWS=14|28|56 in the environment forces the fused Galerkin
    // launch's coarse rows per workgroup.
    static int forced_gal_rows() {
        const char* e = getenv("BAMG_GAL_ROWS");
        const int g = e ? atoi(e) : 0;
        return g == 14 || g == 28 || g == 56 ? g : 0;
    }

    void galerkin(int l, bool profile) {
        auto& f = L[l];
        auto& c = L[l + 1];
        const int nc = c.rows;
        // B_l's rows from its ELL copy; T_l's from its ELL-9 copy (T_0 = I)
        const EllSrc eb = ell_of(l);
        const EllSrc et = l == 0 ? EllSrc{nullptr, nullptr, 0, -1}
                        : f.Tm.cci ? EllSrc{f.Tm.cci, f.Tm.cv, f.Tm.cld, EF_ELL9}
                                   : EllSrc{nullptr, nullptr, 0, EF_CSR};
        // one launch with gr coarse rows per workgroup (every choice gives
        // the same bits); the ELL forms take the tuned choice
        auto run = [&](int gr) {
            ef_dispatch(eb.ef, [&](auto efb) {
                constexpr int EFB = decltype(efb)::value;
                auto launch = [&](auto eft) {
                    constexpr int EFT = decltype(eft)::value;
                    auto go = [&](auto grc) {
                        constexpr int GR = decltype(grc)::value;
                        LAUNCH((k_galerkin_bt<T, EFB, EFT, GR>), ceil_div(nc, GR), 9 * GR, s, nc,
                               (const ChainGeo*)c.dgeo, c.nch, f.qc, (const T*)f.qv, (const int*)f.B.rp,
                               (const int*)f.B.ci, (const T*)f.B.v, eb.c, eb.v, eb.ld, (const int*)f.Tm.rp,
                               (const int*)f.Tm.ci, (const T*)f.Tm.v, et.c, et.v, et.ld, f.pc, (const T*)f.pv, c.B.gci,
                               c.B.gv, f.cnt, c.Tm.gci, c.Tm.gv, f.cnt2);
                    };
                    if constexpr (EFB != EF_CSR && EFT != EF_CSR) {
                        if (gr == 14) go(std::integral_constant<int, 14>{});
                        else if (gr == 56) go(std::integral_constant<int, 56>{});
                        else go(std::integral_constant<int, GAL_ROWS>{});
                    } else {
                        go(std::integral_constant<int, GAL_ROWS>{});
                    }
                };
                if (et.ef < 0) launch(std::integral_constant<int, -1>{});
                else if (et.ef == EF_ELL9) launch(std::integral_constant<int, EF_ELL9>{});
                else launch(std::integral_constant<int, EF_CSR>{});
            });
        };
        const int gr = pick_gal_rows(nc, eb.ef, et.ef, run);
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (profile) ev = ev_begin();
        run(gr);
        if (profile) ev_end(ev, ev_gal);
        scan(nc, f.cnt, c.B.rp);
        scan(nc, f.cnt2, c.Tm.rp);
        if (profile) ev = ev_begin();
        hipLaunchKernelGGL(k_ell9c_to_csr2<T>, dim3(nblk(nc), 2), dim3(BAMG_BLK), 0, s, nc, (const int*)c.B.gci,
                           (const T*)c.B.gv, (const int*)c.B.rp, c.B.ci, c.B.v, (const int*)c.Tm.gci,
                           (const T*)c.Tm.gv, (const int*)c.Tm.rp, c.Tm.ci, c.Tm.v);
        HIPCHK(hipGetLastError());
        if (profile) ev_end(ev, ev_gal_csr);
        zero(err, sizeof(int) * 4);
        LAUNCH(k_dinv<T>, nblk(nc), BAMG_BLK, s, nc, c.B.rp, c.B.ci, c.B.v, o.omega, c.dinv, err);
    }

    void build_level(int l, int use_v, bool inject, bool profile) {
        auto& lv = L[l];
        auto& c = L[l + 1];
        if (lv.ncont == 0) return;
        tv_weights(l, use_v);
        std::pair<hipEvent_t, hipEvent_t> ev;
        if (profile) ev = ev_begin();
        if (unstructured) {
            fit_u(l, use_v, inject);
            if (profile) ev_end(ev, ev_ls);
            galerkin_u(l, profile);
            return;
        }
        if (!use_v && mlp_pk) {
            // learned form of the first pass: network proposal judged by the fit
            const int grid = std::min(learn_grid, nblk(lv.cont_rows));
            LAUNCH((k_ls_fit_learn<T, T, T>), grid, BAMG_BLK, s, lv.cont_rows, (const ChainGeo*)lv.dgeo, lv.ncont, r,
                   (const T*)lv.U, (const double*)wts, WS, o.caliber, lv.pc, lv.pv, inject ? c.U : (T*)nullptr,
                   lv.jcnt, (const int*)lv.B.rp, (const int*)lv.B.ci, (const T*)lv.B.v, (const MlpPack*)mlp_pk,
                   o.mlp_judge, learn_part);
            LAUNCH(k_learn_tally, 1, BAMG_WAVE, s, grid, (const float*)learn_part, learn_acc);
        } else {
            LAUNCH((k_ls_fit<T, T, T>), nblk(lv.cont_rows), BAMG_BLK, s, lv.cont_rows, (const ChainGeo*)lv.dgeo,
                   lv.ncont, r, use_v, (const int*)nvc, VS, (const T*)lv.U, (const T*)lv.V, (const double*)wts, WS,
                   o.caliber, lv.pc, lv.pv, inject ? c.U : (T*)nullptr, lv.jcnt, (const int*)lv.B.rp,
                   (const int*)lv.B.ci, (const T*)lv.B.v, use_v ? (float*)nullptr : lv.feat,
                   use_v ? lv.slotw : lv.slotw0);
        }
        if (profile) ev_end(ev, use_v ? ev_ls2 : ev_ls);
        LAUNCH(k_build_q<T>, nblk(c.rows), BAMG_BLK, s, c.rows, (const ChainGeo*)c.dgeo, (const ChainGeo*)lv.dgeo, c.nch,
               lv.pc, lv.qc, lv.qv, lv.qmask);
        galerkin(l, profile);
        check_colours(l + 1);
    }

    // ---- coarsest pseudo-inverses of every chain into the W pool ------------
    void coarsest_inverse() {
        long long wtot = 0;
        for (auto& d : cdh) wtot += (long long)d.n * d.n;
        LAUNCH(k_fill, nblk(wtot), BAMG_BLK, s, wtot, 0.0, Wp);
        // b_col keeps only the stored entries of the last column: clear it
        LAUNCH(k_fill, nblk(NVt), BAMG_BLK, s, (long long)NVt, 0.0, bcolp);
        const dim3 gv(nblk(maxnL), nch);
        hipLaunchKernelGGL(k_cz_densify<T>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, Wp, bcolp);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_cz_absmax_sparse<T>, dim3(64, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, part);
        LAUNCH(k_cz_absmax_final, nch, BAMG_BLK, s, 64, (const double*)part, scale);
        HIPCHK(hipGetLastError());
        LAUNCH(k_fill, ceil_div(nch, BAMG_BLK), BAMG_BLK, s, (long long)nch, 1e300, minpiv);
        if (dense_fallback) {
            dense_gj_inverse();
        } else {
            int bbmax = 0;
            for (auto& d : cdsh) bbmax = std::max(bbmax, d.ny * d.ny);
            hipLaunchKernelGGL(k_cz_extract, dim3(nblk(bbmax), nxmax, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds,
                               (const double*)Wp, Fp);
            HIPCHK(hipGetLastError());
            bool arrow = false, plain = false;
            for (auto& d : cdsh) {
                if (d.n < 2) continue;
                if (d.periodic && d.nx >= 3) arrow = true; else plain = true;
            }
            // chains without the arrow: divide and conquer over the block
            // rows, the diagonal blocks' inverses joined level by level
            if (plain) {
                hipLaunchKernelGGL(k_dc_leaf, dim3(nxmax, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, Fp, Wp,
                                   (const double*)scale, dcmp);
                for (int t = 0; (1 << t) < nxmax; ++t) {
                    const int joins = ceil_div(nxmax - (1 << t), 2 << t), side = std::min(2 << t, nxmax);
                    hipLaunchKernelGGL(k_dc_core, dim3(joins, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, t, Fp,
                                       (const double*)Wp, dcmp);
                    hipLaunchKernelGGL(k_dc_panels, dim3(nxmax, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, t,
                                       Fp, (const double*)Wp, dcP, dcR, NVt);
                    hipLaunchKernelGGL(k_dc_tiles, dim3(joins * side * side, nch), dim3(BAMG_BLK), 0, s,
                                       (const CoarseDesc*)cds, t, (const double*)dcP, (const double*)dcR, NVt, Wp);
                    HIPCHK(hipGetLastError());
                }
                hipLaunchKernelGGL(k_dc_minpiv, dim3(nch), dim3(BAMG_WAVE), 0, s, (const CoarseDesc*)cds,
                                   (const double*)dcmp, minpiv);
            }
            if (arrow) {
                const dim3 gl(4, nch);
                for (int k = 0; k + 1 < nxmax; ++k) {
                    hipLaunchKernelGGL(k_cz_lu_step, gl, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, k, Fp,
                                       (const double*)scale, minpiv);
                    hipLaunchKernelGGL(k_cz_elim_arrow, dim3(2, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, k,
                                       Fp);
                    HIPCHK(hipGetLastError());
                }
                hipLaunchKernelGGL(k_cz_lu_step, gl, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cds, -1, Fp,
                                   (const double*)scale, minpiv);
            }
            HIPCHK(hipGetLastError());
            if (arrow)
                hipLaunchKernelGGL(k_cz_subst, dim3(ceil_div(maxnL, CZ_SUB_TC), nch), dim3(BAMG_BLK), 0, s,
                                   (const CoarseDesc*)cds, Wp, (const double*)Fp);
            HIPCHK(hipGetLastError());
            if (bordered) bordered_inverse();
        }
        hipLaunchKernelGGL(k_cz_zero_border, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, Wp);
        // y = [-Binv b_col; 1]
        const dim3 gw(ceil_div(maxnL, 4), nch);
        hipLaunchKernelGGL(k_cz_gemv, gw, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, 1, (const double*)Wp,
                           (const double*)bcolp, t1);
        hipLaunchKernelGGL(k_cz_null, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, (const double*)t1, ypool);
        // s = W 1, u = y^T W, y^T s, y^T y, projections
        LAUNCH(k_fill, nblk(NVt), BAMG_BLK, s, (long long)NVt, 1.0, t2);
        hipLaunchKernelGGL(k_cz_gemv, gw, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, 0, (const double*)Wp,
                           (const double*)t2, t1);
        {
            const int nchunk = ceil_div(maxnL, GT_RCH);
            hipLaunchKernelGGL(k_cz_gemv_t_partial, dim3(nblk(maxnL), nchunk, nch), dim3(BAMG_BLK), 0, s,
                               (const CoarseDesc*)cd, (const double*)Wp, (const double*)ypool, gtpart, GT_RCH);
            hipLaunchKernelGGL(k_cz_gemv_t_final, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, nchunk, GT_RCH,
                               (const double*)gtpart, t2);
        }
        LAUNCH(k_cz_dot, nch, BAMG_BLK, s, (const CoarseDesc*)cd, (const double*)ypool, (const double*)t1, csc, SCS);
        LAUNCH(k_cz_dot, nch, BAMG_BLK, s, (const CoarseDesc*)cd, (const double*)ypool, (const double*)ypool, csc + 1,
               SCS);
        hipLaunchKernelGGL(k_cz_project, dim3(nblk((long long)maxnL * maxnL), nch), dim3(BAMG_BLK), 0, s,
                           (const CoarseDesc*)cd, Wp, (const double*)t1, (const double*)t2, (const double*)ypool,
                           (const double*)csc, SCS);
        // c = T^T 1, cy = c^T y
        hipLaunchKernelGGL(k_cz_colsum<T>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, cpool);
        LAUNCH(k_cz_dot, nch, BAMG_BLK, s, (const CoarseDesc*)cd, (const double*)cpool, (const double*)ypool, cy, 1);
        // the smallest pivot is read at the next read-back (check_pivot), so
        // that the host can go on issuing work meanwhile
        pivot_pending = true;
        if (MIXED)
            hipLaunchKernelGGL(k_cz_w_f32, dim3(std::min(2048, nblk((long long)maxnL * maxnL)), nch), dim3(BAMG_BLK), 0,
                               s, (const CoarseDesc*)cd, (const double*)Wp, Wfp);
    }

    // The smallest pivot of the last coarsest inverse (relative to max |B_L|):
    // BAMG_ESINGULAR below 1e-12.  Called before anything read back depends
    // on the inverse; the kernels in between only compute with its values.
    void check_pivot() {
        if (!pivot_pending) return;
        pivot_pending = false;
        std::vector<double> mp = getn(minpiv, nch);
        double mn = 1e300;
        for (double v : mp) mn = std::min(mn, v);
        st.coarsest_min_pivot = mn;
        if (!(mn > 1e-12)) fail(BAMG_ESINGULAR, "coarsest pivot %.3e below 1e-12 of max |B_L|", mn);
    }

    // The coarsest inverse of a bordered grid from the main part's inverse
    // (k_bd_* in k_coarse.h): Z, Y, the Schur complement S and its inverse,
    // G, H, then W in natural order.
    void bordered_inverse() {
        const CoarseDesc& m = cdsh[0];
        const int ne = cdh[0].nx - 1;
        const long long zs = (long long)m.n * GJ_NB;
        const int gz = (int)std::min<long long>(ceil_div(zs, BAMG_BLK), 4096);
        LAUNCH(k_bd_zy, gz, BAMG_BLK, s, (const CoarseDesc*)cd, (const CoarseDesc*)cds, (const double*)Wp, bdZ, bdY);
        LAUNCH(k_bd_schur, 1, BAMG_BLK, s, (const CoarseDesc*)cd, (const double*)Wp, (const double*)bdZ, bdS);
        LAUNCH(k_gj_diag, 1, CZ_GJ_THREADS, s, GJ_NB, 0, ne, bdS, (const double*)scale, minpiv);
        LAUNCH(k_bd_gh, gz, BAMG_BLK, s, (const CoarseDesc*)cd, (const CoarseDesc*)cds, (const double*)bdS,
               (const double*)bdZ, (const double*)bdY, bdG, bdH);
        hipLaunchKernelGGL(k_bd_combine_main, dim3(m.nx, m.nx), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd,
                           (const CoarseDesc*)cds, Wp, (const double*)bdG, (const double*)bdY);
        HIPCHK(hipGetLastError());
        const long long te = (long long)cdh[0].nx * cdh[0].n;
        LAUNCH(k_bd_combine_edge, (int)std::min<long long>(ceil_div(te, BAMG_BLK), 4096), BAMG_BLK, s,
               (const CoarseDesc*)cd, (const CoarseDesc*)cds, Wp, (const double*)bdG, (const double*)bdH,
               (const double*)bdS);
    }

    // Dense blocked Gauss-Jordan (coarse sides > 64; single chain only).
    void dense_gj_inverse() {
        const CoarseDesc& d = cdh[0];
        const int nL = d.n, m = nL - 1;
        if (m <= 0) return;
        const int tiles = ceil_div(m, 64);
        const int ut = ceil_div(m, GJ_T);
        for (int k0 = 0; k0 < m; k0 += GJ_NB) {
            int nb = std::min(GJ_NB, m - k0);
            LAUNCH(k_gj_diag, 1, BAMG_BLK, s, nL, k0, nb, Wp, (const double*)scale, minpiv);
            LAUNCH(k_gj_rowpanel, tiles, BAMG_BLK, s, m, nL, k0, nb, Wp);
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (o.profile) ev = ev_begin();
            LAUNCH(k_gj_update, ut * ut, BAMG_BLK, s, m, nL, k0, nb, Wp);
            if (o.profile) {
                ev_end(ev, ev_gj);
                gj_flops += 2.0 * nb * (double)(m - nb) * (double)(m - nb);
            }
            LAUNCH(k_gj_colpanel, tiles, BAMG_BLK, s, m, nL, k0, nb, Wp);
        }
    }

    // The start vector (basis column 0): u -= y (c^T u)/cy, normalised.
    void arnoldi_start() {
        const dim3 gv(nblk(maxnL), nch);
        hipLaunchKernelGGL(k_cz_arn_dots2, dim3(1, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, -1,
                           (const double*)cpool, (const double*)Vb, dots, DS);
        hipLaunchKernelGGL(k_cz_arn_update2, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, -1, (const double*)ypool,
                           (const double*)cy, (const double*)dots, (const double*)vyb, DS, Vb, Hh, HS, npart);
        hipLaunchKernelGGL(k_cz_arn_normalize, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, -1, Vb, Hh, HS, vyb, DS,
                           (const double*)npart);
        HIPCHK(hipGetLastError());
    }

    // Step j >= 0 after the product u = W T v_j in column j+1: the projection
    // against c with the first Gram-Schmidt pass, the second pass, the norm;
    // t1 = T v_{j+1} for the next step.  K = j + 1 rounded up to 8.
    template <typename F>
    static void arn_dispatch(int j, F&& f) {
        switch ((j + 8) / 8) {
            case 1: f(std::integral_constant<int, 8>{}); break;
            case 2: f(std::integral_constant<int, 16>{}); break;
            case 3: f(std::integral_constant<int, 24>{}); break;
            case 4: f(std::integral_constant<int, 32>{}); break;
            case 5: f(std::integral_constant<int, 40>{}); break;
            case 6: f(std::integral_constant<int, 48>{}); break;
            case 7: f(std::integral_constant<int, 56>{}); break;
            default: f(std::integral_constant<int, 64>{}); break;
        }
    }
    void arnoldi_orthogonalize(int j) {
        static_assert(HQR_MAXM <= 64, "Arnoldi steps beyond the widest accumulator set");
        const dim3 gv(nblk(maxnL), nch);
        hipLaunchKernelGGL(k_cz_arn_dots2, dim3(j + 2, nch), dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j,
                           (const double*)cpool, (const double*)Vb, dots, DS);
        arn_dispatch(j, [&](auto kc) {
            constexpr int K = decltype(kc)::value;
            hipLaunchKernelGGL(k_cz_arn_update2p<K>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j,
                               (const double*)ypool, (const double*)cy, (const double*)dots, (const double*)vyb, DS, Vb,
                               Hh, HS, apart);
            hipLaunchKernelGGL(k_cz_arn_updatep<K>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j,
                               (const double*)ypool, (const double*)apart, DS, (const double*)Vb, Hh, HS, arn_u, npart);
        });
        hipLaunchKernelGGL(k_cz_arn_normtv<T>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j, (const double*)arn_u,
                           Vb, Hh, HS, vyb, DS, (const double*)npart, t1);
        HIPCHK(hipGetLastError());
    }

    // ---- coarsest eigenpairs (Arnoldi, all chains in lockstep) ---------------
    void coarsest_eigs() {
        const int want = o.n_eig - 1;
        const dim3 gv(nblk(maxnL), nch);
        const dim3 gw(ceil_div(maxnL, 4), nch);
        const dim3 gw2(ceil_div(maxnL, 2), nch);
        auto steps = [&](int j0, int j1) {
            for (int j = j0; j < j1; ++j) {
                // the mixed form multiplies by its FP32 copy of W (half the bytes)
                if (MIXED)
                    hipLaunchKernelGGL(k_cz_arn_gemv_f32, gw2, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j,
                                       (const float*)Wfp, (const double*)t1, Vb);
                else
                    hipLaunchKernelGGL(k_cz_arn_gemv, gw, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, j,
                                       (const double*)Wp, (const double*)t1, Vb);
                HIPCHK(hipGetLastError());
                arnoldi_orthogonalize(j);
            }
        };
        auto eig = [&](int mcap) {
            LAUNCH(k_cz_hess, nch, BAMG_WAVE, s, (const CoarseDesc*)cd, want, mcap, (const double*)Hh, HS, nsel, NS,
                   sel_lam, LSS);
            hipLaunchKernelGGL(k_cz_hess_vec, dim3(HSEL_THETA / 2, nch), dim3(BAMG_WAVE), 0, s, (const CoarseDesc*)cd,
                               mcap, (const double*)Hh, HS, (const int*)nsel, NS, (const double*)sel_lam, LSS, sel_s,
                               SS);
            HIPCHK(hipGetLastError());
        };
        // Arnoldi steps used: every chain's am, or a check point k (ARN_CHECK1,
        // ARN_CHECK2) when the Ritz pairs of the first k steps already meet
        // ARN_TOL for every chain that runs more
        arn_used = 1 << 30;
        if (want > 0 && AMmax >= 1) {
            zero(Hh, sizeof(double) * nch * HS);
            hipLaunchKernelGGL(k_cz_arn_start, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, o.seed, Vb);
            HIPCHK(hipGetLastError());
            // the start vector is basis column 0 (no H entry), then t1 = T v_0
            arnoldi_start();
            hipLaunchKernelGGL(k_cz_tv<T>, gv, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)cd, 0, (const double*)Vb, t1);
            int done = 0;
            if (arnoldi_check_on()) {
                for (int k : {ARN_CHECK1, ARN_CHECK2}) {
                    if (k >= AMmax) break;
                    steps(done, k);
                    done = k;
                    eig(k);
                    LAUNCH(k_cz_ritz_check, ceil_div(nch, 64), 64, s, nch, (const CoarseDesc*)cd, k,
                           (const double*)Hh, HS, (const int*)nsel, NS, (const double*)sel_lam, LSS,
                           (const double*)sel_s, SS, ARN_TOL, itmp);
                    check_pivot();
                    std::vector<int> okv = getn(itmp, nch);
                    bool all = true;
                    for (int v : okv) all &= v != 0;
                    if (all) { arn_used = k; break; }
                }
            }
            if (arn_used > AMmax) {
                steps(done, AMmax);
                eig(1 << 30);
            }
        } else {
            eig(1 << 30);
        }
        st.arnoldi_steps = std::min(AMmax, arn_used);
        check_pivot();
        std::vector<int> hs = getn(nsel, (size_t)nch * NS);
        int emax = 0;
        for (int c = 0; c < nch; ++c) {
            if (hs[(size_t)c * NS + 2]) fail(BAMG_EDEVICE, "Hessenberg QR of chain %d's coarsest Arnoldi matrix failed", c);
            emax = std::max(emax, hs[(size_t)c * NS]);
        }
        LAUNCH(k_cz_tables, ceil_div(nch, 64), 64, s, nch, (const int*)nsel, NS, (const double*)sel_lam, LSS, lam, kind,
               ent_col, KV, nvc, nentc);
        nvc_h = getn(nvc, nch);
        nvmax = 1;
        for (int v : nvc_h) nvmax = std::max(nvmax, v);
        if (nvmax > VS) fail(BAMG_EDEVICE, "eigenvector columns exceed the reserved %d", VS);
        // every chain's coarsest rows live on its own level: one launch per level
        for (int l = 0; l < (int)L.size(); ++l) {
            auto& lv = L[l];
            const int c0 = lv.ncont, c1 = lv.nch;          // chains whose coarsest level is l
            if (c1 <= c0) continue;
            const CoarseDesc* cdl = cd + c0;
            const dim3 gvl(nblk(maxnL), c1 - c0);
            hipLaunchKernelGGL(k_cz_ycol<T>, gvl, dim3(BAMG_BLK), 0, s, cdl, (const double*)ypool,
                               (const double*)(cy + c0), lv.V, VS);
            for (int e = 0; e < emax; ++e) {
                hipLaunchKernelGGL(k_cz_ritz, gvl, dim3(BAMG_BLK), 0, s, cdl, e, arn_used,
                                   (const int*)(nsel + (size_t)c0 * NS), NS,
                                   (const double*)Vb, (const double*)(sel_s + (size_t)c0 * SS), SS, rre, rim);
                hipLaunchKernelGGL(k_cz_eigvec<T>, dim3(c1 - c0), dim3(BAMG_BLK), 0, s, cdl, e,
                                   (const int*)(nsel + (size_t)c0 * NS), NS, (const double*)(sel_lam + (size_t)c0 * LSS),
                                   LSS, (const double*)rre, (const double*)rim, (const int*)(ent_col + (size_t)c0 * KV),
                                   KV, lv.V, VS);
            }
            HIPCHK(hipGetLastError());
        }
    }

    // Up-leg step of level l (Algorithm 3): V_l = P_l V_{l+1} for the chains
    // that continue below l, relaxed on (B_l - lam T_l) v = 0, then the
    // eigenvalue approximations updated (Rayleigh quotients).
    void upleg_level(int l) {
        {
            auto& lv = L[l];
            auto& c = L[l + 1];
            if (lv.ncont == 0) return;
            const int rows = lv.cont_rows;
            const EllSrc es = ell_of(l);
            long long tot = (long long)rows * VS;
            FastDiv dR((uint32_t)VS);
            if (VS == 4 || VS == 8 || VS == 12) {
                auto ik = VS == 4 ? k_interp_rows<T, T, 4> : VS == 8 ? k_interp_rows<T, T, 8> : k_interp_rows<T, T, 12>;
                LAUNCH(ik, nblk(rows), BAMG_BLK, s, rows, lv.pc, (const T*)lv.pv, (const T*)c.V, lv.V);
            } else {
                LAUNCH((k_interp<T, T>), nblk(tot), BAMG_BLK, s, rows, VS, dR, lv.pc, (const T*)lv.pv, (const T*)c.V,
                       lv.V);
            }
            T* a = lv.V;
            T* b = sweep_tmp;
            // T_l's rows from its ELL-9 copy where B_l's come from one too
            const bool t9 = es.ef == EF_ELL9 && lv.Tm.cci;
            const int* tec = t9 ? lv.Tm.cci : nullptr;
            const T* tev = t9 ? (const T*)lv.Tm.cv : nullptr;
            const int teld = t9 ? lv.Tm.cld : 0;
            auto teft = [&](auto&& go) {
                if (t9) go(std::integral_constant<int, EF_ELL9>{});
                else go(std::integral_constant<int, EF_CSR>{});
            };
            ef_dispatch(es.ef, [&](auto efc) {
                constexpr int EF = decltype(efc)::value;
                teft([&](auto eftc) {
                    constexpr int EFT = EF == EF_ELL9 ? decltype(eftc)::value : EF_CSR;
                    auto relax = VS == 4 ? k_eig_relax<T, T, 4, EF, EFT>
                               : VS == 8 ? k_eig_relax<T, T, 8, EF, EFT> : k_eig_relax<T, T, 12, EF, EFT>;
                    for (int k = 0; k < o.nu_setup; ++k) {
                        if (mcgs) {      // in place, colour by colour
                            for (int cc = 0; cc < ncol; ++cc)
                                LAUNCH(relax, nblk(rows), BAMG_BLK, s, rows, (const ChainGeo*)lv.dgeo, lv.ncont,
                                       (const int*)nvc, KV, lv.B.rp, lv.B.ci, (const T*)lv.B.v, es.c, es.v, es.ld,
                                       lv.Tm.rp, lv.Tm.ci, (const T*)lv.Tm.v, tec, tev, teld, (const double*)lam,
                                       (const int*)kind, o.gs_omega, cc, (const T*)a, a);
                            continue;
                        }
                        LAUNCH(relax, nblk(rows), BAMG_BLK, s, rows, (const ChainGeo*)lv.dgeo, lv.ncont,
                               (const int*)nvc, KV, lv.B.rp, lv.B.ci, (const T*)lv.B.v, es.c, es.v, es.ld, lv.Tm.rp,
                               lv.Tm.ci, (const T*)lv.Tm.v, tec, tev, teld, (const double*)lam, (const int*)kind,
                               o.omega, -1, (const T*)a, b);
                        std::swap(a, b);
                    }
                });
            });
            if (a != lv.V) HIPCHK(hipMemcpyAsync(lv.V, a, sizeof(T) * tot, hipMemcpyDeviceToDevice, s));
            if (nvmax > 1) {
                ef_dispatch(es.ef, [&](auto efc) {
                    constexpr int EF = decltype(efc)::value;
                    teft([&](auto eftc) {
                        constexpr int EFT = EF == EF_ELL9 ? decltype(eftc)::value : EF_CSR;
                        hipLaunchKernelGGL((k_rayleigh_partial<T, T, EF, EFT>), dim3(lv.cnp, lv.ncont),
                                           dim3(BAMG_BLK), 0, s, (const ChainGeo*)lv.dgeo, VS, KV, (const int*)nentc,
                                           (const int*)ent_col, (const int*)kind, lv.B.rp, lv.B.ci, (const T*)lv.B.v,
                                           es.c, es.v, es.ld, lv.Tm.rp, lv.Tm.ci, (const T*)lv.Tm.v, tec, tev, teld,
                                           (const T*)lv.V, CN_ROWS, part);
                    });
                });
                hipLaunchKernelGGL(k_rayleigh_final, dim3(KV, lv.ncont), dim3(BAMG_BLK), 0, s, (const ChainGeo*)lv.dgeo,
                                   CN_ROWS, lv.cnp, KV,
                                   (const int*)nentc, (const int*)ent_col, (const int*)kind, (const double*)part, lam);
                HIPCHK(hipGetLastError());
            }
        }
    }

    // The setup's state-vector approximation x0 = V_0[:, 0] / sum per chain.
    void state_from_v() {
        LAUNCH((k_get_col_t<T>), nblk(n), BAMG_BLK, s, (int)n, VS, 0, (const T*)L[0].V, x0);
        seg_reduce<RED_SUM>(x0, nullptr, sc);
        LAUNCH(k_seg_scale, nblk(n), BAMG_BLK, s, (int)n, (const ChainGeo*)L[0].dgeo, nch, (const int*)nullptr,
               (const double*)x0, (const double*)nullptr, (const double*)sc, SCS, 0, x0);
    }

    void reorder_input(const int32_t*& rp, const int32_t*& ci, const double*& val, int nnzA) {
        // caller order -> depth order (block-diagonal: columns shift with rows)
        std::vector<int> so(nch), dof(nch), ln(nch);
        for (int c = 0; c < nch; ++c) {
            so[c] = (int)chains[c].uoff;
            dof[c] = L[0].geo[c].off;
            ln[c] = (int)chains[c].n;
        }
        perm_src = A.upload(so);
        perm_dst = A.upload(dof);
        perm_len = A.upload(ln);
        reordered = false;
        for (int c = 0; c < nch; ++c) reordered |= so[c] != dof[c];
        if (!reordered) return;
        zero(err, sizeof(int) * 4);
        LAUNCH(k_check_rp, nblk(n), BAMG_BLK, s, (int)n, rp, nnzA, err);
        if (get1(err) & ERR_RANGE) fail(BAMG_EINVAL, "CSR of A: row_ptr not monotone or outside [0, nnz]");
        int maxn = *std::max_element(ln.begin(), ln.end());
        int* cnt = A.alloc<int>(n + 1);
        int* nrp = A.alloc<int>(n + 1);
        hipLaunchKernelGGL(k_seg_csr_len, dim3(nblk(maxn), nch), dim3(BAMG_BLK), 0, s, nch, (const int*)perm_src,
                           (const int*)perm_dst, (const int*)perm_len, rp, cnt);
        HIPCHK(hipGetLastError());
        scan((int)n, cnt, nrp);
        if (get1(nrp + n) != nnzA) fail(BAMG_EINVAL, "row_ptr does not describe the concatenated chains");
        int* nci = A.alloc<int>(nnzA);
        double* nvv = A.alloc<double>(nnzA);
        hipLaunchKernelGGL(k_seg_csr_fill, dim3(nblk(maxn), nch), dim3(BAMG_BLK), 0, s, (const int*)perm_src,
                           (const int*)perm_dst, (const int*)perm_len, rp, ci, val, (const int*)nrp, nci, nvv);
        HIPCHK(hipGetLastError());
        rp = nrp; ci = nci; val = nvv;
    }

    // Algorithm 3 (bootamg_mle) from level l: relax U_l, then o.mu rounds of
    // fit P_l (to U_l, joined by V_l from the second round on, or from the
    // start when use_v), Q_l, B_{l+1}, T_{l+1} and U_{l+1} = R U_l, the
    // recursion, and the up-leg step.  The bottom (l = depth - 1) forms every
    // chain's coarsest inverse and eigenpairs (a chain whose coarsest level
    // lies higher keeps its operator, so its repeats there change nothing).
    // Returns false where options.stop_after ends the setup.
    // ---- levels without a grid (Section 3.1) --------------------------------
    // The coarsening needs an undirected graph: the pattern of B_0 must be
    // symmetric (then every Q B P is symmetric too).
    void check_symmetric() {
        zero(err, sizeof(int) * 4);
        LAUNCH(k_check_sym, nblk(n), BAMG_BLK, s, (int)n, (const int*)b0rp, (const int*)b0ci, err);
        if (get1(err) & ERR_UNSYM)
            fail(BAMG_EUNSUPPORTED, "coarsening without a grid needs a structurally symmetric A");
    }

    // Drop the captured cycle (its buffers moved); the next cycle recaptures.
    void invalidate_graph() {
        if (gexec) { (void)hipGraphExecDestroy(gexec); gexec = nullptr; }
        if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
    }

    // Standard independent set of the candidates (cand == nullptr: every
    // row) into cr_st, in rounds of the greedy order until none is open.
    void independent_set(int nl, const int* rp, const int* ci, const int* cand) {
        LAUNCH(k_mis_init, nblk(nl), BAMG_BLK, s, nl, cand, cr_st);
        for (int rounds = 0;; rounds += 4) {
            if (rounds > nl + 8) fail(BAMG_EDEVICE, "independent set did not finish in %d rounds", rounds);
            zero(cr_flag + 1, 4 * sizeof(int));
            for (int b = 0; b < 4; ++b)
                LAUNCH(k_mis_round, nblk(nl), BAMG_BLK, s, nl, rp, ci, cr_st, cr_flag + 1 + b);
            if (get1(cr_flag + 4) == 0) break;
        }
    }

    // Algorithm 1 on level l: C from the independent set of all points, then
    // rounds of nu F-relaxation sweeps from random u^0 (stream STREAM_CR + l,
    // counter k n_l + i in round k); while the estimate of eq. meas1 exceeds
    // theta, an independent set of the slow points joins C.  Leaves cmap on the
    // level and returns the number of C points.
    template <typename M>
    int cr_coarsen_t(int l, const int* rp, const int* ci, const M* v) {
        auto& lv = L[l];
        const int nl = lv.rows;
        const int nb = nblk(nl);
        independent_set(nl, rp, ci, nullptr);
        LAUNCH(k_mis_take, nb, BAMG_BLK, s, nl, (const int*)cr_st, 1, cr_isc);
        lv.cr_rho.clear();
        const int rb = std::min(CR_RED_BLOCKS, nb);
        for (int k = 0; k < o.cr_rounds; ++k) {
            LAUNCH(k_cr_start, nb, BAMG_BLK, s, nl, (const int*)cr_isc, (uint64_t)o.seed, STREAM_CR + (uint64_t)l,
                   (uint64_t)k * (uint64_t)nl, cr_u0, cr_ua);
            double* a = cr_ua;
            double* b = cr_ub;
            for (int it = 0; it < o.cr_nu; ++it) {
                LAUNCH((k_cr_sweep<M>), nb, BAMG_BLK, s, nl, rp, ci, v, o.omega, (const int*)cr_isc, (const double*)a,
                       b);
                std::swap(a, b);
            }
            // a = u^nu, b = u^(nu-1)
            LAUNCH(k_cr_ssq_partial, rb, BAMG_BLK, s, nl, (const double*)cr_u0, (const double*)a, cr_part);
            LAUNCH(k_cr_ssq_final, 1, BAMG_WAVE, s, rb, (const double*)cr_part, cr_out);
            std::vector<double> q = getn(cr_out, 2);
            const double rho = q[0] > 0.0 ? std::pow(std::sqrt(q[1]) / std::sqrt(q[0]), 1.0 / o.cr_nu) : 0.0;
            lv.cr_rho.push_back(rho);
            if (!(rho > o.cr_theta)) break;
            zero(cr_flag, sizeof(int));
            LAUNCH(k_cr_cand, nb, BAMG_BLK, s, nl, (const int*)cr_isc, (const double*)b, (const double*)a,
                   o.cr_theta, cr_cand, cr_flag);
            if (get1(cr_flag) == 0) break;
            independent_set(nl, rp, ci, cr_cand);
            LAUNCH(k_mis_take, nb, BAMG_BLK, s, nl, (const int*)cr_st, 0, cr_isc);
        }
        lv.cr_rounds = (int)lv.cr_rho.size();
        scan(nl, cr_isc, cr_pos);
        const int nc = get1(cr_pos + nl);
        if (!lv.cmap) lv.cmap = A.alloc<int>(nl);
        LAUNCH(k_cr_cmap, nb, BAMG_BLK, s, nl, (const int*)cr_isc, (const int*)cr_pos, lv.cmap);
        return nc;
    }

    int cr_coarsen(int l) {
        if (l == 0) return cr_coarsen_t<double>(0, b0rp, b0ci, (const double*)b0v);
        auto& lv = L[l];
        return cr_coarsen_t<T>(l, lv.B.rp, lv.B.ci, (const T*)lv.B.v);
    }

    // Level l without a grid, reached for the first time: coarsen it while
    // l + 1 < options.levels (levels = 0: while n_l > coarse_max), adding
    // level l + 1; otherwise it is the coarsest level.
    void decide_level(int l) {
        auto& lv = L[l];
        lv.decided = true;
        const int nl = lv.rows;
        bool more = o.levels > 0 ? (l + 1 < o.levels) : (nl > o.coarse_max);
        if (more && (int)L.size() >= 63) fail(BAMG_EUNSUPPORTED, "more than 63 levels");
        if (more) {
            const int nc = cr_coarsen(l);
            if (!(nc >= 1 && nc < nl)) {
                if (o.levels > 0)
                    fail(BAMG_EUNSUPPORTED, "compatible relaxation cannot coarsen level %d (%d of %d points coarse)", l,
                         nc, nl);
                more = false;
            } else {
                add_level(l, nc);
            }
        }
        if (!more) alloc_coarsest();
    }

    void add_level(int l, int nc) {
        L.emplace_back();
        auto& lv = L[l];
        auto& c = L[l + 1];
        ChainGeo gg{};
        gg.off = 0; gg.n = nc; gg.nx = 0; gg.ny = 1; gg.periodic = 0; gg.dy = FastDiv(1u);
        gg.coff = 0; gg.cn = 0; gg.ncx = 1; gg.ncy = 1; gg.dcy = FastDiv(1u);
        c.geo = {gg};
        c.nch = 1; c.ncont = 0;
        c.rows = nc; c.cont_rows = 0;
        c.segp = ceil_div(nc, SEG_ROWS);
        c.cnp = ceil_div(nc, CN_ROWS);
        c.zero_into_e2 = ((std::max(0, o.nu_pre - 1) + o.nu_post) % 2) == 1;
        lv.ncont = 1;
        lv.cont_rows = lv.rows;
        lv.geo[0].cn = nc; lv.geo[0].coff = 0; lv.geo[0].ncx = 1; lv.geo[0].ncy = 1; lv.geo[0].dcy = FastDiv(1u);
        HIPCHK(hipMemcpyAsync(lv.dgeo, lv.geo.data(), sizeof(ChainGeo), hipMemcpyHostToDevice, s));
        chains[0].plan.push_back(GridH{nc, 1, 0});
        alloc_level(l + 1, 0);
        alloc_cont(l);
        sync();
    }

    // Interpolation and averaging restriction of a level without a grid.
    void fit_u(int l, int use_v, bool inject) {
        auto& lv = L[l];
        auto& c = L[l + 1];
        const int nl = lv.cont_rows;
        zero(err, sizeof(int) * 4);
        LAUNCH((k_ls_fit_u<T, T>), ceil_div(nl, LSU_BLK), LSU_BLK, s, nl, r, use_v ? nvc_h[0] : 0, VS,
               (const T*)lv.U, (const T*)lv.V, (const double*)wts, o.caliber, (const int*)lv.cmap,
               (const int*)lv.B.rp, (const int*)lv.B.ci, lv.pc, lv.pv, inject ? c.U : (T*)nullptr, lv.jcnt, err);
        const int e = get1(err);
        if (e & ERR_NOCOARSE) fail(BAMG_EDEVICE, "an F point of level %d has no coarse neighbour", l);
        if (e & ERR_WIDEN) fail(BAMG_EUNSUPPORTED, "a point of level %d has more than %d coarse neighbours", l, LSU_K);
        const int nc = c.rows;
        zero(lv.cnt, sizeof(int) * nc);
        LAUNCH(k_qu_count, nblk(nl), BAMG_BLK, s, nl, (const int*)lv.pc, lv.cnt);
        scan(nc, lv.cnt, lv.qrp);
        zero(lv.cnt, sizeof(int) * nc);
        LAUNCH(k_qu_fill, nblk(nl), BAMG_BLK, s, nl, (const int*)lv.pc, (const int*)lv.qrp, lv.cnt, lv.qci);
        LAUNCH((k_qu_finish<T>), nblk(nc), BAMG_BLK, s, nc, (const int*)lv.qrp, lv.qci, (const unsigned char*)lv.jcnt,
               lv.qvv);
    }

    // One row-wise product C = L R (R ELL-4 when !rcsr, else CSR) into Cm:
    // count, scan, (re)allocate when it outgrew its arrays, fill.  Returns
    // whether Cm's arrays moved.
    template <bool RCSR>
    bool rowprod(int rows, int ncols, const int* lrp, const int* lci, const T* lv, const int* rrp, const int* rci,
                 const T* rv, int* cnt, Csr<T>& Cm, const char* what) {
        zero(err, sizeof(int) * 4);
        LAUNCH((k_rowprod<T, RCSR>), rows, BAMG_WAVE, s, rows, ncols, 0, lrp, lci, lv, rrp, rci, rv, cnt,
               (const int*)nullptr, (int*)nullptr, (T*)nullptr, err);
        scan(rows, cnt, Cm.rp);
        const int tot = get1(Cm.rp + rows);
        if (get1(err) & ERR_GALCAP)
            fail(BAMG_EUNSUPPORTED, "a row of %s needs more than %d products", what, RP_CAP);
        bool moved = false;
        if (tot > Cm.cap) {
            Cm.cap = tot + tot / 4;
            Cm.ci = A.alloc<int>(Cm.cap);
            Cm.v = A.alloc<T>(Cm.cap);
            moved = true;
        }
        LAUNCH((k_rowprod<T, RCSR>), rows, BAMG_WAVE, s, rows, ncols, 1, lrp, lci, lv, rrp, rci, rv, cnt,
               (const int*)Cm.rp, Cm.ci, Cm.v, err);
        return moved;
    }

    // B_{l+1} = Q (B P), T_{l+1} = Q (T P) for a level without a grid, each
    // as W = M P, then Q W (T_0 = I: Q P).
    void galerkin_u(int l, bool profile) {
        auto& f = L[l];
        auto& c = L[l + 1];
        const int nc = c.rows, nl = f.cont_rows;
        bool moved = false;
        for (int which = 0; which < 2; ++which) {
            Csr<T>& M = which == 0 ? f.B : f.Tm;
            Csr<T>& Cm = which == 0 ? c.B : c.Tm;
            std::pair<hipEvent_t, hipEvent_t> ev;
            if (profile) ev = ev_begin();
            if (M.rp) {
                rowprod<false>(nl, nc, M.rp, M.ci, M.v, nullptr, f.pc, f.pv, itmp, Wt, "M P");
                moved |= rowprod<true>(nc, nc, f.qrp, f.qci, f.qvv, Wt.rp, Wt.ci, Wt.v, f.cnt, Cm, "Q (M P)");
            } else {
                moved |= rowprod<false>(nc, nc, f.qrp, f.qci, f.qvv, nullptr, f.pc, f.pv, f.cnt, Cm, "Q P");
            }
            if (profile) ev_end(ev, ev_gal);
        }
        zero(err, sizeof(int) * 4);
        LAUNCH(k_dinv<T>, nblk(nc), BAMG_BLK, s, nc, c.B.rp, c.B.ci, c.B.v, o.omega, c.dinv, err);
        if (moved) {
            invalidate_graph();
            if (l + 2 == (int)L.size()) refresh_coarse_desc();
        }
    }

    bool mle_level(int l, bool use_v, bool prof) {
        if (unstructured && !L[l].decided) decide_level(l);
        if (l == (int)L.size() - 1) {
            if (o.stop_after == 1) return false;
            coarsest_inverse();
            coarsest_eigs();
            return o.stop_after != 2;
        }
        sweeps(l, L[l].U, r, o.nu_setup, prof && l == 0);
        for (int m = 0; m < o.mu; ++m) {
            build_level(l, (use_v || m > 0) ? 1 : 0, true, prof && l == 0);
            if (!mle_level(l + 1, use_v, prof)) return false;
            upleg_level(l);
        }
        return true;
    }

    // MLE iteration as a stand-alone solver (Section 4.1): cycles of
    // Algorithm 3, each fitting P_l to U_l and the previous cycle's V_l, until
    // the state-vector approximation meets the tolerance; x (caller-owned,
    // length n) receives it clamped and scaled to sum one.  The handle keeps
    // the last cycle's hierarchy.
    int mle_iterate(double* x, double tol, int max_cycles, bamg_solve_info* info) override {
        auto t0 = std::chrono::steady_clock::now();
        if (nch != 1) fail(BAMG_EUNSUPPORTED, "the MLE iteration runs on single-chain handles");
        bamg_solve_info inf{};
        const int N = (int)n;
        const ChainGeo* g0 = L[0].dgeo;
        if (!rvec) rvec = A.alloc<double>(N);
        auto residual = [&]() {
            outer_spmv((const double*)x0, -1.0, rvec, RowMask{g0, nch, nullptr});
            seg_reduce<RED_ABS>(rvec, nullptr, sc + 1);
            seg_reduce<RED_ABS>(x0, nullptr, sc + 2);
            std::vector<double> h = getn(sc, (size_t)SCS);
            return h[1] / h[2];
        };
        double rel = residual();
        while (!(rel <= tol) && inf.cycles < max_cycles) {
            mle_level(0, true, false);
            state_from_v();
            ++inf.cycles;
            rel = residual();
            if (inf.history_len < 256) inf.history[inf.history_len++] = rel;
            if (!(rel == rel)) fail(BAMG_EDEVICE, "MLE iteration: non-finite residual");
        }
        HIPCHK(hipMemcpyAsync(x, x0, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        seg_reduce<RED_NEGSUM>(x, nullptr, sc + 5);
        LAUNCH(k_clamp, nblk(N), BAMG_BLK, s, N, x);
        seg_reduce<RED_SUM>(x, nullptr, sc);
        LAUNCH(k_seg_scale, nblk(N), BAMG_BLK, s, N, g0, nch, (const int*)nullptr, (const double*)x,
               (const double*)nullptr, (const double*)sc, SCS, 0, x);
        outer_spmv((const double*)x, -1.0, rvec, RowMask{g0, nch, nullptr});
        seg_reduce<RED_ABS>(rvec, nullptr, sc + 1);
        seg_reduce<RED_ABS>(x, nullptr, sc + 2);
        std::vector<double> h = getn(sc, (size_t)SCS);
        inf.residual_l1 = h[1] / h[2];
        inf.clamped_mass = h[5];
        inf.converged = inf.residual_l1 <= tol;
        st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return inf.converged ? BAMG_OK : BAMG_ENOCONV;
    }

    void setup(const int32_t* rp, const int32_t* ci, const double* val) override {
        auto t0 = std::chrono::steady_clock::now();
        A.s = s;
        A.budget = o.mem_budget;
        int hr[2];
        HIPCHK(hipMemcpyAsync(&hr[0], rp, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hr[1], rp + n, sizeof(int), hipMemcpyDeviceToHost, s));
        sync();
        if (hr[0] != 0 || hr[1] < 0) fail(BAMG_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] >= 0");
        const int nnzA = hr[1];
        unstructured = nch == 1 && chains[0].grid.nx == 0;
        L.reserve(64);                   // levels are added in place while coarsening
        plan_levels();
        allocate(nnzA);
        if (nch > 1) reorder_input(rp, ci, val, nnzA);
        build_b0(rp, ci, val, nnzA);
        if (unstructured) check_symmetric();
        check_colours(0);
        const bool prof = o.profile != 0;
        {
            long long tot = (long long)n * r;
            LAUNCH(k_tv_init<T>, nblk(tot), BAMG_BLK, s, tot, r, FastDiv((uint32_t)r), (const ChainGeo*)L[0].dgeo,
                   L[0].nch, o.seed, L[0].U);
        }
        // one cycle of Algorithm 3 from the random test vectors
        if (!mle_level(0, false, prof)) { finish_setup(t0); return; }
        state_from_v();
        if (o.stop_after == 3 || o.setup_passes == 1) { finish_setup(t0); return; }
        // recompute every P, B, T from U u V
        const int depth = (int)L.size();
        for (int l = 0; l + 1 < depth; ++l) build_level(l, 1, false, prof && l == 0);
        coarsest_inverse();
        finish_setup(t0);
    }

    void finish_setup(std::chrono::steady_clock::time_point t0) {
        sync();
        check_pivot();
        st.t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st.n_levels = (int)L.size();
        st.n_v = nvmax;
        // every level's nnz(B) and the deferred error flags in one read-back
        const int nl = (int)L.size();
        for (int l = 0; l < nl; ++l) LAUNCH(k_copy_int, 1, BAMG_WAVE, s, (const int*)(L[l].B.rp + L[l].rows), gath + l);
        LAUNCH(k_copy_int, 1, BAMG_WAVE, s, (const int*)derr, gath + nl);
        const bool t1 = nl > 1 && L[1].Tm.rp;
        if (t1) LAUNCH(k_copy_int, 1, BAMG_WAVE, s, (const int*)(L[1].Tm.rp + L[1].rows), gath + nl + 1);
        std::vector<int> g = getn(gath, (size_t)nl + (t1 ? 2 : 1));
        if (g[nl]) fail(BAMG_EDEVICE, "a coarse grid operator has a row outside the 3 x 3 box");
        long long tot = 0;
        for (int l = 0; l < nl; ++l) tot += g[l];
        st.op_complexity = nnz0 > 0 ? (double)tot / nnz0 : 0.0;
        auto acc = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, double& ms, int& cnt) {
            ms = 0; cnt = 0;
            for (auto& p : v) {
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, p.first, p.second));
                ms += t; ++cnt;
                event_pool().put(p.first); event_pool().put(p.second);
            }
            v.clear();
        };
        acc(ev_sweep, st.sweep_ms, st.sweep_launches);
        st.tune_ms = sweep_tuner().tune_ms;
        if (learn_acc) {
            std::vector<double> la = getn(learn_acc, 2);
            st.mlp_points = (int64_t)la[0];
            st.mlp_fallback = (int64_t)la[1];
        }
        acc(ev_gal, st.galerkin_ms, st.galerkin_launches);
        acc(ev_gal_csr, st.gal_csr_ms, st.gal_csr_launches);
        acc(ev_ls, st.lsfit_ms, st.lsfit_launches);
        acc(ev_ls2, st.lsfit2_ms, st.lsfit2_launches);
        acc(ev_gj, st.dense_update_ms, st.dense_update_launches);
        st.dense_update_flops = gj_flops;
        gj_flops = 0;
        // algorithmic bytes of one level-0 launch
        const long long n0 = L[0].cont_rows;
        const int vb = sizeof(T);
        // (one Gauss-Seidel sweep over all colours moves the same data except
        // D^-1, whose diagonal it takes from the rows)
        st.sweep_bytes = (long long)(n0 + 1) * 4 + (long long)nnz0 * (4 + vb) + (mcgs ? 0 : n0 * vb) +
                         2LL * n0 * r * vb;
        st.sweep_ell = L[0].B.eci ? 1 : 0;
        if (L[0].B.eci && !mcgs)         // the ELL-4 copy: 4 entries per row, no row pointers
            st.sweep_bytes = 4LL * n0 * (4 + vb) + n0 * vb + 2LL * n0 * r * vb;
        if (L.size() > 1 && !unstructured) {
            // every array once (neighbour re-reads served from cache): Q
            // (ELL-9 columns and values), B_0's rows (ELL-4 copy or CSR),
            // P (ELL-4); written: both products' ELL-9 arrays and row
            // counts.  The CSR step reads the row pointers and the stored
            // entries of both ELL-9 copies and writes them as CSR.
            const long long nc = L[1].rows, nnzb1 = g[1];
            const long long nnzt1 = t1 ? g[nl + 1] : 0;
            const long long q = nc * 9 * (4 + vb), pb = n0 * 4 * (4 + vb);
            const long long brows = L[0].B.eci ? 4LL * n0 * (4 + vb) : (n0 + 1) * 4 + (long long)nnz0 * (4 + vb);
            st.galerkin_bytes = q + brows + pb + 2 * nc * 9 * (4 + vb) + 2 * nc * 4;
            st.gal_csr_bytes = 2 * (nc + 1) * 4 + 2 * (nnzb1 + nnzt1) * (4 + vb);
            // the fit reads the test vectors, writes P (ELL-4) and |J_i|;
            // the first pass also injects U on the coarse points
            st.lsfit_bytes = n0 * (long long)r * vb + pb + n0 + nc * (long long)r * vb;
            st.lsfit2_bytes = n0 * (long long)(r + nvmax) * vb + pb + n0;
        }
    }

    // y = alpha * B_0 x in FP64 (the outer iteration), on the ELL-4 copy when
    // there is one.
    void outer_spmv(const double* x, double alpha, double* y, const RowMask& mk) {
        const int N = (int)n;
        if (b0ev)
            LAUNCH(k_spmv_e<double>, nblk(N), BAMG_BLK, s, N, (const int*)L[0].B.eci, (const double*)b0ev, x, alpha, y,
                   mk);
        else
            LAUNCH(k_spmv<double>, nblk(N), BAMG_BLK, s, N, b0rp, b0ci, (const double*)b0v, x, alpha, y, mk);
    }

    // -------------------------------------------------------------- cycle
    // One smoothing sweep of the cycle on level lv: e_out = e + D^-1 (f - B e).
    void cycle_sweep(Level<T>& lv, int rows, int nb, const T* cur, T* oth, const RowMask& mk) {
        if (lv.B.cci)
            LAUNCH((k_sweep_c9<T, T>), nb, BAMG_BLK, s, rows, lv.rows, (const int*)lv.B.cci, (const T*)lv.B.cv,
                   (const T*)lv.dinv, cur, (const T*)lv.f, oth, mk);
        else if (lv.B.eci)
            LAUNCH((k_sweep_e<T, T>), nb, BAMG_BLK, s, rows, (const int*)lv.B.eci, (const T*)lv.B.ev,
                   (const T*)lv.dinv, cur, (const T*)lv.f, oth, mk);
        else
            LAUNCH((k_sweep<T, T>), nb, BAMG_BLK, s, rows, 1, FastDiv(1u), lv.B.rp, lv.B.ci, (const T*)lv.B.v,
                   (const T*)lv.dinv, cur, (const T*)lv.f, oth, mk);
    }

    // e_l = C f_l on level l, result in lv.e (fixed buffers, so that the
    // cycle can be replayed from a graph).  Continuing chains smooth and
    // recurse; chains whose coarsest level is l take the minimal-norm solve.
    void vcycle(int l) {
        auto& lv = L[l];
        if (lv.nch > lv.ncont) {
            const int c0 = lv.ncont, c1 = lv.nch;
            int maxn = 0;
            for (int c = c0; c < c1; ++c) maxn = std::max(maxn, cdh[c].n);
            const dim3 gw(ceil_div(maxn, 4), c1 - c0);
            const int* am = cmask ? cmask + c0 : nullptr;
            if (MIXED)
                hipLaunchKernelGGL(k_cz_gemv_f32, gw, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)(cd + c0),
                                   (const float*)Wfp, (const float*)lv.f, (float*)lv.e, am);
            else
                hipLaunchKernelGGL(k_cz_gemv_rows, gw, dim3(BAMG_BLK), 0, s, (const CoarseDesc*)(cd + c0),
                                   (const double*)Wp, (const double*)lv.f, (double*)lv.e, am);
            HIPCHK(hipGetLastError());
        }
        if (lv.ncont == 0) return;
        auto& c = L[l + 1];
        const int rows = lv.cont_rows;
        T* cur = lv.zero_into_e2 ? lv.e2 : lv.e;
        T* oth = lv.zero_into_e2 ? lv.e : lv.e2;
        const int nb = nblk(rows);
        const RowMask mk{lv.dgeo, lv.ncont, cmask};     // continuing chains' rows
        auto gs_sweeps = [&](int nu) {
            for (int k = 0; k < nu; ++k)
                for (int cc = 0; cc < ncol; ++cc)
                    LAUNCH((k_mcgs<T, T>), nb, BAMG_BLK, s, rows, (const ChainGeo*)lv.dgeo, lv.ncont, cc, o.gs_omega,
                           lv.B.rp, lv.B.ci, (const T*)lv.B.v, (const T*)lv.f, cur, mk);
        };
        if (mcgs) {
            // in place from e = 0
            cur = lv.e;
            LAUNCH((k_fill_t<T>), nb, BAMG_BLK, s, rows, cur, mk);
            gs_sweeps(o.nu_pre);
        } else if (o.nu_pre > 0) {
            int k = 1;
            if (o.nu_pre >= 2 && (lv.B.cci || lv.B.eci)) {
                // the zero-guess sweep and the next one in one pass, into the
                // buffer the second would write
                if (lv.B.cci)
                    LAUNCH((k_sweep2z_c9<T, T>), nb, BAMG_BLK, s, rows, lv.rows, (const int*)lv.B.cci,
                           (const T*)lv.B.cv, (const T*)lv.dinv, (const T*)lv.f, oth, mk);
                else
                    LAUNCH((k_sweep2z_e<T, T>), nb, BAMG_BLK, s, rows, (const int*)lv.B.eci, (const T*)lv.B.ev,
                           (const T*)lv.dinv, (const T*)lv.f, oth, mk);
                std::swap(cur, oth);
                k = 2;
            } else {
                LAUNCH((k_jacobi_zero<T, T>), nb, BAMG_BLK, s, rows, (const T*)lv.dinv, (const T*)lv.f, cur, mk);
            }
            for (; k < o.nu_pre; ++k) {
                cycle_sweep(lv, rows, nb, cur, oth, mk);
                std::swap(cur, oth);
            }
        } else {
            LAUNCH((k_fill_t<T>), nb, BAMG_BLK, s, rows, cur, mk);
        }
        if (lv.B.cci)
            LAUNCH((k_residual_c9<T, T>), nb, BAMG_BLK, s, rows, lv.rows, (const int*)lv.B.cci, (const T*)lv.B.cv,
                   (const T*)cur, (const T*)lv.f, lv.r, mk);
        else if (lv.B.eci)
            LAUNCH((k_residual_e<T, T>), nb, BAMG_BLK, s, rows, (const int*)lv.B.eci, (const T*)lv.B.ev,
                   (const T*)cur, (const T*)lv.f, lv.r, mk);
        else
            LAUNCH((k_residual<T, T>), nb, BAMG_BLK, s, rows, lv.B.rp, lv.B.ci, (const T*)lv.B.v, (const T*)cur,
                   (const T*)lv.f, lv.r, mk);
        if (unstructured)
            LAUNCH(k_restrict_csr<T>, nblk(c.rows), BAMG_BLK, s, c.rows, (const int*)lv.qrp, (const int*)lv.qci,
                   (const T*)lv.qvv, (const T*)lv.r, c.f);
        else
            LAUNCH(k_restrict_box<T>, nblk(c.rows), BAMG_BLK, s, c.rows, (const ChainGeo*)c.dgeo,
                   (const ChainGeo*)lv.dgeo, c.nch, (const unsigned short*)lv.qmask, (const unsigned char*)lv.jcnt,
                   (const T*)lv.r, c.f, (const int*)cmask);
        vcycle(l + 1);
        int k = 0;
        if (lv.B.cci && rows <= FUSE_ROWS && !mcgs && o.nu_post >= 1 && cycle_fuse_on()) {
            // the prolongation and the first post-smoothing sweep in one pass
            // (on small levels, where a launch costs more than recomputing
            // the neighbours' prolongation)
            LAUNCH((k_prolong_sweep_c9<T, T>), nb, BAMG_BLK, s, rows, lv.rows, (const int*)lv.B.cci,
                   (const T*)lv.B.cv, (const T*)lv.dinv, lv.pc, (const T*)lv.pv, (const T*)c.e, (const T*)cur,
                   (const T*)lv.f, oth, mk);
            std::swap(cur, oth);
            k = 1;
        } else {
            LAUNCH((k_prolong_add<T, T>), nb, BAMG_BLK, s, rows, lv.pc, (const T*)lv.pv, (const T*)c.e, cur, mk);
        }
        if (mcgs) {
            gs_sweeps(o.nu_post);
            return;
        }
        for (; k < o.nu_post; ++k) {
            cycle_sweep(lv, rows, nb, cur, oth, mk);
            std::swap(cur, oth);
        }
        if (cur != lv.e) fail(BAMG_EDEVICE, "cycle buffer parity");
    }

    // One cycle from L[0].f into L[0].e, replayed from a captured graph.
    // How a cycle is issued: options.cycle_mode 1 = eager launches, 2 = one
    // captured graph replayed per cycle, 0 = decide on the first cycle: it
    // runs eagerly, timed on the host (launch cost) and on the stream (GPU
    // time); the graph is used when launching takes longer than the GPU
    // time, i.e. when the cycle is launch-bound (small chains, coarse
    // levels).  Otherwise eager launches stay ahead of the GPU and the graph's
    // capture and instantiation (a few hundred microseconds per handle) would
    // not pay back.
    void run_cycle() {
        if (!cycle_decided) {
            cycle_decided = true;
            if (o.cycle_mode == 1 || o.cycle_mode == 2) {
                use_graph = o.cycle_mode == 2;
            } else {
                hipEvent_t a, b;
                a = event_pool().get();
                b = event_pool().get();
                HIPCHK(hipEventRecord(a, s));
                auto t0 = std::chrono::steady_clock::now();
                vcycle(0);
                const double host_us =
                    std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
                HIPCHK(hipEventRecord(b, s));
                HIPCHK(hipEventSynchronize(b));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, a, b));
                event_pool().put(a);
                event_pool().put(b);
                st.cycle_host_us = host_us;
                st.cycle_gpu_us = 1e3 * ms;
                use_graph = host_us > 1e3 * ms;
                st.cycle_graph = use_graph ? 1 : 0;
                return;                          // this cycle has run
            }
            st.cycle_graph = use_graph ? 1 : 0;
        }
        if (!use_graph) {
            vcycle(0);
            return;
        }
        if (!gexec) {
            // Record the launches of one cycle on a private stream (nothing
            // runs during capture), then replay the graph on the handle's
            // stream, which may be the legacy default stream.
            if (!cap_s) HIPCHK(hipStreamCreateWithFlags(&cap_s, hipStreamNonBlocking));
            hipStream_t user = s;
            s = cap_s;
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                vcycle(0);
            } catch (...) {
                hipGraph_t gtmp = nullptr;
                (void)hipStreamEndCapture(s, &gtmp);
                if (gtmp) (void)hipGraphDestroy(gtmp);
                s = user;
                throw;
            }
            const hipError_t ec = hipStreamEndCapture(s, &graph);
            s = user;
            HIPCHK(ec);
            HIPCHK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(gexec, s));
    }

    // z = C v for FP64 finest-level vectors.
    void precondition(const double* v, double* z) {
        auto& l0 = L[0];
        if (MIXED) LAUNCH(k_d2f, nblk(n), BAMG_BLK, s, (int)n, v, (float*)l0.f);
        else LAUNCH(k_copy, nblk(n), BAMG_BLK, s, (long long)n, v, (double*)l0.f);
        run_cycle();
        if (MIXED) LAUNCH(k_f2d, nblk(n), BAMG_BLK, s, (int)n, (const float*)l0.e, z);
        else LAUNCH(k_copy, nblk(n), BAMG_BLK, s, (long long)n, (const double*)l0.e, z);
    }

    // Caller's chain order in and out (the handle's rows are depth-sorted).
    void vcycle_apply(const double* f, double* e) override {
        if (cmask) {
            std::vector<int> ones(nch, 1);
            HIPCHK(hipMemcpyAsync(cmask, ones.data(), sizeof(int) * nch, hipMemcpyHostToDevice, s));
            sync();
        }
        if (!reordered) {
            precondition(f, e);
        } else {
            if (!vin) { vin = A.alloc<double>(n); vout = A.alloc<double>(n); }
            const dim3 gp(nblk(n), nch);
            hipLaunchKernelGGL(k_seg_permute, gp, dim3(BAMG_BLK), 0, s, (const int*)perm_src, (const int*)perm_dst,
                               (const int*)perm_len, f, vin);
            HIPCHK(hipGetLastError());
            precondition(vin, vout);
            hipLaunchKernelGGL(k_seg_permute, gp, dim3(BAMG_BLK), 0, s, (const int*)perm_dst, (const int*)perm_src,
                               (const int*)perm_len, (const double*)vout, e);
            HIPCHK(hipGetLastError());
        }
        sync();
    }

    // -------------------------------------------------------------- solve
    // Flexible GMRES(m) on B x = 0 for every chain at once: vectors are the
    // concatenated finest rows; dot products, Hessenberg matrices and the
    // convergence decisions are per chain.  A chain whose inner iteration has
    // stopped is masked until the restart.
    // Multigrid-preconditioned Arnoldi (Section 4.3) in lockstep over the
    // chains: Arnoldi on C B from the (normalised) iterate, after each step
    // the Ritz vector of the eigenvalue of H_j closest to 0, scaled to sum
    // one, becomes the iterate of every active chain; a chain stops when its
    // ||B x||_1 / ||x||_1 <= tol or its Krylov space breaks down; the others
    // restart from their Ritz vector after m steps.
    void parnoldi_loop(double* xi, double tol, int max_cycles, bamg_solve_info& inf) {
        const int m = std::max(1, o.gmres_m);
        const int N = (int)n;
        const int ld = m + 1, HSg = (m + 1) * m, GS = m + 2;
        const int nb = nblk(N);
        const ChainGeo* g0 = L[0].dgeo;
        if (!hfail) hfail = A.alloc<int>(nch);
        std::vector<int> hact(nch, 1), hkd(nch, 0), done(nch, 0);
        auto residuals = [&](std::vector<double>& rel, std::vector<double>& nu) {
            outer_spmv((const double*)xi, -1.0, rvec, RowMask{g0, nch, nullptr});
            seg_reduce<RED_ABS>(rvec, nullptr, sc + 1);
            seg_reduce<RED_ABS>(xi, nullptr, sc + 2);
            std::vector<double> h = getn(sc, (size_t)nch * SCS);
            double worst = 0;
            for (int c = 0; c < nch; ++c) {
                rel[c] = h[(size_t)c * SCS + 1] / h[(size_t)c * SCS + 2];
                nu[c] = h[(size_t)c * SCS + 6];
                worst = std::max(worst, rel[c]);
            }
            return worst;
        };
        std::vector<double> rel(nch), nu(nch, 1.0);
        {
            const double w = residuals(rel, nu);
            inf.residual_l1 = w;
            if (inf.history_len < 256) inf.history[inf.history_len++] = w;
            for (int c = 0; c < nch; ++c) done[c] = rel[c] <= tol;
        }
        for (;;) {
            bool any = false;
            for (int c = 0; c < nch; ++c) { hact[c] = !done[c]; any |= (bool)hact[c]; }
            if (!any || inf.cycles >= max_cycles) break;
            HIPCHK(hipMemcpyAsync(act, hact.data(), sizeof(int) * nch, hipMemcpyHostToDevice, s));
            // v_0 = x / ||x||_2
            seg_reduce<RED_DOT>(xi, xi, sc + 3);
            LAUNCH(k_seg_scale, nb, BAMG_BLK, s, N, g0, nch, (const int*)nullptr, (const double*)xi,
                   (const double*)nullptr, (const double*)(sc + 3), SCS, 1, Vk);
            zero(Hg, sizeof(double) * nch * HSg);
            for (int j = 0; j < m && inf.cycles < max_cycles; ++j) {
                // w = C (B v_j)
                outer_spmv((const double*)(Vk + (size_t)j * vld), 1.0, rvec, RowMask{g0, nch, act});
                precondition(rvec, wk);
                ++inf.cycles;
                const int P0 = L[0].segp;
                const dim3 gsg(P0, nch);
                gs_dispatch(j, [&](auto kc) {
                    hipLaunchKernelGGL((k_gs_dots<decltype(kc)::value, false>), gsg, dim3(BAMG_BLK), 0, s, g0, SEG_ROWS,
                                       vld, j, (const int*)act, (const double*)Vk, (const double*)wk, part, GS,
                                       (const int*)nullptr, (const double*)nullptr, (const double*)nullptr, 1.0,
                                       (double*)nullptr);
                });
                hipLaunchKernelGGL(k_gs_final, dim3(j + 2, nch), dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, P0,
                                   (const int*)act, (const double*)part, GS, hbuf, GS);
                HIPCHK(hipGetLastError());
                LAUNCH(k_arn_step, ceil_div(nch, 64), 64, s, nch, j, ld, (const int*)act, (const double*)hbuf2,
                       (const double*)hbuf, GS, Hg, HSg, gsaux, GS, gscoef, sc + 6, SCS);
                // Ritz vector of the eigenvalue of H_{j+1} closest to 0
                LAUNCH(k_hess_near0, nch, BAMG_WAVE, s, j + 1, (const int*)act, (const double*)Hg, HSg, ld, ysol, GS,
                       hfail);
                for (int c = 0; c < nch; ++c) hkd[c] = j + 1;
                HIPCHK(hipMemcpyAsync(kd, hkd.data(), sizeof(int) * nch, hipMemcpyHostToDevice, s));
                LAUNCH(k_seg_ritz, nb, BAMG_BLK, s, N, vld, g0, nch, (const int*)act, (const int*)kd,
                       (const double*)Vk, (const double*)ysol, GS, xi);
                // sum one, on the chains that moved only (the others keep their bits)
                seg_reduce<RED_SUM>(xi, nullptr, sc);
                LAUNCH(k_seg_scale, nb, BAMG_BLK, s, N, g0, nch, (const int*)act, (const double*)xi,
                       (const double*)nullptr, (const double*)sc, SCS, 0, xi);
                const double w = residuals(rel, nu);
                inf.residual_l1 = w;
                if (inf.history_len < 256) inf.history[inf.history_len++] = w;
                bool cont = false;
                for (int c = 0; c < nch; ++c) {
                    if (!hact[c]) continue;
                    if (rel[c] <= tol || !(rel[c] == rel[c])) { done[c] = 1; hact[c] = 0; }
                    else if (nu[c] == 0.0) hact[c] = 0;     // invariant subspace: restart
                    cont |= (bool)hact[c];
                }
                if (!cont || j + 1 >= m || inf.cycles >= max_cycles) break;
                HIPCHK(hipMemcpyAsync(act, hact.data(), sizeof(int) * nch, hipMemcpyHostToDevice, s));
                gs_dispatch(j, [&](auto kc) {
                    hipLaunchKernelGGL(k_gs_update<decltype(kc)::value>, gsg, dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, vld,
                                       j, (const int*)act, Vk, (const double*)wk, (const double*)gscoef, part, GS);
                });
                hipLaunchKernelGGL(k_gs_final, dim3(j + 2, nch), dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, P0,
                                   (const int*)act, (const double*)part, GS, hbuf2, GS);
                HIPCHK(hipGetLastError());
            }
            ++inf.restarts;
            for (int c = 0; c < nch; ++c)
                if (!(rel[c] == rel[c])) fail(BAMG_EDEVICE, "preconditioned Arnoldi: non-finite residual (chain %d)", c);
        }
    }

    int solve(double* x, double tol, int max_cycles, uint32_t flags, int32_t* status, double* resid,
              bamg_solve_info* info) override {
        auto t0 = std::chrono::steady_clock::now();
        const int m = std::max(1, o.gmres_m);
        const int N = (int)n;
        const int ld = m + 1;
        const int HSg = (m + 1) * m, GS = m + 2;
        if (m_alloc != m) {
            vld = basis_stride(N);
            Vk = A.alloc<double>((size_t)(m + 1) * vld);
            Zk = A.alloc<double>((size_t)m * vld);
            wk = A.alloc<double>(N);
            rvec = A.alloc<double>(N);
            Hg = A.alloc<double>((size_t)nch * HSg);
            cs = A.alloc<double>((size_t)nch * GS);
            sn = A.alloc<double>((size_t)nch * GS);
            g = A.alloc<double>((size_t)nch * GS);
            ysol = A.alloc<double>((size_t)nch * GS);
            hbuf = A.alloc<double>((size_t)nch * GS);
            hbuf2 = A.alloc<double>((size_t)nch * GS);
            gsaux = A.alloc<double>((size_t)nch * 3 * GS);
            gscoef = A.alloc<double>((size_t)nch * GS_CS);
            est = A.alloc<double>(nch);
            act = cmask;
            itol_d = A.alloc<double>(nch);
            if (!hflag) {
                HIPCHK(hipHostMalloc((void**)&hflag, sizeof(int) * 2 * nch, hipHostMallocDefault));
                fev[0] = event_pool().get();
                fev[1] = event_pool().get();
            }
            kd = A.alloc<int>(nch);
            if (reordered) xperm = A.alloc<double>(N);
            m_alloc = m;
        }
        double* xi = reordered ? xperm : x;
        bamg_solve_info inf{};
        if (!(flags & BAMG_USE_GUESS)) {
            HIPCHK(hipMemcpyAsync(xi, x0, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        } else if (reordered) {
            hipLaunchKernelGGL(k_seg_permute, dim3(nblk(N), nch), dim3(BAMG_BLK), 0, s, (const int*)perm_src,
                               (const int*)perm_dst, (const int*)perm_len, (const double*)x, xi);
            HIPCHK(hipGetLastError());
        }
        const ChainGeo* g0 = L[0].dgeo;
        auto normalise = [&]() {
            seg_reduce<RED_SUM>(xi, nullptr, sc);
            LAUNCH(k_seg_scale, nblk(N), BAMG_BLK, s, N, g0, nch, (const int*)nullptr, (const double*)xi,
                   (const double*)nullptr, (const double*)sc, SCS, 0, xi);
        };
        normalise();
        const int nb = nblk(N);
        std::vector<int> conv(nch, 0), hact(nch);
        std::vector<double> rel(nch, 0.0);
        if (flags & BAMG_PARNOLDI) {
            parnoldi_loop(xi, tol, max_cycles, inf);
        } else {
            for (;;) {
                // r = -B x; per-chain relative 1-norm residual
                outer_spmv((const double*)xi, -1.0, rvec, RowMask{g0, nch, nullptr});
                seg_reduce<RED_ABS>(rvec, nullptr, sc + 1);
                seg_reduce<RED_ABS>(xi, nullptr, sc + 2);
                seg_reduce<RED_DOT>(rvec, rvec, sc + 3);
                std::vector<double> h = getn(sc, (size_t)nch * SCS);
                bool all = true, nan = false;
                double worst = 0;
                for (int c = 0; c < nch; ++c) {
                    rel[c] = h[(size_t)c * SCS + 1] / h[(size_t)c * SCS + 2];
                    conv[c] = rel[c] <= tol;
                    all &= (bool)conv[c];
                    nan |= !(rel[c] == rel[c]);
                    worst = std::max(worst, rel[c]);
                }
                inf.residual_l1 = worst;
                if (inf.history_len < 256) inf.history[inf.history_len++] = worst;
                if (all || inf.cycles >= max_cycles || nan) break;
                // inner iteration for the unconverged chains
                std::vector<double> itol(nch);
                for (int c = 0; c < nch; ++c) {
                    double r1 = h[(size_t)c * SCS + 1], x1 = h[(size_t)c * SCS + 2], b2 = h[(size_t)c * SCS + 3];
                    itol[c] = 0.5 * tol * x1 * std::sqrt(b2) / r1;
                    hact[c] = conv[c] ? 0 : 1;
                }
                HIPCHK(hipMemcpyAsync(act, hact.data(), sizeof(int) * nch, hipMemcpyHostToDevice, s));
                HIPCHK(hipMemcpyAsync(itol_d, itol.data(), sizeof(double) * nch, hipMemcpyHostToDevice, s));
                zero(kd, sizeof(int) * nch);
                zero(Hg, sizeof(double) * nch * HSg);
                LAUNCH(k_seg_gmres_init, nch, 64, s, nch, m, (const double*)(sc + 3), SCS, g, GS);
                LAUNCH(k_seg_scale, nb, BAMG_BLK, s, N, g0, nch, (const int*)nullptr, (const double*)rvec,
                       (const double*)nullptr, (const double*)(sc + 3), SCS, 1, Vk);
                for (int j = 0; j < m && inf.cycles < max_cycles; ++j) {
                    double* vj = Vk + (size_t)j * vld;
                    double* zj = Zk + (size_t)j * vld;
                    // once most chains have stopped, the masked cycle is little
                    // work in many launches: replay it from a graph instead
                    if (nch > 1 && o.cycle_mode == 0 && cycle_decided && !use_graph) {
                        long long act_rows = 0;
                        for (int c = 0; c < nch; ++c) act_rows += hact[c] ? chains[c].n : 0;
                        if (4 * act_rows < n) { use_graph = true; st.cycle_graph = 1; }
                    }
                    precondition(vj, zj);
                    ++inf.cycles;
                    // w = B z_j, then Gram-Schmidt with the delayed second
                    // pass: dots of w, the per-chain step (finish v_j, correct
                    // column j-1, column j, Givens), and, for chains that go
                    // on, the update pass that finishes q_j and makes v_{j+1}
                    // with its dots.  With the ELL-4 copy of B_0 the product
                    // is formed inside the dots pass.
                    const int P0 = L[0].segp;
                    const dim3 gsg(P0, nch);
                    if (!b0ev) outer_spmv((const double*)zj, 1.0, wk, RowMask{g0, nch, cmask});
                    gs_dispatch(j, [&](auto kc) {
                        constexpr int K = decltype(kc)::value;
                        if (b0ev)
                            hipLaunchKernelGGL((k_gs_dots<K, true>), gsg, dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, vld, j,
                                               (const int*)act, (const double*)Vk, (const double*)nullptr, part, GS,
                                               (const int*)L[0].B.eci, (const double*)b0ev, (const double*)zj, 1.0,
                                               wk);
                        else
                            hipLaunchKernelGGL((k_gs_dots<K, false>), gsg, dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, vld,
                                               j, (const int*)act, (const double*)Vk, (const double*)wk, part, GS,
                                               (const int*)nullptr, (const double*)nullptr, (const double*)nullptr,
                                               1.0, (double*)nullptr);
                    });
                    hipLaunchKernelGGL(k_gs_final, dim3(j + 2, nch), dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, P0,
                                       (const int*)act, (const double*)part, GS, hbuf, GS);
                    HIPCHK(hipGetLastError());
                    // the step also records kd = j + 1 and clears act[c] once the
                    // estimate |g_{j+1}| reaches itol (or 0: a breakdown), on the
                    // device, so every later kernel skips that chain
                    LAUNCH(k_gs_step, ceil_div(nch, 64), 64, s, nch, j, ld, act, (const double*)hbuf2,
                           (const double*)hbuf, GS, Hg, HSg, cs, sn, g, gsaux, GS, gscoef, est,
                           (const double*)itol_d, kd);
                    HIPCHK(hipMemcpyAsync(hflag + (j & 1) * nch, act, sizeof(int) * nch, hipMemcpyDeviceToHost, s));
                    HIPCHK(hipEventRecord(fev[j & 1], s));
                    const bool more = j + 1 < m && inf.cycles < max_cycles;
                    if (more) {
                        gs_dispatch(j, [&](auto kc) {
                            hipLaunchKernelGGL(k_gs_update<decltype(kc)::value>, gsg, dim3(BAMG_BLK), 0, s, g0,
                                               SEG_ROWS, vld, j, (const int*)act, Vk, (const double*)wk,
                                               (const double*)gscoef, part, GS);
                        });
                        hipLaunchKernelGGL(k_gs_final, dim3(j + 2, nch), dim3(BAMG_BLK), 0, s, g0, SEG_ROWS, P0,
                                           (const int*)act, (const double*)part, GS, hbuf2, GS);
                        HIPCHK(hipGetLastError());
                    }
                    // the flags of step j - 1, whose work finished while this
                    // step's was queued: with no chain left, step j ran on
                    // masked kernels only and does not count
                    if (j >= 1) {
                        HIPCHK(hipEventSynchronize(fev[(j - 1) & 1]));
                        bool any = false;
                        for (int c = 0; c < nch; ++c) {
                            hact[c] = hflag[((j - 1) & 1) * nch + c];
                            any |= (bool)hact[c];
                        }
                        if (!any) { --inf.cycles; break; }
                    }
                    if (!more) break;
                }
                LAUNCH(k_seg_gmres_y, ceil_div(nch, 64), 64, s, nch, ld, (const int*)kd, (const double*)Hg, HSg,
                       (const double*)g, GS, ysol);
                LAUNCH(k_seg_xupdate, nb, BAMG_BLK, s, N, vld, g0, nch, (const int*)kd, (const double*)Zk,
                       (const double*)ysol, GS, xi);
                normalise();
                ++inf.restarts;
            }
        }
        // the cycle works on every chain again outside the solve
        HIPCHK(hipMemcpyAsync(cmask, ones_d, sizeof(int) * nch, hipMemcpyDeviceToDevice, s));
        // x >= 0, sum 1 per chain
        seg_reduce<RED_NEGSUM>(xi, nullptr, sc + 5);
        LAUNCH(k_clamp, nb, BAMG_BLK, s, N, xi);
        normalise();
        outer_spmv((const double*)xi, -1.0, rvec, RowMask{g0, nch, nullptr});
        seg_reduce<RED_ABS>(rvec, nullptr, sc + 1);
        seg_reduce<RED_ABS>(xi, nullptr, sc + 2);
        if (reordered) {
            // back to the caller's order (source and destination swapped)
            hipLaunchKernelGGL(k_seg_permute, dim3(nblk(N), nch), dim3(BAMG_BLK), 0, s, (const int*)perm_dst,
                               (const int*)perm_src, (const int*)perm_len, (const double*)xi, x);
            HIPCHK(hipGetLastError());
        }
        std::vector<double> h = getn(sc, (size_t)nch * SCS);
        double worst = 0, cm = 0;
        bool all = true;
        for (int c = 0; c < nch; ++c) {
            double rc = h[(size_t)c * SCS + 1] / h[(size_t)c * SCS + 2];
            worst = std::max(worst, rc);
            cm = std::max(cm, h[(size_t)c * SCS + 5]);
            all &= rc <= tol;
            const int u = chains[c].uidx;
            if (status) status[u] = rc <= tol ? 1 : 0;
            if (resid) resid[u] = rc;
        }
        inf.residual_l1 = worst;
        inf.clamped_mass = cm;
        inf.converged = all;
        st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return all ? BAMG_OK : BAMG_ENOCONV;
    }

    // -------------------------------------------------------------- inspection
    void level_info(int l, bamg_level_info* out) override {
        if (l < 0 || l >= (int)L.size()) fail(BAMG_EINVAL, "level %d out of range", l);
        auto& lv = L[l];
        memset(out, 0, sizeof *out);
        out->n = lv.rows;
        out->nx = lv.geo[0].nx; out->ny = unstructured ? 0 : lv.geo[0].ny; out->periodic = lv.geo[0].periodic;
        out->cr_rounds = lv.cr_rounds;
        out->nnz_b = get1(lv.B.rp + lv.rows);
        if (lv.Tm.rp) out->nnz_t = get1(lv.Tm.rp + lv.rows);
        if (lv.pc) out->nnz_p = 4LL * lv.cont_rows;
        out->r = r;
        out->n_v = nvmax;
    }

    template <typename X>
    void copy_out(const X* src, size_t count, void* dst, size_t bytes) {
        if (bytes < count * sizeof(X)) fail(BAMG_EINVAL, "export buffer too small (%zu < %zu)", bytes, count * sizeof(X));
        if (count) HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(X), hipMemcpyDeviceToHost, s));
        sync();
    }
    // T array (rows x ldv) -> host doubles (rows x cols)
    void copy_out_T(const T* src, size_t rows, size_t ldv, size_t cols, void* dst, size_t bytes) {
        if (bytes < rows * cols * sizeof(double)) fail(BAMG_EINVAL, "export buffer too small");
        std::vector<T> h(rows * ldv);
        if (!h.empty()) HIPCHK(hipMemcpyAsync(h.data(), src, h.size() * sizeof(T), hipMemcpyDeviceToHost, s));
        sync();
        double* o2 = (double*)dst;
        for (size_t i = 0; i < rows; ++i)
            for (size_t k = 0; k < cols; ++k) o2[i * cols + k] = (double)h[i * ldv + k];
    }

    // Training pairs of every non-coarsest level kept with options.collect
    // (k_pair_* in k_learn.h), in level order; written only when they fit
    // in cap rows.  Returns their count.
    long long collect_pairs(float* F, float* Tg, long long cap, float fcap, float tcap) override {
        const int nl = (int)L.size();
        long long total = 0;
        int* keep = nullptr;
        int* pos = nullptr;
        for (int l = 0; l + 1 < nl; ++l) {
            auto& lv = L[l];
            if (!lv.feat) continue;
            const int rows = lv.cont_rows;
            if (!keep) { keep = A.alloc<int>((size_t)n + 1); pos = A.alloc<int>((size_t)n + 1); }
            const float* w = o.setup_passes == 1 ? lv.slotw0 : lv.slotw;
            LAUNCH(k_pair_flag, nblk(rows), BAMG_BLK, s, rows, (const float*)lv.feat, w, (const float*)lv.slotw0,
                   fcap, tcap, keep);
            scan(rows, keep, pos);
            const long long cnt = get1(pos + rows);
            if (F && Tg && total + cnt <= cap)
                LAUNCH(k_pair_write, nblk(rows), BAMG_BLK, s, rows, (const float*)lv.feat, w, (const float*)lv.slotw0,
                       (const int*)keep, (const int*)pos, total, F, Tg);
            total += cnt;
        }
        sync();
        return total;
    }

    void export_item(int l, int what, void* dst, size_t bytes) override {
        if (nch != 1) fail(BAMG_EINVAL, "export is available for single-chain handles");
        if (l < 0 || l >= (int)L.size()) fail(BAMG_EINVAL, "level %d out of range", l);
        auto& lv = L[l];
        sync();
        const int rows = lv.rows;
        const int nnzb = get1(lv.B.rp + rows);
        const int nnzt = lv.Tm.rp ? get1(lv.Tm.rp + rows) : 0;
        const bool last = l == (int)L.size() - 1;
        const int nL = cdh[0].n;
        switch (what) {
            case BAMG_X_B_ROWPTR: copy_out(lv.B.rp, rows + 1, dst, bytes); break;
            case BAMG_X_B_COL: copy_out(lv.B.ci, nnzb, dst, bytes); break;
            case BAMG_X_B_VAL:
                if (l == 0) copy_out((const double*)b0v, nnzb, dst, bytes);
                else copy_out_T(lv.B.v, nnzb, 1, 1, dst, bytes);
                break;
            case BAMG_X_T_ROWPTR: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out(lv.Tm.rp, rows + 1, dst, bytes); break;
            case BAMG_X_T_COL: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out(lv.Tm.ci, nnzt, dst, bytes); break;
            case BAMG_X_T_VAL: if (!lv.Tm.rp) fail(BAMG_EINVAL, "T_0 = I is not stored"); copy_out_T(lv.Tm.v, nnzt, 1, 1, dst, bytes); break;
            case BAMG_X_P_COL: if (!lv.pc) fail(BAMG_EINVAL, "no P on the coarsest level"); copy_out(lv.pc, (size_t)rows * 4, dst, bytes); break;
            case BAMG_X_P_VAL: if (!lv.pc) fail(BAMG_EINVAL, "no P on the coarsest level"); copy_out_T(lv.pv, (size_t)rows * 4, 1, 1, dst, bytes); break;
            case BAMG_X_U: copy_out_T(lv.U, (size_t)rows * r, 1, 1, dst, bytes); break;
            case BAMG_X_V: copy_out_T(lv.V, rows, VS, nvmax, dst, bytes); break;
            case BAMG_X_LAMBDA: copy_out(lam, 2 * (size_t)nvmax, dst, bytes); break;
            case BAMG_X_VKIND: copy_out(kind, nvmax, dst, bytes); break;
            case BAMG_X_X0: if (l != 0) fail(BAMG_EINVAL, "x0 lives on level 0"); copy_out(x0, rows, dst, bytes); break;
            case BAMG_X_W: if (!last) fail(BAMG_EINVAL, "W lives on the coarsest level"); copy_out(Wp, (size_t)nL * nL, dst, bytes); break;
            case BAMG_X_Y: if (!last) fail(BAMG_EINVAL, "y lives on the coarsest level"); copy_out(ypool, nL, dst, bytes); break;
            case BAMG_X_U0: {
                if (l != 0) fail(BAMG_EINVAL, "U0 lives on level 0");
                long long tot = (long long)n * r;
                LAUNCH(k_tv_init<T>, nblk(tot), BAMG_BLK, s, tot, r, FastDiv((uint32_t)r), (const ChainGeo*)L[0].dgeo,
                       L[0].nch, o.seed, sweep_tmp);
                copy_out_T(sweep_tmp, (size_t)n * r, 1, 1, dst, bytes);
                break;
            }
            case BAMG_X_FEATURES:
                if (!lv.feat) fail(BAMG_EINVAL, "features are kept only with options.collect on non-coarsest levels");
                copy_out(lv.feat, (size_t)rows * 24, dst, bytes);
                break;
            case BAMG_X_SLOTW:
            case BAMG_X_SLOTW0:
                if (!lv.slotw) fail(BAMG_EINVAL, "slot weights are kept only with options.collect on non-coarsest levels");
                // with one setup pass the first-pass weights are the final ones
                copy_out(what == BAMG_X_SLOTW0 || o.setup_passes == 1 ? lv.slotw0 : lv.slotw, (size_t)rows * 4, dst,
                         bytes);
                break;
            case BAMG_X_CMAP:
                if (!lv.cmap) fail(BAMG_EINVAL, "level %d was not coarsened by compatible relaxation", l);
                copy_out(lv.cmap, rows, dst, bytes);
                break;
            case BAMG_X_CR_RHO:
                if (bytes < lv.cr_rho.size() * sizeof(double)) fail(BAMG_EINVAL, "export buffer too small");
                if (!lv.cr_rho.empty()) memcpy(dst, lv.cr_rho.data(), lv.cr_rho.size() * sizeof(double));
                break;
            default: fail(BAMG_EINVAL, "unknown export item %d", what);
        }
    }
};

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

void check_options(const bamg_options& o) {
    if (o.nu_setup < 0 || o.nu_pre < 0 || o.nu_post < 0 || !(o.omega > 0) || o.caliber < 1 || o.n_eig < 1 ||
        o.n_eig > 8 || o.gmres_m < 1 || o.gmres_m > GS_MAXB - 1 || o.arnoldi_m < 1 || o.levels < 0 || o.coarse_max < 1)
        fail(BAMG_EINVAL, "invalid options");
    if (o.cycle_mode < 0 || o.cycle_mode > 2) fail(BAMG_EINVAL, "cycle_mode %d not in {0, 1, 2}", o.cycle_mode);
    if (o.interp != BAMG_INTERP_LS && o.interp != BAMG_INTERP_MLP)
        fail(BAMG_EINVAL, "unknown interpolation mode %d", o.interp);
    if (o.interp == BAMG_INTERP_MLP && !o.mlp_weights && !o.mlp_weights_path)
        fail(BAMG_EINVAL, "learned form needs options.mlp_weights or options.mlp_weights_path");
    if (o.setup_passes < 0 || o.setup_passes > 2) fail(BAMG_EINVAL, "setup_passes must be 1 or 2");
    if (!(o.mlp_judge > 0)) fail(BAMG_EINVAL, "mlp_judge must be positive");
    if (o.precision != BAMG_FP64 && o.precision != BAMG_MIXED) fail(BAMG_EINVAL, "unknown precision %d", o.precision);
    if (o.relax != BAMG_RELAX_JACOBI && o.relax != BAMG_RELAX_MCGS) fail(BAMG_EINVAL, "unknown relaxation %d", o.relax);
    if (!(o.gs_omega > 0 && o.gs_omega < 2)) fail(BAMG_EINVAL, "gs_omega must lie in (0, 2)");
    if (o.mu < 1 || o.mu > 2) fail(BAMG_EINVAL, "mu must be 1 (V-cycle) or 2 (W-cycle)");
}

// The options a chain without a grid needs (compatible relaxation).
void check_options_cr(const bamg_options& o) {
    if (!(o.cr_theta > 0 && o.cr_theta < 1)) fail(BAMG_EINVAL, "cr_theta must lie in (0, 1)");
    if (o.cr_nu < 1 || o.cr_nu > 1000 || o.cr_rounds < 1 || o.cr_rounds > 100000)
        fail(BAMG_EINVAL, "cr_nu and cr_rounds must be positive");
    if (o.nbr_dist != 1) fail(BAMG_EUNSUPPORTED, "candidate sets at graph distance %d are not built (only 1)", o.nbr_dist);
    if (o.caliber > 4) fail(BAMG_EUNSUPPORTED, "caliber above 4 without a grid");
    if (o.relax != BAMG_RELAX_JACOBI) fail(BAMG_EUNSUPPORTED, "multicolour Gauss-Seidel needs a grid");
    if (o.interp != BAMG_INTERP_LS) fail(BAMG_EUNSUPPORTED, "the learned interpolation needs a grid");
}

bamg_ctx* make_ctx(const bamg_options& o) {
    if (o.precision == BAMG_MIXED) return new Engine<float>();
    return new Engine<double>();
}

int setup_common(int32_t nchains, const int64_t* off, const int32_t* row_ptr, const int32_t* col_idx,
                 const double* val, const bamg_grid* grids, int32_t r, const bamg_options* opt, void* stream,
                 bamg_handle* out) {
    bamg_ctx* ctx = nullptr;
    int rc = run_guarded([&] {
        if (!out) fail(BAMG_EINVAL, "out is NULL");
        *out = nullptr;
        if (!row_ptr || !col_idx || !val || !grids || !off) fail(BAMG_EINVAL, "NULL argument");
        if (nchains < 1 || nchains > 4096) fail(BAMG_EINVAL, "nchains = %d out of range", nchains);
        if (r < 1 || r > 32) fail(BAMG_EINVAL, "r = %d out of range [1, 32]", r);
        if (off[0] != 0) fail(BAMG_EINVAL, "chain_row_off[0] must be 0");
        const long long n = off[nchains];
        if (n < 1 || n > (1LL << 30)) fail(BAMG_EINVAL, "n = %lld out of range", n);
        // the relaxation kernels number their (row, test-vector column) pairs
        // in 32 bits: n times the widest test set (r + up to 8 eigenvector
        // columns) must stay below 2^31
        if (n * (long long)(r + 8) >= (1LL << 31))
            fail(BAMG_EUNSUPPORTED, "n * (r + 8) = %lld exceeds the 2^31 (row, column) pairs the sweeps index",
                 n * (long long)(r + 8));
        bamg_options o;
        if (opt) o = *opt; else bamg_options_default(&o);
        check_options(o);
        std::vector<ChainH> ch(nchains);
        for (int c = 0; c < nchains; ++c) {
            const bamg_grid& gr = grids[c];
            const long long nc = off[c + 1] - off[c];
            if (nc < 1) fail(BAMG_EINVAL, "chain %d is empty", c);
            if (gr.nx == 0 && gr.ny == 0) {
                // no grid: compatible relaxation decides every level
                if (nchains != 1) fail(BAMG_EUNSUPPORTED, "chains without a grid are set up one at a time");
                check_options_cr(o);
                ch[c].uidx = c;
                ch[c].uoff = off[c];
                ch[c].n = nc;
                ch[c].grid = GridH{0, 0, 0};
                ch[c].plan = {GridH{(int)nc, 1, 0}};
                continue;
            }
            if (gr.nx < 1 || gr.ny < 1 || (long long)gr.nx * gr.ny != nc)
                fail(BAMG_EINVAL, "grid %dx%d of chain %d does not match its %lld states", gr.nx, gr.ny, c, nc);
            if (gr.periodic && (gr.nx < 3 || gr.ny < 3)) fail(BAMG_EUNSUPPORTED, "periodic sides must be >= 3");
            ch[c].uidx = c;
            ch[c].uoff = off[c];
            ch[c].n = nc;
            ch[c].grid = GridH{gr.nx, gr.ny, gr.periodic ? 1 : 0};
            ch[c].plan = level_plan(ch[c].grid, o.levels, o.coarse_max);
        }
        std::stable_sort(ch.begin(), ch.end(),
                         [](const ChainH& a, const ChainH& b) { return a.plan.size() > b.plan.size(); });
        ctx = make_ctx(o);
        ctx->s = (hipStream_t)stream;
        ctx->o = o;
        ctx->r = r;
        ctx->n = n;
        ctx->nch = nchains;
        ctx->chains = ch;
        ctx->setup(row_ptr, col_idx, val);
        *out = ctx;
    });
    if (rc != BAMG_OK) delete ctx;
    return rc;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
// ------------------------------------------------------------------ scratch
// The allocation-free inference entry point keeps its staging in one
// file-scope device array per GPU: the packed network (MlpPack, padded to 256
// bytes), then the inputs as bfloat16 rows of MLP_INP values for at most
// NOALLOC_MLP_MAXN points (8.02 MiB in all).  Host code never uses the
// array's name as an address: its device address comes from
// hipGetSymbolAddress, once per device with that device current.
constexpr long long NOALLOC_MLP_MAXN = 1LL << 17;
constexpr size_t NOALLOC_PK_BYTES = (sizeof(MlpPack) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_PK_BYTES + (size_t)NOALLOC_MLP_MAXN * MLP_INP * sizeof(unsigned short);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEV] = {};

// Device address of the current device's scratch (looked up on its first use).
unsigned char* noalloc_scratch() {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) fail(BAMG_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) fail(BAMG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    return (unsigned char*)g_scratch_ptr[dev];
}

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
    opt->arnoldi_m = 40;
    opt->gmres_m = 50;
    opt->precision = BAMG_FP64;
    opt->interp = BAMG_INTERP_LS;
    opt->seed = 0;
    opt->setup_passes = 2;
    opt->mlp_judge = 2.0f;
    opt->relax = BAMG_RELAX_JACOBI;
    opt->gs_omega = 1.0;
    opt->mu = 1;
    opt->cr_theta = 0.85;
    opt->cr_nu = 8;
    opt->cr_rounds = 64;
    opt->nbr_dist = 1;
}

const char* bamg_last_error(void) { return g_last_error.c_str(); }

int bamg_setup(int64_t n, const int32_t* row_ptr, const int32_t* col_idx, const double* val, bamg_grid grid,
               int32_t r, const bamg_options* opt, void* stream, bamg_handle* out) {
    int64_t off[2] = {0, n};
    if (n < 1) {
        if (out) *out = nullptr;
        g_last_error = "n < 1";
        return BAMG_EINVAL;
    }
    return setup_common(1, off, row_ptr, col_idx, val, &grid, r, opt, stream, out);
}

int bamg_setup_batched(int32_t nchains, const int64_t* chain_row_off, const int32_t* row_ptr, const int32_t* col_idx,
                       const double* val, const bamg_grid* grids, int32_t r, const bamg_options* opt, void* stream,
                       bamg_handle* out) {
    return setup_common(nchains, chain_row_off, row_ptr, col_idx, val, grids, r, opt, stream, out);
}

int bamg_solve(bamg_handle h, double* x, double tol, int32_t max_cycles, uint32_t flags, bamg_solve_info* info) {
    int code = BAMG_OK;
    int rc = run_guarded([&] {
        if (!h || !x) fail(BAMG_EINVAL, "NULL handle or x");
        if (!(tol > 0) || max_cycles < 0) fail(BAMG_EINVAL, "invalid tol or max_cycles");
        if (flags & ~(BAMG_USE_GUESS | BAMG_PARNOLDI)) fail(BAMG_EINVAL, "unknown solve flags 0x%x", flags);
        code = h->solve(x, tol, max_cycles, flags, nullptr, nullptr, info);
    });
    if (rc != BAMG_OK) return rc;
    if (code == BAMG_ENOCONV) g_last_error = "tolerance not reached within max_cycles";
    return code;
}

int bamg_solve_batched(bamg_handle h, double* x, double tol, int32_t max_cycles, uint32_t flags, int32_t* chain_status,
                       double* chain_residual, bamg_solve_info* info) {
    int code = BAMG_OK;
    int rc = run_guarded([&] {
        if (!h || !x) fail(BAMG_EINVAL, "NULL handle or x");
        if (!(tol > 0) || max_cycles < 0) fail(BAMG_EINVAL, "invalid tol or max_cycles");
        if (flags & ~(BAMG_USE_GUESS | BAMG_PARNOLDI)) fail(BAMG_EINVAL, "unknown solve flags 0x%x", flags);
        code = h->solve(x, tol, max_cycles, flags, chain_status, chain_residual, info);
    });
    if (rc != BAMG_OK) return rc;
    if (code == BAMG_ENOCONV) g_last_error = "tolerance not reached within max_cycles for some chain";
    return code;
}

int bamg_mle_iterate(bamg_handle h, double* x, double tol, int32_t max_cycles, bamg_solve_info* info) {
    int code = BAMG_OK;
    int rc = run_guarded([&] {
        if (!h || !x) fail(BAMG_EINVAL, "NULL handle or x");
        if (!(tol > 0) || max_cycles < 0) fail(BAMG_EINVAL, "invalid tol or max_cycles");
        code = h->mle_iterate(x, tol, max_cycles, info);
    });
    if (rc != BAMG_OK) return rc;
    if (code == BAMG_ENOCONV) g_last_error = "tolerance not reached within max_cycles MLE cycles";
    return code;
}

int bamg_free(bamg_handle h) {
    return run_guarded([&] { delete h; });
}

int bamg_trim(void) {
    return run_guarded([&] { device_cache().trim(-1); });
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

// ---- learned interpolation: network calls ------------------------------
int bamg_mlp_init(uint64_t seed, float* params, void* stream) {
    return run_guarded([&] {
        if (!params) fail(BAMG_EINVAL, "NULL params");
        hipStream_t s = (hipStream_t)stream;
        LAUNCH(k_mlp_init, ceil_div(MLP_NPARAM, BAMG_BLK), BAMG_BLK, s, seed, params);
        HIPCHK(hipStreamSynchronize(s));
    });
}

namespace {
// Device copies the network calls share: inputs as padded bfloat16 rows and
// the packed weights.
struct MlpBatch {
    Arena A;
    unsigned short* xb = nullptr;
    MlpPack* pk = nullptr;
    MlpBatch(hipStream_t s) { A.s = s; }
    ~MlpBatch() { A.release(); }
    unsigned short* prep(const float* feat, long long n) {
        unsigned short* x = A.alloc<unsigned short>((size_t)n * MLP_INP);
        const long long tot = n * MLP_INP;
        LAUNCH(k_mlp_prep, (int)((tot + BAMG_BLK - 1) / BAMG_BLK), BAMG_BLK, A.s, n, feat, x);
        return x;
    }
    void pack(const float* params) {
        if (!pk) pk = A.alloc<MlpPack>(1);
        LAUNCH(k_mlp_pack, 16, BAMG_BLK, A.s, params, pk);
    }
};

// Loss (masked MSE normalised by the chunk's own count) and gradient of the
// points [first, first + bsz) of xb, or of bsz points drawn with `seed` at
// `step`; grad may be null.  Returns {loss, count} on the host when sync.
struct MlpStep {
    Arena& A;
    int cap;                         // largest batch
    float *cpart, *cnt, *wpart, *lpart, *lossd, *gbuf;
    MlpStep(Arena& a, int capacity) : A(a), cap(capacity) {
        const int nb = ceil_div(cap, BAMG_BLK);
        cpart = A.alloc<float>(nb);
        cnt = A.alloc<float>(1);
        wpart = A.alloc<float>((size_t)nb * 4 * MLP_NPARAM);
        lpart = A.alloc<float>((size_t)nb * 4);
        lossd = A.alloc<float>(1);
        gbuf = A.alloc<float>(MLP_NPARAM);
    }
    void run(long long n, int bsz, long long first, uint64_t seed, long long step, const unsigned short* xb,
             const float* tgt, const MlpPack* pk, float* grad) {
        const int nb = ceil_div(bsz, BAMG_BLK);
        LAUNCH(k_mlp_count, nb, BAMG_BLK, A.s, n, bsz, first, seed, step, xb, cpart);
        LAUNCH(k_mlp_sum, 1, BAMG_BLK, A.s, nb, (const float*)cpart, cnt);
        LAUNCH(k_mlp_fwdbwd, nb, BAMG_BLK, A.s, n, bsz, first, seed, step, xb, tgt, pk, (const float*)cnt, wpart,
               lpart);
        LAUNCH(k_mlp_reduce, ceil_div(MLP_NPARAM, BAMG_BLK), BAMG_BLK, A.s, nb * 4, (const float*)wpart,
               grad ? grad : gbuf);
        LAUNCH(k_mlp_sum, 1, BAMG_BLK, A.s, nb * 4, (const float*)lpart, lossd);
    }
    std::pair<double, double> read() {
        float h[2];
        HIPCHK(hipMemcpyAsync(&h[0], lossd, sizeof(float), hipMemcpyDeviceToHost, A.s));
        HIPCHK(hipMemcpyAsync(&h[1], cnt, sizeof(float), hipMemcpyDeviceToHost, A.s));
        HIPCHK(hipStreamSynchronize(A.s));
        return {h[0], h[1]};
    }
};

// Loss over a whole set, in chunks, normalised by the set's total count.
double mlp_set_loss(MlpStep& st, const unsigned short* xb, const float* tgt, long long n, const MlpPack* pk) {
    double num = 0, den = 0;
    for (long long f = 0; f < n; f += st.cap) {
        const int b = (int)std::min<long long>(st.cap, n - f);
        st.run(n, b, f, 0, 0, xb, tgt, pk, nullptr);
        auto lc = st.read();
        num += lc.first * std::max(1.0, lc.second);
        den += lc.second;
    }
    return den > 0 ? num / den : 0.0;
}
}  // namespace

int bamg_mlp_forward(const float* feat, int64_t n, const float* params, float* out, void* stream) {
    return run_guarded([&] {
        if (!feat || !params || !out) fail(BAMG_EINVAL, "NULL argument");
        if (n < 0 || n > (1LL << 30)) fail(BAMG_EINVAL, "n out of range");
        if (n == 0) return;
        hipStream_t s = (hipStream_t)stream;
        MlpBatch mb(s);
        unsigned short* xb = mb.prep(feat, n);
        mb.pack(params);
        const int grid = (int)std::min<long long>(1024, (n + 255) / 256);
        LAUNCH(k_mlp_infer, grid, BAMG_BLK, s, (long long)n, (const unsigned short*)xb, (const MlpPack*)mb.pk, out);
        HIPCHK(hipStreamSynchronize(s));
    });
}

int bamg_mlp_forward_noalloc(const float* feat, int64_t n, const float* params, float* out, void* stream) {
    return run_guarded([&] {
        if (!feat || !params || !out) fail(BAMG_EINVAL, "NULL argument");
        if (n < 0 || n > NOALLOC_MLP_MAXN)
            fail(BAMG_EINVAL, "n = %lld outside [0, %lld] (the points the static scratch holds)", (long long)n,
                 NOALLOC_MLP_MAXN);
        if (n == 0) return;
        hipStream_t s = (hipStream_t)stream;
        unsigned char* base = noalloc_scratch();
        MlpPack* pk = (MlpPack*)base;
        unsigned short* xb = (unsigned short*)(base + NOALLOC_PK_BYTES);
        // the same launches as bamg_mlp_forward; every byte they read from
        // the scratch is written first by this call
        LAUNCH(k_mlp_pack, 16, BAMG_BLK, s, params, pk);
        const long long tot = (long long)n * MLP_INP;
        LAUNCH(k_mlp_prep, (int)((tot + BAMG_BLK - 1) / BAMG_BLK), BAMG_BLK, s, (long long)n, feat, xb);
        const int grid = (int)std::min<long long>(1024, (n + 255) / 256);
        LAUNCH(k_mlp_infer, grid, BAMG_BLK, s, (long long)n, (const unsigned short*)xb, (const MlpPack*)pk, out);
        HIPCHK(hipStreamSynchronize(s));
    });
}
int bamg_mlp_loss_grad(const float* feat, const float* tgt, int64_t n, const float* params, float* grad,
                       double* loss, void* stream) {
    return run_guarded([&] {
        if (!feat || !tgt || !params || !grad) fail(BAMG_EINVAL, "NULL argument");
        if (n < 1 || n > (1 << 24)) fail(BAMG_EINVAL, "n out of range [1, 2^24]");
        hipStream_t s = (hipStream_t)stream;
        MlpBatch mb(s);
        unsigned short* xb = mb.prep(feat, n);
        mb.pack(params);
        MlpStep st(mb.A, (int)n);
        st.run(n, (int)n, 0, 0, 0, xb, tgt, mb.pk, grad);
        auto lc = st.read();
        if (loss) *loss = lc.first;
    });
}

int bamg_mlp_train(const float* feat, const float* tgt, int64_t n, const float* vfeat, const float* vtgt, int64_t nv,
                   float* params, const bamg_mlp_train_opts* opt, bamg_mlp_train_info* info, void* stream) {
    return run_guarded([&] {
        auto t0 = std::chrono::steady_clock::now();
        if (!feat || !tgt || !params) fail(BAMG_EINVAL, "NULL argument");
        if (n < 1 || n > (1LL << 30) || nv < 0 || (nv > 0 && (!vfeat || !vtgt))) fail(BAMG_EINVAL, "bad sizes");
        bamg_mlp_train_opts o{8, 4096, 1e-3f, 0.9f, 0.999f, 1e-8f, 6};
        if (opt) o = *opt;
        if (o.epochs < 0 || o.batch < 256 || o.batch % 256 || o.batch > (1 << 20) || !(o.lr > 0))
            fail(BAMG_EINVAL, "bad training options");
        hipStream_t s = (hipStream_t)stream;
        MlpBatch mb(s);
        unsigned short* xb = mb.prep(feat, n);
        unsigned short* vxb = nv > 0 ? mb.prep(vfeat, nv) : nullptr;
        float* m = mb.A.alloc<float>(MLP_NPARAM);
        float* v = mb.A.alloc<float>(MLP_NPARAM);
        HIPCHK(hipMemsetAsync(m, 0, MLP_NPARAM * sizeof(float), s));
        HIPCHK(hipMemsetAsync(v, 0, MLP_NPARAM * sizeof(float), s));
        MlpStep st(mb.A, std::max(o.batch, 65536));
        bamg_mlp_train_info inf{};
        mb.pack(params);
        if (nv > 0) inf.val_loss_first = mlp_set_loss(st, vxb, vtgt, nv, mb.pk);
        const long long spe = (n + o.batch - 1) / o.batch;
        long long step = 0;
        for (int ep = 0; ep < o.epochs; ++ep) {
            for (long long k = 0; k < spe; ++k, ++step) {
                const long long first = o.seed ? 0 : k * o.batch;
                const int bsz = o.seed ? (int)std::min<long long>(o.batch, n)
                                       : (int)std::min<long long>(o.batch, n - first);
                mb.pack(params);
                st.run(n, bsz, first, o.seed, step, xb, tgt, mb.pk, st.gbuf);
                const double t = (double)(step + 1);
                const float c1 = (float)(1.0 / (1.0 - std::pow((double)o.beta1, t)));
                const float c2 = (float)(1.0 / (1.0 - std::pow((double)o.beta2, t)));
                LAUNCH(k_mlp_adam, ceil_div(MLP_NPARAM, BAMG_BLK), BAMG_BLK, s, params, m, v, (const float*)st.gbuf,
                       o.lr, o.beta1, o.beta2, o.eps, c1, c2);
                if (step == 0) inf.train_loss_first = st.read().first;
            }
            if (spe > 0) inf.train_loss_last = st.read().first;
            if (nv > 0 && inf.val_len < 64) {
                mb.pack(params);
                inf.val_history[inf.val_len++] = mlp_set_loss(st, vxb, vtgt, nv, mb.pk);
            }
        }
        inf.steps = (int)step;
        if (nv > 0) {
            mb.pack(params);
            inf.val_loss_last = mlp_set_loss(st, vxb, vtgt, nv, mb.pk);
        }
        HIPCHK(hipStreamSynchronize(s));
        inf.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
    });
}

int bamg_mlp_collect(bamg_handle h, float* feat, float* tgt, int64_t cap, int64_t* count) {
    return run_guarded([&] {
        if (!h || !count) fail(BAMG_EINVAL, "NULL argument");
        if (cap < 0) fail(BAMG_EINVAL, "cap < 0");
        if (!h->o.collect) fail(BAMG_EINVAL, "training pairs are kept only with options.collect");
        const long long c = h->collect_pairs(feat, tgt, cap, MLP_FEATURE_CAP, MLP_TARGET_CAP);
        *count = c;
        if (feat && tgt && c > cap)
            fail(BAMG_EINVAL, "%lld training pairs do not fit in cap = %lld rows", c, (long long)cap);
    });
}

void bamg_train_spec_default(bamg_train_spec* sp) {
    if (!sp) return;
    std::memset(sp, 0, sizeof(*sp));
    sp->n_chains = 32;
    sp->n_val = 4;
    sp->side_min = 256;
    sp->side_max = 1024;
    sp->jitter = 0.2;
    sp->seed = 0;
    sp->r = 12;
    sp->levels = 6;
    sp->init_seed = 5;
    sp->train = bamg_mlp_train_opts{8, 4096, 1e-3f, 0.9f, 0.999f, 1e-8f, 6};
}

namespace {
// The tandem queue of Section 5 (Table 2) as CSR of A (row = destination
// state, entries in ascending source state): states (a, b), 0 <= a, b <= N,
// s = a (N + 1) + b; arrival (a, b) -> (a + 1, b), service (a, b) ->
// (a - 1, b + 1) and departure (a, b) -> (a, b - 1) with the uniformised
// rates 11/31, 10/31, 10/31, each times 1 + jitter (2u - 1) with u from the
// counter generator (seed, stream 3, 3 chain + k) when jitter != 0; a
// blocked move stays as a self-loop, so every column sums to one.  N >= 2.
void tandem_csr(int N, double jitter, uint64_t seed, int chain, std::vector<int>& rp, std::vector<int>& ci,
                std::vector<double>& v) {
    double rate[3] = {11.0 / 31, 10.0 / 31, 10.0 / 31};
    if (jitter != 0.0)
        for (int k = 0; k < 3; ++k)
            rate[k] = rate[k] * (1.0 + jitter * (2.0 * splitmix_u01(seed, 3, 3ull * chain + k) - 1.0));
    const double tot = rate[0] + rate[1] + rate[2];
    const double pa = rate[0] / tot, ps = rate[1] / tot, pd = rate[2] / tot;
    const int side = N + 1;
    const long long n = (long long)side * side;
    rp.assign(n + 1, 0);
    ci.clear();
    v.clear();
    ci.reserve(4 * n);
    v.reserve(4 * n);
    for (int a = 0; a <= N; ++a)
        for (int b = 0; b <= N; ++b) {
            const int st = a * side + b;
            if (a >= 1) { ci.push_back(st - side); v.push_back(pa); }              // arrival from (a-1, b)
            const double blocked = pa * (a >= N ? 1.0 : 0.0) + ps * ((a == 0 || b >= N) ? 1.0 : 0.0) +
                                   pd * (b == 0 ? 1.0 : 0.0);
            if (blocked > 0) { ci.push_back(st); v.push_back(blocked); }           // self-loop
            if (b <= N - 1) { ci.push_back(st + 1); v.push_back(pd); }             // departure from (a, b+1)
            if (a <= N - 1 && b >= 1) { ci.push_back(st + side - 1); v.push_back(ps); }   // service from (a+1, b-1)
            rp[st + 1] = (int)ci.size();
        }
}
}  // namespace

int bamg_mlp_train_spec(const bamg_train_spec* spec, const char* out_path, float* params,
                        bamg_mlp_train_info* info, void* stream) {
    return run_guarded([&] {
        if (!spec) fail(BAMG_EINVAL, "NULL spec");
        const bamg_train_spec& sp = *spec;
        if (sp.n_chains < 1 || sp.n_chains > 4096 || sp.n_val < 0 || sp.n_val >= sp.n_chains)
            fail(BAMG_EINVAL, "n_chains = %d, n_val = %d out of range", sp.n_chains, sp.n_val);
        if (sp.side_min < 3 || sp.side_max < sp.side_min || sp.side_max > 4096)
            fail(BAMG_EINVAL, "sides [%d, %d] out of range [3, 4096]", sp.side_min, sp.side_max);
        if (sp.r < 1 || sp.r > 32 || sp.levels < 2) fail(BAMG_EINVAL, "r = %d, levels = %d out of range", sp.r,
                                                         sp.levels);
        hipStream_t s = (hipStream_t)stream;
        Arena A;
        A.s = s;
        struct Part { float* f; float* t; long long n; };
        std::vector<Part> parts;
        bamg_options o;
        bamg_options_default(&o);
        o.levels = sp.levels;
        o.collect = 1;
        for (int c = 0; c < sp.n_chains; ++c) {
            // chain c: side drawn from (seed, stream 8, c), rates jittered
            const double u = splitmix_u01(sp.seed, 8, (uint64_t)c);
            const int N = (sp.side_min - 1) + (int)(u * (double)(sp.side_max - sp.side_min + 1));
            std::vector<int> rp, ci;
            std::vector<double> v;
            tandem_csr(N, sp.jitter, sp.seed, 1000 + c, rp, ci, v);
            const long long n = (long long)rp.size() - 1;
            int* drp = A.upload(rp);
            int* dci = A.upload(ci);
            double* dv = A.upload(v);
            bamg_handle h = nullptr;
            const bamg_grid g{N + 1, N + 1, 0};
            int rc = bamg_setup(n, drp, dci, dv, g, sp.r, &o, stream, &h);
            if (rc != BAMG_OK) fail(rc, "training chain %d: %s", c, bamg_last_error());
            std::unique_ptr<bamg_ctx, int (*)(bamg_handle)> guard(h, bamg_free);
            int64_t cnt = 0;
            rc = bamg_mlp_collect(h, nullptr, nullptr, 0, &cnt);
            if (rc != BAMG_OK) fail(rc, "training chain %d: %s", c, bamg_last_error());
            Part pt{A.alloc<float>((size_t)cnt * 24), A.alloc<float>((size_t)cnt * 4), cnt};
            rc = bamg_mlp_collect(h, pt.f, pt.t, cnt, &cnt);
            if (rc != BAMG_OK) fail(rc, "training chain %d: %s", c, bamg_last_error());
            parts.push_back(pt);
        }
        // the first n_chains - n_val chains train, the others validate
        auto concat = [&](int c0, int c1, float*& f, float*& t) {
            long long tot = 0;
            for (int c = c0; c < c1; ++c) tot += parts[c].n;
            f = A.alloc<float>((size_t)std::max(tot, 1LL) * 24);
            t = A.alloc<float>((size_t)std::max(tot, 1LL) * 4);
            long long at = 0;
            for (int c = c0; c < c1; ++c) {
                HIPCHK(hipMemcpyAsync(f + at * 24, parts[c].f, sizeof(float) * 24 * parts[c].n, hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(t + at * 4, parts[c].t, sizeof(float) * 4 * parts[c].n, hipMemcpyDeviceToDevice, s));
                at += parts[c].n;
            }
            return tot;
        };
        float *ftr, *ttr, *fva = nullptr, *tva = nullptr;
        const long long ntr = concat(0, sp.n_chains - sp.n_val, ftr, ttr);
        const long long nva = sp.n_val ? concat(sp.n_chains - sp.n_val, sp.n_chains, fva, tva) : 0;
        if (ntr < 1) fail(BAMG_EINVAL, "the training chains gave no training pairs");
        float* th = params ? params : A.alloc<float>(MLP_NPARAM);
        LAUNCH(k_mlp_init, ceil_div(MLP_NPARAM, BAMG_BLK), BAMG_BLK, s, sp.init_seed, th);
        const int rc = bamg_mlp_train(ftr, ttr, ntr, fva, tva, nva, th, &sp.train, info, stream);
        if (rc != BAMG_OK) fail(rc, "%s", bamg_last_error());
        if (out_path) {
            std::vector<float> hp(MLP_NPARAM);
            HIPCHK(hipMemcpyAsync(hp.data(), th, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            write_mlp_file(out_path, hp);
        }
        A.release();
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
            ~Rel() { A.release(); }
        } rel{A};
        int hr[2];
        HIPCHK(hipMemcpyAsync(&hr[0], row_ptr, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&hr[1], row_ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hr[0] != 0 || hr[1] < 0) fail(BAMG_EINVAL, "row_ptr[0] must be 0");
        const int N = (int)n;
        // relaxation needs no grid: one chain on an N x 1 grid, box test ignored
        std::vector<ChainGeo> gv(1);
        gv[0].off = 0; gv[0].n = N; gv[0].nx = N; gv[0].ny = 1; gv[0].periodic = 0; gv[0].dy = FastDiv(1u);
        ChainGeo* dg = A.upload(gv);
        double* colsum = A.alloc<double>(N);
        int* cnt = A.alloc<int>(N);
        int* brp = A.alloc<int>(N + 1);
        int* err = A.alloc<int>(4);
        int* bsum = A.alloc<int>(nblk(N) + 1);
        int* total = A.alloc<int>(2);
        HIPCHK(hipMemsetAsync(colsum, 0, sizeof(double) * N, s));
        HIPCHK(hipMemsetAsync(err, 0, sizeof(int) * 4, s));
        LAUNCH(k_check_a, nblk(N), BAMG_BLK, s, N, row_ptr, col_idx, val, (const ChainGeo*)dg, 1, hr[1], colsum, cnt,
               err);
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
               (double*)nullptr, omega, dinv, (double*)nullptr, (int*)nullptr, (double*)nullptr, (double*)nullptr,
               err);
        HIPCHK(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (e & ERR_ZERODIAG) fail(BAMG_EZERODIAG, "b_ii <= 0");
        double* tmp = A.alloc<double>((size_t)N * R);
        double* a = X;
        double* b = tmp;
        FastDiv dR((uint32_t)R);
        for (int k = 0; k < nu; ++k) {
            LAUNCH((k_sweep<double, double>), nblk((long long)N * R), BAMG_BLK, s, N, R, dR, (const int*)brp,
                   (const int*)bci, (const double*)bv, (const double*)dinv, (const double*)a, F, b,
                   RowMask{(const ChainGeo*)dg, 1, nullptr});
            std::swap(a, b);
        }
        if (a != X) HIPCHK(hipMemcpyAsync(X, a, sizeof(double) * N * R, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    });
}

}  // extern "C"
