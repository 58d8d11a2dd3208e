// Plan runtime and C ABI of the DM stray-field library (host side).
//
// A plan fixes one grid (n, d) and precision.  Creating it computes the
// demagnetization-tensor spectrum once (the paper's "setup" column: the
// auxiliary constants depend only on geometry and discretization, Sec. 4) and
// allocates the two spectrum scratch buffers; each field evaluation then
// enqueues five pass kernels and, for the energy, one reduction.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <mutex>
#include <type_traits>
#include <vector>

#include "../../include/demag.h"
#include "fft_reg.hpp"
#include "internal.hpp"

using namespace demag;

// ---------------------------------------------------------------------------
// profiler ranges: every API call that enqueues work, and each pass of a field
// evaluation, is a named host-side range (rocprofv3 --marker-trace); a range
// covers the enqueue on the host, the kernels run later on the stream
namespace {
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

// ---------------------------------------------------------------------------
// device allocation with a test hook: while DEMAG_FAIL_ALLOC_AT=k is set, the
// k-th allocation counted since the variable last changed fails as out of
// memory (to exercise every failure path of plan creation and set-up)
namespace {
template <typename T>
hipError_t dev_malloc(T** ptr, size_t bytes) {
    static std::mutex mu;
    static std::string seen;
    static long count = 0;
    if (const char* e = std::getenv("DEMAG_FAIL_ALLOC_AT")) {
        std::lock_guard<std::mutex> lock(mu);
        if (seen != e) {
            seen = e;
            count = 0;
        }
        if (++count == std::atol(e)) {
            *ptr = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc((void**)ptr, bytes);
}
}  // namespace

// ---------------------------------------------------------------------------
// errors
namespace {
thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) {  // an allocation, e.g. set-up scratch: not a device fault
        (void)hipGetLastError();
        return fail(DEMAG_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    }
    return fail(DEMAG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #call);   \
    } while (0)

constexpr int kPassMarks = 7;  // before X, Y, Z, Y^-1, X^-1, energy; end
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846264338327950288;
constexpr int kMaxLen = 4096;
constexpr size_t kMaxLdsBytes = 65536;  // dynamic LDS per workgroup, generic kernels
size_t g_p2_lds = 65536;                 // power-of-two kernels: the device's per-workgroup LDS (set per plan)

// ---------------------------------------------------------------------------
// lengths, radices, twiddles
bool is_smooth(long v) {
    for (int p : {2, 3, 5})
        while (v % p == 0) v /= p;
    return v == 1;
}

int smooth_at_least(int n) {
    long v = n;
    while (!is_smooth(v)) ++v;
    return (int)v;
}

FftPlanDev make_fft_plan(int P) {
    FftPlanDev pl{};
    pl.P = P;
    int v = P, ns = 0;
    while (v % 8 == 0) { pl.radix[ns++] = 8; v /= 8; }
    while (v % 4 == 0) { pl.radix[ns++] = 4; v /= 4; }
    while (v % 2 == 0) { pl.radix[ns++] = 2; v /= 2; }
    while (v % 5 == 0) { pl.radix[ns++] = 5; v /= 5; }
    while (v % 3 == 0) { pl.radix[ns++] = 3; v /= 3; }
    pl.nstages = ns;
    return pl;
}

// tw[t] = exp(-2 pi i t / P), evaluated in long double and rounded once.
template <typename T>
std::vector<cx<T>> twiddles(int P) {
    std::vector<cx<T>> tw(P);
    const long double twopi = 6.283185307179586476925286766559005768L;
    for (int t = 0; t < P; ++t) {
        long double a = twopi * (long double)t / (long double)P;
        tw[t].re = (T)cosl(a);
        tw[t].im = (T)(-sinl(a));
    }
    return tw;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_q, long double).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
    x.resize(q);
    w.resize(q);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < q; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (q + 0.5L)), dp = 1;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= q; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        long double p0 = 1, p1 = z;
        for (int k = 2; k <= q; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = q * (z * p1 - p0) / (z * z - 1);
        x[i] = (double)z;
        w[i] = (double)(2 / ((1 - z * z) * dp * dp));
    }
}

int pick_E(long elems, int threads) {
    for (int E : {4, 8, 16, 32})
        if ((long)threads * E >= elems) return E;
    return -1;
}

}  // namespace

// ---------------------------------------------------------------------------
struct PassCfgs {
    LaunchCfg xf, yf, zc, yi, xi;
};

// Tensor-grid (TG) state of a plan (after demag_tg_prepare): Sinc nodes,
// Gaussian matrices, stacked mode-3 factors, GEMM scratch and the device
// pointer arrays of the mode-2 batch.
struct TGState {
    void* handle = nullptr;  // rocblas_handle
    int R = 0;
    double step = 0;
    double* tau = nullptr;
    double* c = nullptr;
    void *D1E = nullptr, *D1O = nullptr, *D2E = nullptr, *D2O = nullptr, *B3E = nullptr, *B3O = nullptr;
    void *Y1 = nullptr, *Y2 = nullptr;
    void **Y1k = nullptr, **Y2k = nullptr, **D2kE = nullptr, **D2kO = nullptr;
    size_t bytes = 0;
    int sol1 = 0, sol2 = 0, sol3 = 0;  // rocBLAS solutions of the mode-product GEMMs (0: the default)
    // FP32 with the fused mode-1/2 kernel: D1E..D2O hold the tiled matrices, Y1 and
    // the pointer arrays are not used; band: lo/hi of D1E, D1O, D2E, D2O in that order
    bool fused = false;
    int* band = nullptr;
    double flops_issued = 0;  // mode-product flops per evaluation after the skipped zero blocks
};

// Low-rank tensor-grid state (after demag_tg_lowrank_prepare): nodes,
// weights, stacked Gaussian matrices per axis, energy partials, expansion
// scratch (grown on demand).
struct LRState {
    void* handle = nullptr;  // rocblas_handle
    int R = 0;
    double* tau = nullptr;
    double* c = nullptr;
    void* DE[3] = {nullptr, nullptr, nullptr};
    void* DO[3] = {nullptr, nullptr, nullptr};
    double* partials = nullptr;
    double* gram = nullptr;  // 27 R r^2 Gram values (grown on demand)
    size_t gram_bytes = 0;
    void* W = nullptr;
    size_t w_bytes = 0;
    size_t bytes = 0;
};

struct demag_plan_s {
    int n[3];
    double d[3];
    demag_dtype dtype;
    int L[3], P[3], Kx;
    FftPlanDev fp[3];
    void* tw[3] = {nullptr, nullptr, nullptr};
    void* twt[3][3] = {};  // thread-major twiddles of register-kernel axes, per radix schedule
    void* nhat = nullptr;
    void* shat = nullptr;  // scalar-potential kernel spectrum (after demag_sp_prepare)
    TGState* tg = nullptr; // tensor-grid state (after demag_tg_prepare)
    LRState* lr = nullptr; // low-rank tensor-grid state (after demag_tg_lowrank_prepare)
    size_t lr_cap = (size_t)256 << 20;  // byte cap of the low-rank expansion scratch
    int tg_mode12 = 1;                   // 1: fused FP32 mode-1/2 kernel where it fits, 0: library GEMMs
    void* als_handle = nullptr;          // rocblas_handle of the ALS compression (created on first use)
    LaunchCfg zs;          // launch shape of the scalar-potential Z pass
    void* B1 = nullptr;
    void* B2 = nullptr;
    double* partials = nullptr;
    double* e_dev = nullptr;
    int npartials = 0;
    size_t scratch_bytes = 0, tensor_bytes = 0;
    TensorBands bands;
    PassCfgs cfg;
    double setup_us = 0;
    int device = 0;
    hipEvent_t done = nullptr;
    hipEvent_t busy = nullptr;  // marks the plan's last enqueued work: `done`, or its batch's event
    hipStream_t last_stream = nullptr;
    bool used = false;
    // optional pass timing: kPassMarks events per evaluation in a ring of tcap slots
    std::vector<hipEvent_t> tev;
    int tcap = 0;
    long tcount = 0;
};

// A batch groups its plans by geometry (grid, cell, precision): the members of
// a group share the tensor spectrum of the first ("lead") plan and run every
// pass as one launch over the group, driven by per-member pointer lists.
struct BatchGroup {
    demag_plan_s* lead = nullptr;
    int count = 0;
    void** lists = nullptr;  // device: m[count], H[count], B1[count], B2[count]
    PassCfgs cfg;            // launch shapes of the group's passes (the lead's until tuned)
    double cost = 0;         // relative run time: modelled (count x padded cells), measured once tuned
};

struct demag_batch_s {
    std::vector<demag_plan_t> plans;
    std::vector<BatchGroup> groups;
    void* dev_lists = nullptr;
    hipEvent_t done = nullptr;  // recorded after every replay; the members' busy marker
    double Ms = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int lanes = 0;  // capture streams the groups are spread over (0: one per hardware queue)
    int used_lanes = 0;  // streams of the recorded graph
};

namespace {

size_t csize(demag_dtype t) { return t == DEMAG_F32 ? sizeof(cx<float>) : sizeof(cx<double>); }

// Default launch shapes: about `target` complex elements per workgroup, tiles
// rounded to what the pass needs, E the smallest instance that covers them.
LaunchCfg cfg_rows(int P, int rows, size_t cbytes) {
    LaunchCfg c;
    long target = (long)(32768 / cbytes);  // 32 KB of LDS
    int pencils = (int)std::max<long>(1, target / P);
    int Ty = std::min(2 * pencils, rows + (rows & 1));
    Ty = std::max(2, Ty & ~1);
    c.t0 = Ty;
    c.E = pick_E((long)(Ty / 2) * P, c.threads);
    return c;
}

LaunchCfg cfg_pencils(int P, int Kx, int nzr, size_t cbytes) {
    LaunchCfg c;
    long target = (long)(32768 / cbytes);
    int B = (int)std::max<long>(1, target / P);
    int Tz = std::min(B, nzr);
    int Tx = std::max(1, std::min(B / Tz, Kx));
    c.t0 = Tx;
    c.t1 = Tz;
    c.E = pick_E((long)Tx * Tz * P, c.threads);
    return c;
}

LaunchCfg cfg_zconv(int P, int Kx, size_t cbytes) {
    LaunchCfg c;
    long target = (long)(32768 / cbytes);
    int Tx = (int)std::max<long>(1, target / (6L * P));
    Tx = std::min(Tx, Kx);
    c.t0 = Tx;
    c.E = pick_E(6L * Tx * P, c.threads);
    return c;
}

int ilog2i(long v) {
    int l = 0;
    while ((1L << (l + 1)) <= v) ++l;
    return l;
}
int pow2_ceil_log(long v) {
    int l = 0;
    while ((1L << l) < v) ++l;
    return l;
}

// p2 tiles: about `target` threads per workgroup, bounded by the extent the
// tile covers and by LDS: the X and Y tiles keep two workgroups per CU (one
// workgroup's barriers then overlap the other's memory traffic).
LaunchCfg p2_rows(int P, int rows, size_t cbytes, int target = 1024) {
    LaunchCfg c;
    c.p2 = 1;
    target = std::min(target, p2_max_threads(P));
    const int TP = p2_threads_per_pencil(P);
    int lgB = ilog2i(std::max(1, target / TP));
    lgB = std::min(lgB, std::max(0, pow2_ceil_log(rows) - 1));
    while (lgB > 0 && ((size_t)p2_slab_elems(P) << lgB) * cbytes + p2_twiddle_lds_bytes(P, cbytes) > g_p2_lds / 2)
        --lgB;
    c.t0 = lgB + 1;  // Ty = 2 * pencils
    c.threads = TP << lgB;
    return c;
}

LaunchCfg p2_pencils(int P, int Kx, int nz, size_t cbytes, int target = 1024) {
    LaunchCfg c;
    c.p2 = 1;
    target = std::min(target, p2_max_threads(P));
    const int TP = p2_threads_per_pencil(P);
    int lgB = ilog2i(std::max(1, target / TP));
    while (lgB > 0 && ((size_t)p2_slab_elems(P) << lgB) * cbytes + p2_twiddle_lds_bytes(P, cbytes) > g_p2_lds / 2)
        --lgB;
    int lgTz = std::min(lgB, pow2_ceil_log(nz));
    int lgTx = std::min(lgB - lgTz, pow2_ceil_log(Kx));
    c.t0 = lgTx;
    c.t1 = lgTz;
    c.threads = TP << (lgTx + lgTz);
    return c;
}

LaunchCfg p2_zconv(int P, int Py, size_t cbytes, int target = 64) {
    LaunchCfg c;
    c.p2 = 1;
    const int TP = p2_threads_per_pencil(P);
    // t1 = ky rows per workgroup: a row and its mirror (2) unless that pair
    // of pencils would exceed the workgroup, then one row (1)
    const int rows = 2 * TP <= kP2MaxThreadsZ ? 2 : 1;
    int lgTx = std::max(0, ilog2i(std::max(1, target / (rows * TP))));
    lgTx = std::min(lgTx, pow2_ceil_log(Py / 2 + 1));
    while (lgTx > 0 && p2_z_lds_bytes(P, rows, lgTx, cbytes) > g_p2_lds - 256) --lgTx;
    while (lgTx > 0 && (rows * TP << lgTx) > kP2MaxThreadsZ) --lgTx;
    c.t0 = lgTx;
    c.t1 = rows;
    c.threads = rows * TP << lgTx;
    return c;
}

bool p2_cfg_ok(const LaunchCfg& c, int P, size_t cbytes, int kind /*0 rows, 1 pencils, 2 z*/) {
    if (!p2_supported(P) || c.t0 < 0 || c.t1 < 0 || c.t0 > 12 || c.t1 > 12) return false;
    if (c.sched < 0 || c.sched >= p2_num_schedules(P)) return false;
    const long TP = p2_threads_per_pencil(P);
    long pencils = kind == 0 ? (1L << (c.t0 - 1)) : kind == 1 ? (1L << (c.t0 + c.t1)) : ((long)c.t1 << c.t0);
    if (kind == 0 && c.t0 < 1) return false;
    if (kind == 2 && c.t1 != (2 * TP <= kP2MaxThreadsZ ? 2 : 1)) return false;
    long threads = pencils * TP;
    long maxthr = kind == 2 ? kP2MaxThreadsZ : p2_max_threads(P);
    if (kind == 2 && !p2_z_supported(P, cbytes)) return false;
    const size_t lds = kind == 2 ? p2_z_lds_bytes(P, c.t1, c.t0, cbytes)
                                 : (size_t)pencils * p2_slab_elems(P) * cbytes + p2_twiddle_lds_bytes(P, cbytes);
    return threads == c.threads && threads <= maxthr && lds <= g_p2_lds - 256;  // + static reduction scratch
}

// byte spans the power-of-two Z pass addresses with 32-bit buffer offsets
bool p2_z_ranges_ok(const demag_plan_s* p) {
    const size_t cb = csize(p->dtype), rb = cb / 2;
    const size_t b2 = (size_t)p->P[1] * p->Kx * p->n[2] * cb;
    const size_t oct = (size_t)(p->P[1] / 2 + 1) * 6 * p->Kx * (p->P[2] / 2 + 1) * rb;
    return b2 < kP2BufLimit && oct < kP2BufLimit;
}

bool cfg_ok(const LaunchCfg& c, long pencils, int P, size_t cbytes) {
    return c.E > 0 && c.threads > 0 && c.threads <= kMaxThreads && c.threads % 64 == 0 &&
           (long)c.threads * c.E >= pencils * P && (size_t)pencils * P * cbytes <= kMaxLdsBytes;
}

bool one_cfg_ok(const LaunchCfg& c, int P, size_t cb, int kind) {
    if (c.p2) return p2_cfg_ok(c, P, cb, kind);
    if (kind == 0) return cfg_ok(c, (c.t0 + 1) / 2, P, cb) && c.t0 % 2 == 0;
    if (kind == 1) return cfg_ok(c, (long)c.t0 * c.t1, P, cb);
    // the generic fused Z pass may use the whole LDS of a workgroup (its
    // launcher raises the per-kernel limit): six pencils of the tile
    const long pencils = 6L * c.t0;
    return c.E > 0 && c.threads > 0 && c.threads <= kMaxThreads && c.threads % 64 == 0 &&
           (long)c.threads * c.E >= pencils * P && (size_t)pencils * P * cb <= g_p2_lds;
}

bool plan_cfgs_ok(const demag_plan_s* p, const PassCfgs& c) {
    size_t cb = csize(p->dtype);
    return one_cfg_ok(c.xf, p->P[0], cb, 0) && one_cfg_ok(c.xi, p->P[0], cb, 0) &&
           one_cfg_ok(c.yf, p->P[1], cb, 1) && one_cfg_ok(c.yi, p->P[1], cb, 1) && one_cfg_ok(c.zc, p->P[2], cb, 2) &&
           (!c.zc.p2 || p2_z_ranges_ok(p));
}

// Generic kernels (any 2^a 3^b 5^c length) unless the padded length is 2^a or
// 3 * 2^a, where the compile-time register kernels are used.
PassCfgs default_cfgs(const demag_plan_s* p) {
    size_t cb = csize(p->dtype);
    PassCfgs c;
    c.xf = p2_supported(p->P[0]) ? p2_rows(p->P[0], p->n[1], cb) : cfg_rows(p->P[0], p->n[1], cb);
    c.xi = c.xf;
    c.yf = p2_supported(p->P[1]) ? p2_pencils(p->P[1], p->Kx, p->n[2], cb) : cfg_pencils(p->P[1], p->Kx, p->n[2], cb);
    c.yi = c.yf;
    c.zc = p2_z_supported(p->P[2], cb) && p2_z_ranges_ok(p) ? p2_zconv(p->P[2], p->P[1], cb)
                                                             : cfg_zconv(p->P[2], p->Kx, cb);
    return c;
}

PassCfgs generic_cfgs(const demag_plan_s* p) {
    size_t cb = csize(p->dtype);
    PassCfgs c;
    c.xf = cfg_rows(p->P[0], p->n[1], cb);
    c.xi = c.xf;
    c.yf = cfg_pencils(p->P[1], p->Kx, p->n[2], cb);
    c.yi = c.yf;
    c.zc = cfg_zconv(p->P[2], p->Kx, cb);
    return c;
}

template <typename T>
int upload(void** dst, const std::vector<T>& v) {
    HIP_TRY(dev_malloc(dst, v.size() * sizeof(T)));
    HIP_TRY(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return DEMAG_OK;
}

// ---------------------------------------------------------------------------
// tensor setup (FP64 throughout, cast at the end)
struct SetupBufs {
    double* Noct = nullptr;
    double* A = nullptr;
    cx<double>* B1 = nullptr;
    cx<double>* B2 = nullptr;
    void* tw[3] = {nullptr, nullptr, nullptr};
    double* glx = nullptr;
    double* glw = nullptr;
    ~SetupBufs() {
        (void)hipFree(Noct);
        (void)hipFree(A);
        (void)hipFree(B1);
        (void)hipFree(B2);
        for (auto t : tw) (void)hipFree(t);
        (void)hipFree(glx);
        (void)hipFree(glw);
    }
};

void reduced_cell(const double d[3], double dt[3]) {
    double h = std::max(d[0], std::max(d[1], d[2]));
    for (int k = 0; k < 3; ++k) dt[k] = d[k] / h;
}

int compute_octant(demag_plan_s* p, hipStream_t st, SetupBufs& sb) {
    const size_t ncell = (size_t)p->n[0] * p->n[1] * p->n[2];
    HIP_TRY(dev_malloc(&sb.Noct, 6 * ncell * sizeof(double)));
    std::vector<double> gx, gw;
    gauss_legendre(p->bands.gl_q, gx, gw);
    int rc = upload((void**)&sb.glx, gx);
    if (rc) return rc;
    rc = upload((void**)&sb.glw, gw);
    if (rc) return rc;
    double dt[3];
    reduced_cell(p->d, dt);
    HIP_TRY(launch_tensor_octant(st, p->n[0], p->n[1], p->n[2], dt, p->bands, sb.glx, sb.glw, sb.Noct));
    return DEMAG_OK;
}

template <typename T>
int setup_spectrum(demag_plan_s* p, hipStream_t st) {
    SetupBufs sb;
    int rc = compute_octant(p, st, sb);
    if (rc) return rc;
    const int Px = p->P[0], Py = p->P[1], Pz = p->P[2], Kx = p->Kx;
    const size_t nA = (size_t)Px * Py * Pz, nS = (size_t)Pz * Kx * Py;
    HIP_TRY(dev_malloc(&sb.A, nA * sizeof(double)));
    HIP_TRY(dev_malloc(&sb.B1, nS * sizeof(cx<double>)));
    HIP_TRY(dev_malloc(&sb.B2, nS * sizeof(cx<double>)));
    for (int k = 0; k < 3; ++k) {
        rc = upload(&sb.tw[k], twiddles<double>(p->P[k]));
        if (rc) return rc;
    }
    const size_t cb = sizeof(cx<double>);
    LaunchCfg xf = cfg_rows(Px, Py, cb), yf = cfg_pencils(Py, Kx, Pz, cb), zf;
    zf.t0 = (int)std::max<long>(1, std::min<long>(Py, 2048 / Pz));  // ky pencils per workgroup
    zf.E = pick_E((long)zf.t0 * Pz, zf.threads);
    const double scale = -1.0 / ((double)Px * Py * Pz);
    for (int comp = 0; comp < 6; ++comp) {
        HIP_TRY(launch_tensor_embed(st, comp, p->n[0], p->n[1], p->n[2], Px, Py, Pz, sb.Noct, sb.A));
        HIP_TRY(launch_x_fwd<double>(xf, st, sb.A, sb.B1, Px, Py, Pz, Kx, 1, p->fp[0], (const cx<double>*)sb.tw[0]));
        HIP_TRY(launch_y_fwd<double>(yf, st, sb.B1, sb.B2, Py, Pz, Kx, Pz, 1, p->fp[1], (const cx<double>*)sb.tw[1]));
        HIP_TRY(launch_z_fwd<double>(zf, st, sb.B2, Py, Kx, p->fp[2], (const cx<double>*)sb.tw[2]));
        HIP_TRY(launch_tensor_extract<T>(st, comp, Px, Py, Pz, Kx, scale, sb.B2, (T*)p->nhat));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return DEMAG_OK;
}

// Scalar-potential kernel: octant S_a (FP64, reduced units), odd mirror, FP64
// FFT passes, Im on the octant with h / (Px Py Pz) folded in (S scales as
// length: S_physical = h S_reduced, h the largest cell edge).
int compute_sp_octant(demag_plan_s* p, hipStream_t st, SetupBufs& sb) {
    const size_t ncell = (size_t)p->n[0] * p->n[1] * p->n[2];
    HIP_TRY(dev_malloc(&sb.Noct, 3 * ncell * sizeof(double)));
    std::vector<double> gx, gw;
    gauss_legendre(p->bands.gl_q, gx, gw);
    int rc = upload((void**)&sb.glx, gx);
    if (rc) return rc;
    rc = upload((void**)&sb.glw, gw);
    if (rc) return rc;
    double dt[3];
    reduced_cell(p->d, dt);
    HIP_TRY(launch_sp_kernel_octant(st, p->n[0], p->n[1], p->n[2], dt, p->bands, sb.glx, sb.glw, sb.Noct));
    return DEMAG_OK;
}

template <typename T>
int setup_sp_spectrum(demag_plan_s* p, hipStream_t st) {
    SetupBufs sb;
    int rc = compute_sp_octant(p, st, sb);
    if (rc) return rc;
    const int Px = p->P[0], Py = p->P[1], Pz = p->P[2], Kx = p->Kx;
    const size_t nA = (size_t)Px * Py * Pz, nS = (size_t)Pz * Kx * Py;
    HIP_TRY(dev_malloc(&sb.A, nA * sizeof(double)));
    HIP_TRY(dev_malloc(&sb.B1, nS * sizeof(cx<double>)));
    HIP_TRY(dev_malloc(&sb.B2, nS * sizeof(cx<double>)));
    for (int k = 0; k < 3; ++k) {
        rc = upload(&sb.tw[k], twiddles<double>(p->P[k]));
        if (rc) return rc;
    }
    const size_t cb = sizeof(cx<double>);
    LaunchCfg xf = cfg_rows(Px, Py, cb), yf = cfg_pencils(Py, Kx, Pz, cb), zf;
    zf.t0 = (int)std::max<long>(1, std::min<long>(Py, 2048 / Pz));  // ky pencils per workgroup
    zf.E = pick_E((long)zf.t0 * Pz, zf.threads);
    const double h = std::max(p->d[0], std::max(p->d[1], p->d[2]));
    const double scale = h / ((double)Px * Py * Pz);
    for (int a = 0; a < 3; ++a) {
        HIP_TRY(launch_sp_embed(st, a, p->n[0], p->n[1], p->n[2], Px, Py, Pz, sb.Noct, sb.A));
        HIP_TRY(launch_x_fwd<double>(xf, st, sb.A, sb.B1, Px, Py, Pz, Kx, 1, p->fp[0], (const cx<double>*)sb.tw[0]));
        HIP_TRY(launch_y_fwd<double>(yf, st, sb.B1, sb.B2, Py, Pz, Kx, Pz, 1, p->fp[1], (const cx<double>*)sb.tw[1]));
        HIP_TRY(launch_z_fwd<double>(zf, st, sb.B2, Py, Kx, p->fp[2], (const cx<double>*)sb.tw[2]));
        HIP_TRY(launch_sp_extract<T>(st, a, Py, Pz, Kx, scale, sb.B2, (T*)p->shat));
    }
    HIP_TRY(hipStreamSynchronize(st));
    return DEMAG_OK;
}

// Operands of the fused chain: the odd matrix on axis p for component p.
TGFused tg_fused_operands(const demag_plan_s* p) {
    const TGState* g = p->tg;
    const int R = g->R, b1 = R * tg_band_blocks(p->n[0]), b2 = R * tg_band_blocks(p->n[1]);
    const int* lo1E = g->band;
    const int* lo1O = lo1E + 2 * b1;
    const int* lo2E = lo1O + 2 * b1;
    const int* lo2O = lo2E + 2 * b2;
    TGFused f;
    for (int c = 0; c < 3; ++c) {
        const bool o1 = c == 0, o2 = c == 1;
        f.D1[c] = (const float*)(o1 ? g->D1O : g->D1E);
        f.D2[c] = (const float*)(o2 ? g->D2O : g->D2E);
        f.lo1[c] = o1 ? lo1O : lo1E;
        f.hi1[c] = f.lo1[c] + b1;
        f.lo2[c] = o2 ? lo2O : lo2E;
        f.hi2[c] = f.lo2[c] + b2;
    }
    return f;
}

// Mode-product flops per evaluation that the fused kernel issues (groups of 16
// columns outside a row block's band skipped) plus the dense mode-3 GEMMs.
double tg_fused_flops(const demag_plan_s* p, const std::vector<int>& band) {
    const int n1 = p->n[0], n2 = p->n[1], n3 = p->n[2], R = p->tg->R;
    const int nb1 = tg_band_blocks(n1), nb2 = tg_band_blocks(n2), b1 = R * nb1, b2 = R * nb2;
    auto span = [](int lo, int hi, int n) { return hi < 0 ? 0 : std::min(16 * ((hi >> 4) + 1), n) - 16 * (lo >> 4); };
    double f = 0;
    for (int c = 0; c < 3; ++c) {
        const int* lo1 = band.data() + (c == 0 ? 2 * b1 : 0);
        const int* lo2 = band.data() + 4 * b1 + (c == 1 ? 2 * b2 : 0);
        for (int l = 0; l < R; ++l) {
            for (int b = 0; b < nb1; ++b)
                f += 2.0 * std::min(64, n1 - 64 * b) * span(lo1[l * nb1 + b], lo1[b1 + l * nb1 + b], n1) * n2 * n3;
            for (int b = 0; b < nb2; ++b)
                f += 2.0 * n1 * std::min(64, n2 - 64 * b) * span(lo2[l * nb2 + b], lo2[b2 + l * nb2 + b], n2) * n3;
        }
    }
    return f + 3.0 * 2.0 * R * (double)n1 * n2 * n3 * n3;
}

// One tensor-grid evaluation: Phi by the GEMM chain into B2's memory, then
// the finite-difference gradient (and energy) as for SP.
template <typename T>
int run_tg_field(demag_plan_s* p, const T* m, double Ms, T* H, double* E_dev, hipStream_t st) {
    const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
    TGState* g = p->tg;
    T* phi = (T*)p->B2;
    T* Hout = H ? H : (T*)p->B1;
    const T* const* D2p[3] = {(const T* const*)g->D2kE, (const T* const*)g->D2kO, (const T* const*)g->D2kE};
    const T* B3[3] = {(const T*)g->B3E, (const T*)g->B3E, (const T*)g->B3O};
    const double hmax = std::max(p->d[0], std::max(p->d[1], p->d[2]));
    int rc = 0;
    if constexpr (std::is_same<T, float>::value) {
        if (g->fused) {
            const TGFused f = tg_fused_operands(p);
            rc = tg_potential_fused(g->handle, st, nx, ny, nz, g->R, m, f, B3, (float*)g->Y2, phi, Ms * hmax, g->sol3);
        }
    }
    if (!g->fused)
        rc = tg_potential<T>(g->handle, st, nx, ny, nz, g->R, m, (const T*)g->D1E, (const T*)g->D1O, D2p,
                             (const T* const*)g->Y1k, (T* const*)g->Y2k, B3, (T*)g->Y1, (T*)g->Y2, phi, Ms * hmax,
                             g->sol1, g->sol2, g->sol3);
    if (rc) return fail(DEMAG_EHIP, "tensor-grid GEMM failed (%d)", rc);
    int nparts = 0;
    HIP_TRY(launch_sp_gradient<T>(st, nx, ny, nz, p->d, phi, Hout, E_dev ? m : nullptr, E_dev ? p->partials : nullptr,
                                  &nparts));
    if (E_dev) {
        const double V = p->d[0] * p->d[1] * p->d[2];
        HIP_TRY(launch_energy_reduce(st, p->partials, nparts, -0.5 * kMu0 * Ms * V, E_dev));
    }
    return DEMAG_OK;
}

template <typename T>
int setup_tg(demag_plan_s* p, hipStream_t st, double step) {
    auto* g = new TGState();
    p->tg = g;
    const int n1 = p->n[0], n2 = p->n[1], n3 = p->n[2];
    const size_t N = (size_t)n1 * n2 * n3;
    double dt[3];
    reduced_cell(p->d, dt);
    const double rmin = std::min(dt[0], std::min(dt[1], dt[2]));
    const double rmax = std::sqrt((n1 * dt[0]) * (n1 * dt[0]) + (n2 * dt[1]) * (n2 * dt[1]) + (n3 * dt[2]) * (n3 * dt[2]));
    std::vector<double> tau, w;
    const int R = tg_sinc_nodes(rmin, std::max(rmax, rmin), step, tau, w);
    if (R <= 0) return fail(DEMAG_EINVAL, "tensor-grid quadrature");
    g->R = R;
    g->step = step;
    g->fused = std::is_same<T, float>::value && p->tg_mode12 == 1 && tg_mode12_fits(n2);
    const size_t sz = sizeof(T);
    const size_t nband = (size_t)4 * R * (tg_band_blocks(n1) + tg_band_blocks(n2));  // lo and hi of four matrices
    // the fused path keeps D1 and D2 in the tiled operand order (zero-padded to 16)
    const size_t mat1 = g->fused ? tg_tiled_floats(n1) : (size_t)n1 * n1;
    const size_t mat2 = g->fused ? tg_tiled_floats(n2) : (size_t)n2 * n2;
    const size_t need = sz * ((size_t)R * 2 * (mat1 + mat2) + 2 * (size_t)R * n3 * n3 +
                              (g->fused ? 1 : 2) * (size_t)R * N) +
                        (g->fused ? nband * sizeof(int) : 4 * sizeof(void*) * (size_t)R * n3);
    g->bytes = need;
    int rc = DEMAG_OK;
    auto alloc = [&](void** ptr, size_t bytes, const char* what) {
        if (rc) return;
        if (dev_malloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            rc = fail(DEMAG_ENOMEM, "cannot allocate %zu bytes for the tensor-grid %s", bytes, what);
        }
    };
    void *D3E = nullptr, *D3O = nullptr;
    alloc((void**)&g->tau, R * sizeof(double), "nodes");
    alloc((void**)&g->c, R * sizeof(double), "weights");
    alloc(&g->D1E, (size_t)R * mat1 * sz, "matrices");
    alloc(&g->D1O, (size_t)R * mat1 * sz, "matrices");
    alloc(&g->D2E, (size_t)R * mat2 * sz, "matrices");
    alloc(&g->D2O, (size_t)R * mat2 * sz, "matrices");
    alloc(&D3E, (size_t)R * n3 * n3 * sz, "matrices");
    alloc(&D3O, (size_t)R * n3 * n3 * sz, "matrices");
    alloc(&g->B3E, (size_t)R * n3 * n3 * sz, "mode-3 factors");
    alloc(&g->B3O, (size_t)R * n3 * n3 * sz, "mode-3 factors");
    alloc(&g->Y2, (size_t)R * N * sz, "scratch");
    const size_t nb = (size_t)R * n3;
    if (g->fused) {
        alloc((void**)&g->band, nband * sizeof(int), "band tables");
    } else {
        alloc(&g->Y1, (size_t)R * N * sz, "scratch");
        alloc((void**)&g->Y1k, nb * sizeof(void*), "pointer arrays");
        alloc((void**)&g->Y2k, nb * sizeof(void*), "pointer arrays");
        alloc((void**)&g->D2kE, nb * sizeof(void*), "pointer arrays");
        alloc((void**)&g->D2kO, nb * sizeof(void*), "pointer arrays");
    }
    if (!rc && hipMemcpy(g->tau, tau.data(), R * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(DEMAG_EHIP, "upload");
    if (!rc && hipMemcpy(g->c, w.data(), R * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(DEMAG_EHIP, "upload");
    if (!rc && !g->fused) {
        std::vector<void*> y1(nb), y2(nb), de(nb), dO(nb);
        for (int l = 0; l < R; ++l)
            for (int k = 0; k < n3; ++k) {
                const size_t b = (size_t)l * n3 + k, off = (size_t)l * N + (size_t)k * n1 * n2;
                y1[b] = (T*)g->Y1 + off;
                y2[b] = (T*)g->Y2 + off;
                de[b] = (T*)g->D2E + (size_t)l * n2 * n2;
                dO[b] = (T*)g->D2O + (size_t)l * n2 * n2;
            }
        if (hipMemcpy(g->Y1k, y1.data(), nb * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->Y2k, y2.data(), nb * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->D2kE, de.data(), nb * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(g->D2kO, dO.data(), nb * sizeof(void*), hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(DEMAG_EHIP, "upload");
    }
    if (!rc) {
        hipError_t e = hipSuccess;
        if constexpr (std::is_same<T, float>::value) {
            if (g->fused) {
                e = launch_tg_axis_tiled(st, n1, dt[0], R, g->tau, (float*)g->D1E, (float*)g->D1O);
                if (e == hipSuccess) e = launch_tg_axis_tiled(st, n2, dt[1], R, g->tau, (float*)g->D2E, (float*)g->D2O);
            }
        }
        if (!g->fused) {
            e = launch_tg_axis<T>(st, n1, dt[0], R, g->tau, (T*)g->D1E, (T*)g->D1O);
            if (e == hipSuccess) e = launch_tg_axis<T>(st, n2, dt[1], R, g->tau, (T*)g->D2E, (T*)g->D2O);
        }
        if (e == hipSuccess) e = launch_tg_axis<T>(st, n3, dt[2], R, g->tau, (T*)D3E, (T*)D3O);
        if (e == hipSuccess) e = launch_tg_stack3<T>(st, n3, R, g->c, (const T*)D3E, (T*)g->B3E);
        if (e == hipSuccess) e = launch_tg_stack3<T>(st, n3, R, g->c, (const T*)D3O, (T*)g->B3O);
        if constexpr (std::is_same<T, float>::value) {
            if (g->fused) {
                // bands of D1E, D1O, D2E, D2O (lo then hi per matrix)
                const size_t b1 = (size_t)R * tg_band_blocks(n1), b2 = (size_t)R * tg_band_blocks(n2);
                int* lo = g->band;
                const float* mats[4] = {(const float*)g->D1E, (const float*)g->D1O, (const float*)g->D2E,
                                        (const float*)g->D2O};
                for (int i = 0; i < 4 && e == hipSuccess; ++i) {
                    const size_t bi = i < 2 ? b1 : b2;
                    e = launch_tg_band(st, i < 2 ? n1 : n2, R, mats[i], lo, lo + bi);
                    lo += 2 * bi;
                }
                if (e == hipSuccess) e = tg_mode12_init(n2);
            }
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "tensor-grid setup");
    }
    if (!rc && g->fused) {
        std::vector<int> band(nband);
        if (hipMemcpy(band.data(), g->band, nband * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(DEMAG_EHIP, "band tables");
        else
            g->flops_issued = tg_fused_flops(p, band);
    } else if (!rc) {
        g->flops_issued = 3.0 * 2.0 * R * (double)N * (n1 + n2 + n3);
    }
    (void)hipFree(D3E);
    (void)hipFree(D3O);
    if (!rc) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) rc = fail(DEMAG_EHIP, "rocblas_create_handle failed");
        g->handle = h;
    }
    if (!rc) {
        // the mode-1 and mode-3 GEMMs' rocBLAS solutions, timed on the plan's buffers: a
        // mode-1 input and Y2 filled with a finite pattern (bytes 0x3C: 0.0115 in FP32) in
        // the plan's B1 scratch and in Y2, the plan's B2 scratch as the mode-3 output
        if (hipMemsetAsync(g->Y2, 0x3C, (size_t)R * N * sz, st) != hipSuccess ||
            hipMemsetAsync(p->B1, 0x3C, N * sz, st) != hipSuccess)
            rc = fail(DEMAG_EHIP, "tuning fill");
        if (!rc && tg_tune<T>(g->handle, st, n1, n2, n3, R, (const T*)g->D1E, (const T*)p->B1, (T*)g->Y1,
                              (const T* const*)g->Y1k, (const T* const*)g->D2kE, (T* const*)g->Y2k, (T*)g->Y2,
                              (const T*)g->B3E, (T*)p->B2, &g->sol1, &g->sol2, &g->sol3))
            rc = fail(DEMAG_EHIP, "tensor-grid GEMM tuning failed");
    }
    return rc;
}

int run_setup(demag_plan_s* p, hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    int rc = p->dtype == DEMAG_F32 ? setup_spectrum<float>(p, st) : setup_spectrum<double>(p, st);
    p->setup_us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

void free_tg(TGState* g) {
    if (!g) return;
    if (g->handle) rocblas_destroy_handle((rocblas_handle)g->handle);
    for (void* q : {(void*)g->tau, (void*)g->c, g->D1E, g->D1O, g->D2E, g->D2O, g->B3E, g->B3O, g->Y1, g->Y2,
                    (void*)g->Y1k, (void*)g->Y2k, (void*)g->D2kE, (void*)g->D2kO, (void*)g->band})
        (void)hipFree(q);
    delete g;
}

void free_lr(LRState* g) {
    if (!g) return;
    if (g->handle) rocblas_destroy_handle((rocblas_handle)g->handle);
    for (void* q : {(void*)g->tau, (void*)g->c, g->DE[0], g->DE[1], g->DE[2], g->DO[0], g->DO[1], g->DO[2],
                    (void*)g->partials, (void*)g->gram, g->W})
        (void)hipFree(q);
    delete g;
}

// Nodes (the dense TG quadrature: same range and step) and the stacked
// Gaussian matrices of the three axes.
template <typename T>
int setup_lr(demag_plan_s* p, hipStream_t st, double step) {
    auto* g = new LRState();
    p->lr = g;
    double dt[3];
    reduced_cell(p->d, dt);
    const int* n = p->n;
    const double rmin = std::min(dt[0], std::min(dt[1], dt[2]));
    const double rmax = std::sqrt((n[0] * dt[0]) * (n[0] * dt[0]) + (n[1] * dt[1]) * (n[1] * dt[1]) +
                                  (n[2] * dt[2]) * (n[2] * dt[2]));
    std::vector<double> tau, w;
    const int R = tg_sinc_nodes(rmin, std::max(rmax, rmin), step, tau, w);
    if (R <= 0) return fail(DEMAG_EINVAL, "tensor-grid quadrature");
    g->R = R;
    int rc = DEMAG_OK;
    auto alloc = [&](void** ptr, size_t bytes, const char* what) {
        if (rc) return;
        if (dev_malloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            rc = fail(DEMAG_ENOMEM, "cannot allocate %zu bytes for the low-rank %s", bytes, what);
        }
        g->bytes += bytes;
    };
    alloc((void**)&g->tau, R * sizeof(double), "nodes");
    alloc((void**)&g->c, R * sizeof(double), "weights");
    alloc((void**)&g->partials, 9 * (size_t)R * sizeof(double), "energy partials");
    for (int q = 0; q < 3; ++q) {
        const size_t per = sizeof(T) == 4 ? lr_swizzled_elems(n[q]) : (size_t)2 * n[q] * n[q];
        alloc(&g->DE[q], (size_t)R * per * sizeof(T), "Gaussian matrices");
        alloc(&g->DO[q], (size_t)R * per * sizeof(T), "Gaussian matrices");
    }
    if (!rc && (hipMemcpy(g->tau, tau.data(), R * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(g->c, w.data(), R * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))
        rc = fail(DEMAG_EHIP, "upload");
    if (!rc) {
        hipError_t e = hipSuccess;
        for (int q = 0; q < 3 && e == hipSuccess; ++q)
            e = sizeof(T) == 4 ? launch_lr_axis_sw(st, n[q], dt[q], R, g->tau, (float*)g->DE[q], (float*)g->DO[q])
                               : launch_lr_axis<T>(st, n[q], dt[q], p->d[q], R, g->tau, (T*)g->DE[q], (T*)g->DO[q]);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "low-rank tensor-grid setup");
    }
    if (!rc) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) rc = fail(DEMAG_EHIP, "rocblas_create_handle failed");
        g->handle = h;
    }
    return rc;
}

void free_plan(demag_plan_s* p) {
    for (auto t : p->tw) (void)hipFree(t);
    for (auto& axis : p->twt)
        for (auto t : axis) (void)hipFree(t);
    (void)hipFree(p->nhat);
    (void)hipFree(p->shat);
    free_tg(p->tg);
    free_lr(p->lr);
    if (p->als_handle) rocblas_destroy_handle((rocblas_handle)p->als_handle);
    (void)hipFree(p->B1);
    (void)hipFree(p->B2);
    (void)hipFree(p->partials);
    (void)hipFree(p->e_dev);
    if (p->done) (void)hipEventDestroy(p->done);
    for (auto e : p->tev) (void)hipEventDestroy(e);
    delete p;
}

// ---------------------------------------------------------------------------
// one evaluation: X-R2C -> Y -> Z (x N) -> Y^-1 -> X-C2R (+ energy)
// One pass of one evaluation with launch shape lc (which: 0 X-R2C, 1 Y, 2 fused
// Z, 3 Y-inverse, 4 X-C2R).  m: input of pass 0; H, me, partials, accumulate:
// outputs of pass 4.
template <typename T>
hipError_t launch_pass(demag_plan_s* p, int which, const LaunchCfg& lc, hipStream_t st, const T* m, double Ms, T* H,
                       const T* me, double* partials, int accumulate, const BatchIO& bio = BatchIO()) {
    const int nx = p->n[0], ny = p->n[1], nz = p->n[2], Kx = p->Kx;
    const int Px = p->P[0], Py = p->P[1], Pz = p->P[2];
    auto* B1 = (cx<T>*)p->B1;
    auto* B2 = (cx<T>*)p->B2;
    const auto* twx = (const cx<T>*)p->tw[0];
    const auto* twy = (const cx<T>*)p->tw[1];
    const auto* twz = (const cx<T>*)p->tw[2];
    const int sc = lc.p2 && lc.sched >= 0 && lc.sched < 3 ? lc.sched : 0;
    const auto* ttx = (const cx<T>*)p->twt[0][sc];
    const auto* tty = (const cx<T>*)p->twt[1][sc];
    const auto* ttz = (const cx<T>*)p->twt[2][sc];
    switch (which) {
    case 0:
        return lc.p2 ? launch_x_fwd_p2<T>(lc.t0, lc.sched, st, m, B1, nx, ny, nz, 3, Px, ttx, bio)
                     : launch_x_fwd<T>(lc, st, m, B1, nx, ny, nz, Kx, 3, p->fp[0], twx, bio);
    case 1:
        return lc.p2 ? launch_y_fwd_p2<T>(lc.t1, lc.t0, lc.sched, st, B1, B2, ny, nz, Kx, 3, Py, tty, bio)
                     : launch_y_fwd<T>(lc, st, B1, B2, ny, nz, Kx, nz, 3, p->fp[1], twy, bio);
    case 2:
        return lc.p2 ? launch_z_conv_p2<T>(lc.t0, lc.t1, lc.sched, st, B2, (const T*)p->nhat, (T)Ms, nz, Py, Kx, Pz,
                                           ttz, bio)
                     : launch_z_conv<T>(lc, st, B2, (const T*)p->nhat, (T)Ms, nz, Py, Kx, p->fp[2], twz, bio);
    case 3:
        return lc.p2 ? launch_y_inv_p2<T>(lc.t1, lc.t0, lc.sched, st, B2, B1, ny, nz, Kx, 3, Py, tty, bio)
                     : launch_y_inv<T>(lc, st, B2, B1, ny, nz, Kx, 3, p->fp[1], twy, bio);
    default:
        return lc.p2 ? launch_x_inv_p2<T>(lc.t0, lc.sched, st, B1, H, me, partials, nx, ny, nz, 3, accumulate, Px, ttx,
                                          bio)
                     : launch_x_inv<T>(lc, st, B1, H, me, partials, nx, ny, nz, Kx, 3, accumulate, p->fp[0], twx,
                                       bio);
    }
}

const LaunchCfg& pass_cfg(const PassCfgs& c, int which) {
    const LaunchCfg* slot[5] = {&c.xf, &c.yf, &c.zc, &c.yi, &c.xi};
    return *slot[which];
}

// The caller's stream is being captured into a graph: the plan's busy
// tracking (an event query, an event record) and its pass timing stay out of
// the capture.
bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
}

// one evaluation: X-R2C -> Y -> Z (x N) -> Y^-1 -> X-C2R (+ energy)
template <typename T>
int run_field(demag_plan_s* p, const PassCfgs& c, const T* m, double Ms, T* H, const T* m_energy, double* E_dev,
              int accumulate, hipStream_t st) {
    hipEvent_t* mark = nullptr;
    if (p->tcap > 0 && !stream_capturing(st))
        mark = &p->tev[(size_t)(p->tcount % p->tcap) * kPassMarks];
    double* partials = E_dev ? p->partials : nullptr;
    const T* me = E_dev ? m_energy : nullptr;
    static const char* const kPassNames[5] = {"x_r2c", "y_fwd", "z_conv", "y_inv", "x_c2r"};
    for (int which = 0; which < 5; ++which) {
        const Range range_(kPassNames[which]);
        if (mark) HIP_TRY(hipEventRecord(mark[which], st));
        HIP_TRY(launch_pass<T>(p, which, pass_cfg(c, which), st, m, Ms, H, me, partials, accumulate));
    }
    if (mark) HIP_TRY(hipEventRecord(mark[5], st));
    if (E_dev) {
        const int Ty = c.xi.p2 ? (1 << c.xi.t0) : c.xi.t0;
        const int ny = p->n[1], nz = p->n[2];
        const int nparts = ((ny + Ty - 1) / Ty) * nz * 3;
        const double V = p->d[0] * p->d[1] * p->d[2];
        HIP_TRY(launch_energy_reduce(st, p->partials, nparts, -0.5 * kMu0 * Ms * V, E_dev));
    }
    if (mark) {
        HIP_TRY(hipEventRecord(mark[6], st));
        ++p->tcount;
    }
    return DEMAG_OK;
}

// One scalar-potential evaluation: the DM forward X and Y passes on m, the
// fused SP Z pass (phi^ into component 0 of B2), one-component Y-inverse and
// X-C2R (phi into B2's memory), the gradient (H; energy partials when E_dev).
template <typename T>
int run_sp_field(demag_plan_s* p, const T* m, double Ms, T* H, double* E_dev, hipStream_t st) {
    const int nx = p->n[0], ny = p->n[1], nz = p->n[2], Kx = p->Kx;
    const int Px = p->P[0], Py = p->P[1], Pz = p->P[2];
    auto* B1 = (cx<T>*)p->B1;
    auto* B2 = (cx<T>*)p->B2;
    T* phi = (T*)p->B2;                 // free once the Y-inverse has read B2
    T* Hout = H ? H : (T*)p->B1;        // energy only: the field goes to scratch
    const PassCfgs& c = p->cfg;
    HIP_TRY(launch_pass<T>(p, 0, c.xf, st, m, Ms, nullptr, nullptr, nullptr, 0));
    HIP_TRY(launch_pass<T>(p, 1, c.yf, st, nullptr, Ms, nullptr, nullptr, nullptr, 0));
    HIP_TRY(launch_z_sp_p2<T>(p->zs.t0, p->zs.t1, p->zs.sched, st, B2, (const T*)p->shat, (T)Ms, nz, Py, Kx, Pz,
                              (const cx<T>*)p->twt[2][p->zs.sched]));
    const LaunchCfg& yi = c.yi;
    HIP_TRY(yi.p2 ? launch_y_inv_p2<T>(yi.t1, yi.t0, yi.sched, st, B2, B1, ny, nz, Kx, 1, Py,
                                       (const cx<T>*)p->twt[1][yi.sched])
                  : launch_y_inv<T>(yi, st, B2, B1, ny, nz, Kx, 1, p->fp[1], (const cx<T>*)p->tw[1]));
    const LaunchCfg& xi = c.xi;
    HIP_TRY(xi.p2 ? launch_x_inv_p2<T>(xi.t0, xi.sched, st, B1, phi, nullptr, nullptr, nx, ny, nz, 1, 0, Px,
                                       (const cx<T>*)p->twt[0][xi.sched])
                  : launch_x_inv<T>(xi, st, B1, phi, nullptr, nullptr, nx, ny, nz, Kx, 1, 0, p->fp[0],
                                    (const cx<T>*)p->tw[0]));
    int nparts = 0;
    HIP_TRY(launch_sp_gradient<T>(st, nx, ny, nz, p->d, phi, Hout, E_dev ? m : nullptr, E_dev ? p->partials : nullptr,
                                  &nparts));
    if (E_dev) {
        const double V = p->d[0] * p->d[1] * p->d[2];
        HIP_TRY(launch_energy_reduce(st, p->partials, nparts, -0.5 * kMu0 * Ms * V, E_dev));
    }
    return DEMAG_OK;
}


// The energy alone (no field): X-R2C, Y, then the fused Z pass's forward half
// with the quadratic form of Parseval's identity in place of the product and
// the inverse passes (sum_i m_i . (N * m)_i = sum_k Re(M^H Nhat M) on the
// padded grid, m being zero off the grid), partials summed in a fixed order.
// Three passes instead of five; B2 is only read by the third.
template <typename T>
int run_energy_only(demag_plan_s* p, const PassCfgs& c, const T* m, double Ms, double* E_dev, hipStream_t st) {
    static const char* const kPassNames[3] = {"x_r2c", "y_fwd", "z_energy"};
    {
        const Range range_(kPassNames[0]);
        HIP_TRY(launch_pass<T>(p, 0, c.xf, st, m, Ms, nullptr, nullptr, nullptr, 0));
    }
    {
        const Range range_(kPassNames[1]);
        HIP_TRY(launch_pass<T>(p, 1, c.yf, st, nullptr, Ms, nullptr, nullptr, nullptr, 0));
    }
    const LaunchCfg& z = c.zc;
    const int sc = z.sched >= 0 && z.sched < 3 ? z.sched : 0;
    int nparts = 0;
    {
        const Range range_(kPassNames[2]);
        HIP_TRY(launch_z_energy_p2<T>(z.t0, z.t1, sc, st, (cx<T>*)p->B2, (const T*)p->nhat, p->n[2], p->P[1], p->Kx,
                                      p->P[2], (const cx<T>*)p->twt[2][sc], p->partials, &nparts));
    }
    if (nparts > p->npartials) return fail(DEMAG_EHIP, "energy partials exceed their buffer");
    const double V = p->d[0] * p->d[1] * p->d[2];
    HIP_TRY(launch_energy_reduce(st, p->partials, nparts, -0.5 * kMu0 * Ms * Ms * V, E_dev));
    return DEMAG_OK;
}

int dispatch_field(demag_plan_s* p, const void* m, double Ms, void* H, double* E_dev, int accumulate,
                   hipStream_t st) {
    if (!H && E_dev && p->cfg.zc.p2 && !accumulate)
        return p->dtype == DEMAG_F32 ? run_energy_only<float>(p, p->cfg, (const float*)m, Ms, E_dev, st)
                                     : run_energy_only<double>(p, p->cfg, (const double*)m, Ms, E_dev, st);
    if (p->dtype == DEMAG_F32)
        return run_field<float>(p, p->cfg, (const float*)m, Ms, (float*)H, (const float*)m, E_dev, accumulate, st);
    return run_field<double>(p, p->cfg, (const double*)m, Ms, (double*)H, (const double*)m, E_dev, accumulate, st);
}

// One plan on one stream at a time: refuse a call on another stream while
// the plan's previous work is still pending.
int enter(demag_plan_s* p, hipStream_t st) {
    if (stream_capturing(st)) return DEMAG_OK;
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != p->device) return fail(DEMAG_ESTATE, "plan was created on device %d, current device is %d", p->device, cur);
    if (p->used && st != p->last_stream && p->busy) {
        hipError_t q = hipEventQuery(p->busy);
        if (q == hipErrorNotReady)
            return fail(DEMAG_ESTATE, "plan is still busy on another stream");
        if (q != hipSuccess) return hip_fail(q, "hipEventQuery");
    }
    return DEMAG_OK;
}

int leave(demag_plan_s* p, hipStream_t st) {
    if (stream_capturing(st)) return DEMAG_OK;
    HIP_TRY(hipEventRecord(p->done, st));
    p->busy = p->done;
    p->last_stream = st;
    p->used = true;
    return DEMAG_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

// LLG Heun steps (Sec. 2) on the workspace `work` (9 N values of the plan
// precision: H, k1, the predictor; nothing is allocated).
int llg_heun_impl(demag_plan_s* p, void* m, double Ms, double alpha, double gamma, double hx, double hy, double hz,
                  double dt, int nsteps, void* work, void* stream) {
    if (!p || !m || !work) return fail(DEMAG_EINVAL, "NULL plan, m or work");
    if (!std::isfinite(Ms) || !(alpha >= 0) || !std::isfinite(alpha) || !(gamma > 0) || !std::isfinite(gamma) ||
        !std::isfinite(hx) || !std::isfinite(hy) || !std::isfinite(hz) || !(dt > 0) || !std::isfinite(dt) || nsteps < 0)
        return fail(DEMAG_EINVAL, "need finite Ms, alpha >= 0, gamma > 0, finite H_ext, dt > 0, nsteps >= 0");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const size_t N = (size_t)p->n[0] * p->n[1] * p->n[2];
    const double hext[3] = {hx, hy, hz};
    const double g = gamma / (1.0 + alpha * alpha);
    auto steps = [&](auto proto) -> int {
        using T = decltype(proto);
        T* mm = (T*)m;
        T* H = (T*)work;
        T* k1 = H + 3 * N;
        T* ms = k1 + 3 * N;
        for (int s = 0; s < nsteps; ++s) {
            int r = run_field<T>(p, p->cfg, mm, Ms, H, nullptr, nullptr, 0, st);
            if (r) return r;
            HIP_TRY(launch_llg_predict<T>(st, N, mm, H, hext, g, alpha, dt, k1, ms));
            r = run_field<T>(p, p->cfg, ms, Ms, H, nullptr, nullptr, 0, st);
            if (r) return r;
            HIP_TRY(launch_llg_correct<T>(st, N, mm, H, k1, ms, hext, g, alpha, dt));
        }
        return DEMAG_OK;
    };
    rc = p->dtype == DEMAG_F32 ? steps(float()) : steps(double());
    if (rc) return rc;
    return leave(p, st);
}

// Workspace of demag_llg_heun_static, for callers that cannot allocate: a
// file-scope device array, which every GPU the library runs on holds from the
// library's load until the process ends.  In host code its name stands for
// the symbol only; its device address comes from hipGetSymbolAddress, looked
// up once per device (with that device current) and kept.  Nothing in it
// needs to start at zero (each step writes H, k1 and the predictor before
// reading them); calls on one device share it, so calls that overlap race.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DEMAG_EUNSUPPORTED, "device %d beyond the static scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(DEMAG_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DEMAG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
template <typename T>
int run_compress(demag_plan_s* p, hipStream_t st, int format, int r, int sweeps, const T* m, T* core, T* U,
                 double* relerr) {
    const int* n = p->n;
    const int nmax = std::max(n[0], std::max(n[1], n[2]));
    const size_t rr = (size_t)r * r, r3 = rr * r;
    const size_t nT = std::max((size_t)n[0] * n[1], (size_t)n[1] * n[2]) * r;
    const size_t nY = (size_t)nmax * rr, nW = r3, nP = (size_t)nmax * r, nQ = std::max((size_t)nmax * r, r3);
    const size_t elems = nT + nY + nW + nP + nQ + rr;
    const size_t dbl = 4 * rr + 1024 + 1 + 6;
    void* buf = nullptr;
    const size_t bytes = elems * sizeof(T) + dbl * sizeof(double) + 64;
    if (dev_malloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DEMAG_ENOMEM, "cannot allocate %zu bytes of ALS scratch", bytes);
    }
    double* d = (double*)buf;
    AlsScratch<T> w;
    for (int i = 0; i < 4; ++i) w.G[i] = d + i * rr;
    w.partials = d + 4 * rr;
    w.scal = w.partials + 1024;
    double* err2 = w.scal + 1;
    w.flag = (int*)(err2 + 6);
    T* t = (T*)((char*)buf + dbl * sizeof(double) + 64);
    w.Tm = t;
    w.Y = w.Tm + nT;
    w.W = w.Y + nY;
    w.P = w.W + nW;
    w.Q = w.P + nP;
    w.Rinv = w.Q + nQ;
    int rc = DEMAG_OK;
    if (!p->als_handle) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) rc = fail(DEMAG_EHIP, "rocblas_create_handle failed");
        p->als_handle = h;
    }
    double e2[6] = {0, 0, 0, 0, 0, 0};
    int flag = 0;
    if (!rc) {
        hipError_t e = hipMemsetAsync(w.flag, 0, sizeof(int), st);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemsetAsync");
    }
    if (!rc) {
        const int k = als_compress<T>(p->als_handle, st, n, r, format == DEMAG_TUCKER, sweeps, m, core, U, err2, w);
        if (k) rc = fail(DEMAG_EHIP, "ALS compression failed (%d)", k);
    }
    if (!rc) {
        hipError_t e = hipMemcpyAsync(e2, err2, sizeof(e2), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "ALS compression");
    }
    (void)hipFree(buf);
    if (rc) return rc;
    if (flag)
        return fail(DEMAG_EINVAL, "a Gram matrix of the factors is not positive definite (rank %d above the "
                                  "numerical rank of the data or of the initial guess)", r);
    if (relerr) {
        const double res = e2[0] + e2[2] + e2[4], xx = e2[1] + e2[3] + e2[5];
        *relerr = xx > 0 ? std::sqrt(std::max(0.0, res) / xx) : 0.0;
    }
    return DEMAG_OK;
}

extern "C" {

const char* demag_last_error(void) { return g_last_error.c_str(); }

int demag_plan_create(demag_plan_t* out, int nx, int ny, int nz, double dx, double dy, double dz,
                      demag_dtype dtype, void* setup_stream) {
    const Range range_("demag_plan_create");
    if (!out) return fail(DEMAG_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(DEMAG_EINVAL, "grid must be at least 1x1x1 (got %d x %d x %d)", nx, ny, nz);
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(DEMAG_EINVAL, "cell sizes must be finite and > 0");
    if (dtype != DEMAG_F32 && dtype != DEMAG_F64) return fail(DEMAG_EINVAL, "unknown dtype %d", (int)dtype);
    const int n[3] = {nx, ny, nz};
    int L[3], P[3];
    for (int k = 0; k < 3; ++k) {
        if (n[k] > kMaxLen / 2) return fail(DEMAG_EUNSUPPORTED, "axis %d: n = %d exceeds %d", k, n[k], kMaxLen / 2);
        L[k] = smooth_at_least(n[k]);
        P[k] = 2 * L[k];
        if (P[k] > kMaxLen) return fail(DEMAG_EUNSUPPORTED, "axis %d: padded length %d exceeds %d", k, P[k], kMaxLen);
        const size_t cb = dtype == DEMAG_F32 ? sizeof(cx<float>) : sizeof(cx<double>);
        if ((size_t)P[k] * cb > kMaxLdsBytes || (size_t)P[k] * sizeof(cx<double>) > kMaxLdsBytes)
            return fail(DEMAG_EUNSUPPORTED, "axis %d: padded length %d does not fit one LDS pencil in FP64", k, P[k]);
    }
    const int Kx = P[0] / 2 + 1;
    // all device buffers are indexed with 64-bit bases; per-dimension extents fit in int
    const long double big = (long double)P[0] * P[1] * P[2];
    if (big > 4.0e12L) return fail(DEMAG_EINVAL, "padded grid too large");

    auto* p = new demag_plan_s();
    for (int k = 0; k < 3; ++k) {
        p->n[k] = n[k];
        p->L[k] = L[k];
        p->P[k] = P[k];
        p->fp[k] = make_fft_plan(P[k]);
    }
    p->d[0] = dx;
    p->d[1] = dy;
    p->d[2] = dz;
    p->dtype = dtype;
    p->Kx = Kx;
    if (const char* xe = getenv("DEMAG_XCDS")) {  // workgroup swizzle width (1 = off)
        int v = atoi(xe);
        if (v >= 1 && v <= 64) kXcds = v;
    }
    hipError_t he = hipGetDevice(&p->device);
    if (he != hipSuccess) {
        delete p;
        return hip_fail(he, "hipGetDevice");
    }
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) == hipSuccess &&
        lds_max >= 65536)
        g_p2_lds = std::min<size_t>((size_t)lds_max, 163840);
    hipStream_t st = (hipStream_t)setup_stream;
    const size_t cb = csize(dtype), rb = dtype == DEMAG_F32 ? 4 : 8;
    const size_t nB1 = 3ull * nz * Kx * ny, nB2 = 3ull * P[1] * Kx * nz;
    const size_t nH = (size_t)(P[1] / 2 + 1) * 6 * Kx * (P[2] / 2 + 1);
    p->cfg = default_cfgs(p);
    if (!one_cfg_ok(p->cfg.zc, P[2], cb, 2)) {
        // the register Z kernel holds a pencil and its mirror in one workgroup
        // (2 P / 8 threads <= 512, i.e. P <= 2048, or 3 * 2^a in FP32); the LDS
        // kernel holds six pencils (6 P complex values within a workgroup's LDS)
        const LaunchCfg g = cfg_zconv(P[2], Kx, cb);
        if (!one_cfg_ok(g, P[2], cb, 2)) {
            const int pz = P[2];
            free_plan(p);
            return fail(DEMAG_EUNSUPPORTED,
                        "z axis: no fused Z pass for padded length %d in %s (register kernel: powers of two up to "
                        "2048, and 3 * 2^a in FP32; LDS kernel: 6 P complex values within a workgroup's LDS)",
                        pz, dtype == DEMAG_F32 ? "FP32" : "FP64");
        }
        p->cfg.zc = g;
    }
    int rc = DEMAG_OK;
    auto alloc = [&](void** ptr, size_t bytes, const char* what) {
        if (rc) return;
        if (dev_malloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            rc = fail(DEMAG_ENOMEM, "cannot allocate %zu bytes for %s", bytes, what);
        }
    };
    alloc(&p->B1, nB1 * cb, "spectrum scratch B1");
    alloc(&p->B2, nB2 * cb, "spectrum scratch B2");
    alloc(&p->nhat, nH * rb, "tensor spectrum");
    // upper bound: X-inverse tiles of >= 2 rows; gradient workgroups (SP, TG);
    // fused-Z workgroups of the energy alone (at most Kx Py)
    p->npartials = (int)std::max<long>(std::max<long>(3L * nz * ((ny + 1) / 2), sp_gradient_tiles(nx, ny, nz, 1)),
                                       (long)Kx * P[1]);
    alloc((void**)&p->partials, (size_t)p->npartials * sizeof(double), "energy partials");
    alloc((void**)&p->e_dev, sizeof(double), "energy scalar");
    p->scratch_bytes = (nB1 + nB2) * cb;
    p->tensor_bytes = nH * rb;
    if (!rc) {
        auto tables = [&](auto proto, int k) {
            using T = decltype(proto);
            const std::vector<cx<T>> tw = twiddles<T>(P[k]);
            int r = upload(&p->tw[k], tw);
            for (int sc = 0; !r && sc < p2_num_schedules(P[k]); ++sc)
                r = upload(&p->twt[k][sc], p2_thread_twiddles<T>(P[k], sc, tw));
            return r;
        };
        for (int k = 0; k < 3 && !rc; ++k) rc = dtype == DEMAG_F32 ? tables(float(), k) : tables(double(), k);
    }
    if (!rc && hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess)
        rc = fail(DEMAG_EHIP, "hipEventCreate failed");
    if (!rc) rc = run_setup(p, st);
    if (rc) {
        free_plan(p);
        return rc;
    }
    *out = p;
    return DEMAG_OK;
}

int demag_plan_set_option(demag_plan_t p, const char* key, double value) {
    if (!p || !key) return fail(DEMAG_EINVAL, "NULL plan or key");
    TensorBands b = p->bands;
    if (!strcmp(key, "far_cut") || !strcmp(key, "far_cutoff")) {
        if (!(value > 0) || std::isnan(value)) return fail(DEMAG_EINVAL, "far_cut must be > 0");
        b.far_cut = value;
    } else if (!strcmp(key, "fg_cut") || !strcmp(key, "fg_cutoff")) {
        if (!(value >= 0) || value != std::floor(value) || value > 1e9)
            return fail(DEMAG_EINVAL, "fg_cut must be a non-negative integer");
        b.fg_cut = (int)value;
    } else if (!strcmp(key, "generic_kernels")) {
        if (value != 0 && value != 1) return fail(DEMAG_EINVAL, "generic_kernels must be 0 or 1");
        const size_t cb = csize(p->dtype);
        PassCfgs c = value == 1 ? generic_cfgs(p) : default_cfgs(p);
        if (!one_cfg_ok(c.zc, p->P[2], cb, 2)) {
            if (value == 1)
                return fail(DEMAG_EUNSUPPORTED, "generic kernels: padded z length %d needs more LDS than a workgroup has",
                            p->P[2]);
            c.zc = cfg_zconv(p->P[2], p->Kx, cb);  // as at plan creation, where this fallback was verified
        }
        HIP_TRY(hipDeviceSynchronize());
        p->cfg = c;
        return DEMAG_OK;
    } else if (!strcmp(key, "pass_timing")) {
        if (!(value >= 0) || value != std::floor(value) || value > 1e6)
            return fail(DEMAG_EINVAL, "pass_timing must be an integer in [0, 1e6]");
        HIP_TRY(hipDeviceSynchronize());
        for (auto e : p->tev) (void)hipEventDestroy(e);
        p->tev.assign((size_t)value * kPassMarks, nullptr);
        for (auto& e : p->tev) HIP_TRY(hipEventCreate(&e));
        p->tcap = (int)value;
        p->tcount = 0;
        return DEMAG_OK;
    } else if (!strcmp(key, "radix_schedule")) {
        if (value != 0 && value != 1 && value != 2) return fail(DEMAG_EINVAL, "radix_schedule must be 0, 1 or 2");
        HIP_TRY(hipDeviceSynchronize());
        LaunchCfg* slot[5] = {&p->cfg.xf, &p->cfg.yf, &p->cfg.zc, &p->cfg.yi, &p->cfg.xi};
        for (int w = 0; w < 5; ++w) {
            const int P = p->P[w == 0 || w == 4 ? 0 : w == 2 ? 2 : 1];
            if (slot[w]->p2) slot[w]->sched = (int)value < p2_num_schedules(P) ? (int)value : 0;
        }
        return DEMAG_OK;
    } else if (!strcmp(key, "tg_mode12")) {
        if (value != 0 && value != 1) return fail(DEMAG_EINVAL, "tg_mode12 must be 0 or 1");
        if (p->tg_mode12 == (int)value) return DEMAG_OK;
        p->tg_mode12 = (int)value;
        if (!p->tg) return DEMAG_OK;
        // a prepared tensor grid is rebuilt for the other path
        HIP_TRY(hipDeviceSynchronize());
        free_tg(p->tg);
        p->tg = nullptr;
        return demag_tg_prepare(p, nullptr);
    } else if (!strcmp(key, "lowrank_scratch")) {
        if (!(value >= 0) || value > 1e15) return fail(DEMAG_EINVAL, "lowrank_scratch must be in [0, 1e15] bytes");
        p->lr_cap = (size_t)value;
        return DEMAG_OK;
    } else {
        return fail(DEMAG_EINVAL, "unknown option '%s'", key);
    }
    HIP_TRY(hipDeviceSynchronize());
    p->bands = b;
    return run_setup(p, nullptr);
}

int demag_plan_destroy(demag_plan_t p) {
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    (void)hipDeviceSynchronize();
    free_plan(p);
    return DEMAG_OK;
}

int demag_plan_info(demag_plan_t p, int64_t* info) {
    if (!p || !info) return fail(DEMAG_EINVAL, "NULL argument");
    int64_t v[16] = {p->n[0], p->n[1], p->n[2], p->P[0], p->P[1], p->P[2], p->Kx, (int64_t)p->dtype,
                     (int64_t)p->scratch_bytes, (int64_t)p->tensor_bytes, (int64_t)p->setup_us, 0, 0, 0, 0, 0};
    memcpy(info, v, sizeof v);
    return DEMAG_OK;
}

int demag_field(demag_plan_t p, const void* m, double Ms, void* H, void* stream) {
    const Range range_("demag_field");
    if (!p || !m || !H) return fail(DEMAG_EINVAL, "NULL plan, m or H");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = dispatch_field(p, m, Ms, H, nullptr, 0, st);
    if (rc) return rc;
    return leave(p, st);
}

int demag_field_adjoint(demag_plan_t p, const void* gH, double Ms, void* gm, int accumulate, void* stream) {
    const Range range_("demag_field_adjoint");
    if (!p || !gH || !gm) return fail(DEMAG_EINVAL, "NULL plan, gH or gm");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    if (accumulate != 0 && accumulate != 1) return fail(DEMAG_EINVAL, "accumulate must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = dispatch_field(p, gH, Ms, gm, nullptr, accumulate, st);
    if (rc) return rc;
    return leave(p, st);
}

int demag_field_energy(demag_plan_t p, const void* m, double Ms, void* H, double* E_dev, void* stream) {
    const Range range_("demag_field_energy");
    if (!p || !m || !E_dev) return fail(DEMAG_EINVAL, "NULL plan, m or E_dev");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = dispatch_field(p, m, Ms, H, E_dev, 0, st);
    if (rc) return rc;
    return leave(p, st);
}

int demag_energy_async(demag_plan_t p, const void* m, double Ms, double* E_dev, void* stream) {
    const Range range_("demag_energy_async");
    return demag_field_energy(p, m, Ms, nullptr, E_dev, stream);
}

int demag_energy_gradient(demag_plan_t p, const void* H, double Ms, const double* gE_dev, void* gm, int accumulate,
                          void* stream) {
    const Range range_("demag_energy_gradient");
    if (!p || !H || !gm) return fail(DEMAG_EINVAL, "NULL plan, H or gm");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    if (H == gm) return fail(DEMAG_EINVAL, "H and gm must be distinct buffers");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const size_t n = 3ull * p->n[0] * p->n[1] * p->n[2];
    const double c = -kMu0 * Ms * p->d[0] * p->d[1] * p->d[2];
    HIP_TRY(p->dtype == DEMAG_F32
                ? launch_energy_grad<float>(st, n, (const float*)H, gE_dev, c, (float*)gm, accumulate ? 1 : 0)
                : launch_energy_grad<double>(st, n, (const double*)H, gE_dev, c, (double*)gm, accumulate ? 1 : 0));
    return leave(p, st);
}

int demag_energy(demag_plan_t p, const void* m, double Ms, double* E_host, void* stream) {
    const Range range_("demag_energy");
    if (!E_host) return fail(DEMAG_EINVAL, "E_host is NULL");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    int rc = demag_field_energy(p, m, Ms, nullptr, p->e_dev, stream);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(E_host, p->e_dev, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return DEMAG_OK;
}

int demag_plan_spectrum(demag_plan_t p, void* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    HIP_TRY(hipDeviceSynchronize());
    std::vector<unsigned char> dev(p->tensor_bytes);
    HIP_TRY(hipMemcpy(dev.data(), p->nhat, p->tensor_bytes, hipMemcpyDeviceToHost));
    // device [Kx][Ly+1][Lz+1][6] -> documented [Ly+1][6][Kx][Lz+1]
    const size_t rb = p->dtype == DEMAG_F32 ? 4 : 8;
    const size_t Ly1 = p->P[1] / 2 + 1, Kx = p->Kx, Lz1 = p->P[2] / 2 + 1;
    unsigned char* o = (unsigned char*)out;
    for (size_t ky = 0; ky < Ly1; ++ky)
        for (size_t kx = 0; kx < Kx; ++kx)
            for (size_t kz = 0; kz < Lz1; ++kz)
                for (size_t c = 0; c < 6; ++c)
                    std::memcpy(o + (((ky * 6 + c) * Kx + kx) * Lz1 + kz) * rb,
                                dev.data() + (((kx * Ly1 + ky) * Lz1 + kz) * 6 + c) * rb, rb);
    return DEMAG_OK;
}

int demag_plan_tensor(demag_plan_t p, double* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    HIP_TRY(hipDeviceSynchronize());
    SetupBufs sb;
    int rc = compute_octant(p, nullptr, sb);
    if (rc) return rc;
    const size_t ncell = (size_t)p->n[0] * p->n[1] * p->n[2];
    HIP_TRY(hipMemcpy(out, sb.Noct, 6 * ncell * sizeof(double), hipMemcpyDeviceToHost));
    return DEMAG_OK;
}

int demag_sp_prepare(demag_plan_t p, void* stream) {
    const Range range_("demag_sp_prepare");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    if (p->shat) return DEMAG_OK;
    const size_t cb = csize(p->dtype), rb = cb / 2;
    const LaunchCfg zs = p->cfg.zc.p2 ? p->cfg.zc : p2_zconv(p->P[2], p->P[1], cb);
    if (!p2_z_supported(p->P[2], cb) || !p2_z_ranges_ok(p) || !p2_cfg_ok(zs, p->P[2], cb, 2))
        return fail(DEMAG_EUNSUPPORTED, "scalar-potential method: padded z length %d not supported in %s", p->P[2],
                    p->dtype == DEMAG_F32 ? "FP32" : "FP64");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const size_t bytes = (size_t)(p->P[1] / 2 + 1) * 3 * p->Kx * (p->P[2] / 2 + 1) * rb;
    if (dev_malloc(&p->shat, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->shat = nullptr;
        return fail(DEMAG_ENOMEM, "cannot allocate %zu bytes for the scalar-potential spectrum", bytes);
    }
    rc = p->dtype == DEMAG_F32 ? setup_sp_spectrum<float>(p, st) : setup_sp_spectrum<double>(p, st);
    if (rc) {
        (void)hipFree(p->shat);
        p->shat = nullptr;
        return rc;
    }
    p->zs = zs;
    return leave(p, st);
}

int demag_sp_field_energy(demag_plan_t p, const void* m, double Ms, void* H, double* E_dev, void* stream) {
    const Range range_("demag_sp_field_energy");
    if (!p || !m || (!H && !E_dev)) return fail(DEMAG_EINVAL, "NULL plan or m, or neither H nor E_dev");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    if (!p->shat) return fail(DEMAG_ESTATE, "scalar-potential method not prepared (call demag_sp_prepare)");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = p->dtype == DEMAG_F32 ? run_sp_field<float>(p, (const float*)m, Ms, (float*)H, E_dev, st)
                               : run_sp_field<double>(p, (const double*)m, Ms, (double*)H, E_dev, st);
    if (rc) return rc;
    return leave(p, st);
}

int demag_sp_field(demag_plan_t p, const void* m, double Ms, void* H, void* stream) {
    if (!H) return fail(DEMAG_EINVAL, "H is NULL");
    return demag_sp_field_energy(p, m, Ms, H, nullptr, stream);
}

int demag_sp_kernel(demag_plan_t p, double* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    HIP_TRY(hipDeviceSynchronize());
    SetupBufs sb;
    int rc = compute_sp_octant(p, nullptr, sb);
    if (rc) return rc;
    const size_t ncell = (size_t)p->n[0] * p->n[1] * p->n[2];
    const double h = std::max(p->d[0], std::max(p->d[1], p->d[2]));
    std::vector<double> tmp(3 * ncell);
    HIP_TRY(hipMemcpy(tmp.data(), sb.Noct, 3 * ncell * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < tmp.size(); ++i) out[i] = tmp[i] * h;
    return DEMAG_OK;
}

int demag_llg_heun(demag_plan_t p, void* m, double Ms, double alpha, double gamma, double hx, double hy, double hz,
                   double dt, int nsteps, void* work, void* stream) {
    const Range range_("demag_llg_heun");
    if (!work) return fail(DEMAG_EINVAL, "NULL work");
    return llg_heun_impl(p, m, Ms, alpha, gamma, hx, hy, hz, dt, nsteps, work, stream);
}

int demag_llg_heun_static(demag_plan_t p, void* m, double Ms, double alpha, double gamma, double hx, double hy,
                          double hz, double dt, int nsteps, void* stream) {
    const Range range_("demag_llg_heun_static");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    const size_t N = (size_t)p->n[0] * p->n[1] * p->n[2];
    const size_t need = 9 * N * (p->dtype == DEMAG_F32 ? sizeof(float) : sizeof(double));
    if (need > kStaticScratchBytes)
        return fail(DEMAG_EINVAL, "workspace of %zu bytes exceeds the static scratch (%zu bytes); use demag_llg_heun",
                    need, kStaticScratchBytes);
    void* work = nullptr;
    const int rc = static_scratch(&work);
    if (rc) return rc;
    return llg_heun_impl(p, m, Ms, alpha, gamma, hx, hy, hz, dt, nsteps, work, stream);
}

int demag_tg_prepare(demag_plan_t p, void* stream) {
    const Range range_("demag_tg_prepare");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    if (p->tg) return DEMAG_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const double step = p->dtype == DEMAG_F32 ? 0.25 : 0.15;
    rc = p->dtype == DEMAG_F32 ? setup_tg<float>(p, st, step) : setup_tg<double>(p, st, step);
    if (rc) {
        free_tg(p->tg);
        p->tg = nullptr;
        return rc;
    }
    return leave(p, st);
}

int demag_tg_field_energy(demag_plan_t p, const void* m, double Ms, void* H, double* E_dev, void* stream) {
    const Range range_("demag_tg_field_energy");
    if (!p || !m || (!H && !E_dev)) return fail(DEMAG_EINVAL, "NULL plan or m, or neither H nor E_dev");
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    if (!p->tg) return fail(DEMAG_ESTATE, "tensor-grid method not prepared (call demag_tg_prepare)");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = p->dtype == DEMAG_F32 ? run_tg_field<float>(p, (const float*)m, Ms, (float*)H, E_dev, st)
                               : run_tg_field<double>(p, (const double*)m, Ms, (double*)H, E_dev, st);
    if (rc) return rc;
    return leave(p, st);
}

int demag_tg_field(demag_plan_t p, const void* m, double Ms, void* H, void* stream) {
    if (!H) return fail(DEMAG_EINVAL, "H is NULL");
    return demag_tg_field_energy(p, m, Ms, H, nullptr, stream);
}

int demag_tg_info(demag_plan_t p, int64_t* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    if (!p->tg) return fail(DEMAG_ESTATE, "tensor-grid method not prepared");
    out[0] = p->tg->R;
    out[1] = (int64_t)p->tg->bytes;
    const double n1 = p->n[0], n2 = p->n[1], n3 = p->n[2];
    out[2] = (int64_t)(3.0 * 2.0 * p->tg->R * n1 * n2 * n3 * (n1 + n2 + n3));  // flops per evaluation
    return DEMAG_OK;
}

int demag_tg_path(demag_plan_t p, int64_t* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    if (!p->tg) return fail(DEMAG_ESTATE, "tensor-grid method not prepared");
    out[0] = p->tg->fused ? 1 : 0;
    out[1] = (int64_t)p->tg->flops_issued;
    return DEMAG_OK;
}

int demag_tg_lowrank_prepare(demag_plan_t p, void* stream) {
    const Range range_("demag_tg_lowrank_prepare");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    if (p->lr) return DEMAG_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const double step = p->dtype == DEMAG_F32 ? 0.25 : 0.15;
    rc = p->dtype == DEMAG_F32 ? setup_lr<float>(p, st, step) : setup_lr<double>(p, st, step);
    if (rc) {
        free_lr(p->lr);
        p->lr = nullptr;
        return rc;
    }
    return leave(p, st);
}

int demag_tg_lowrank_field(demag_plan_t p, int format, int rank, const void* core, const void* U, double Ms, void* FG,
                           void* H, double* E_dev, void* stream) {
    const Range range_("demag_tg_lowrank_field");
    if (!p || !core || !U || !FG) return fail(DEMAG_EINVAL, "NULL plan, core, U or FG");
    if (format != DEMAG_TUCKER && format != DEMAG_CP) return fail(DEMAG_EINVAL, "format must be DEMAG_TUCKER or DEMAG_CP");
    const int rmax = format == DEMAG_TUCKER ? DEMAG_TUCKER_MAX_RANK : DEMAG_CP_MAX_RANK;
    if (rank < 1 || rank > rmax) return fail(DEMAG_EINVAL, "rank %d outside [1, %d]", rank, rmax);
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    if (!p->lr) return fail(DEMAG_ESTATE, "low-rank tensor grid not prepared (call demag_tg_lowrank_prepare)");
    LRState* g = p->lr;
    const size_t tsz = p->dtype == DEMAG_F32 ? 4 : 8;
    size_t w_elems = 0;
    if (H) {  // expansion scratch: the z slices of one GEMM, within the cap
        const size_t per_slice = (size_t)3 * g->R * rank * p->n[1] * tsz;
        const size_t want = std::min<size_t>((size_t)p->n[2] * per_slice, std::max(p->lr_cap, per_slice));
        if (want != g->w_bytes && (want > g->w_bytes || g->w_bytes > std::max(p->lr_cap, per_slice))) {
            HIP_TRY(hipDeviceSynchronize());  // the old scratch may still be in use
            (void)hipFree(g->W);
            g->bytes -= g->w_bytes;
            g->W = nullptr;
            g->w_bytes = 0;
            if (dev_malloc(&g->W, want) != hipSuccess) {
                (void)hipGetLastError();
                g->W = nullptr;
                return fail(DEMAG_ENOMEM, "cannot allocate %zu bytes of low-rank expansion scratch", want);
            }
            g->w_bytes = want;
            g->bytes += want;
        }
        w_elems = g->w_bytes / tsz;
    }
    if (E_dev) {  // Gram matrices of the energy: 27 R r^2 values
        const size_t want = (size_t)27 * g->R * rank * rank * sizeof(double);
        if (want > g->gram_bytes) {
            HIP_TRY(hipDeviceSynchronize());  // the old buffer may still be in use
            (void)hipFree(g->gram);
            g->bytes -= g->gram_bytes;
            g->gram = nullptr;
            g->gram_bytes = 0;
            if (dev_malloc((void**)&g->gram, want) != hipSuccess) {
                (void)hipGetLastError();
                g->gram = nullptr;
                return fail(DEMAG_ENOMEM, "cannot allocate %zu bytes for the low-rank Gram matrices", want);
            }
            g->gram_bytes = want;
            g->bytes += want;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const double hmax = std::max(p->d[0], std::max(p->d[1], p->d[2]));
    const bool tucker = format == DEMAG_TUCKER;
    double* parts = E_dev ? g->partials : nullptr;
    if (p->dtype == DEMAG_F32) {
        const float* DE[3] = {(const float*)g->DE[0], (const float*)g->DE[1], (const float*)g->DE[2]};
        const float* DO[3] = {(const float*)g->DO[0], (const float*)g->DO[1], (const float*)g->DO[2]};
        rc = lr_evaluate<float>(g->handle, st, p->n, p->d, g->R, rank, tucker, (const float*)core, (const float*)U, DE, DO,
                                g->c, Ms * hmax, (float*)FG, parts, g->gram, (float*)H, (float*)g->W, w_elems);
    } else {
        const double* DE[3] = {(const double*)g->DE[0], (const double*)g->DE[1], (const double*)g->DE[2]};
        const double* DO[3] = {(const double*)g->DO[0], (const double*)g->DO[1], (const double*)g->DO[2]};
        rc = lr_evaluate<double>(g->handle, st, p->n, p->d, g->R, rank, tucker, (const double*)core, (const double*)U, DE,
                                 DO, g->c, Ms * hmax, (double*)FG, parts, g->gram, (double*)H, (double*)g->W,
                                 w_elems);
    }
    if (rc) return fail(DEMAG_EHIP, "low-rank tensor-grid evaluation failed (%d)", rc);
    if (E_dev) {
        const double V = p->d[0] * p->d[1] * p->d[2];
        HIP_TRY(launch_energy_reduce(st, g->partials, 9 * g->R, -0.5 * kMu0 * Ms * V, E_dev));
    }
    return leave(p, st);
}

int demag_lowrank_compress(demag_plan_t p, int format, int rank, int sweeps, const void* m, void* core, void* U,
                           double* relerr, void* stream) {
    const Range range_("demag_lowrank_compress");
    if (!p || !m || !core || !U) return fail(DEMAG_EINVAL, "NULL plan, m, core or U");
    if (format != DEMAG_TUCKER && format != DEMAG_CP) return fail(DEMAG_EINVAL, "format must be DEMAG_TUCKER or DEMAG_CP");
    const int rmax = format == DEMAG_TUCKER ? std::min(DEMAG_TUCKER_MAX_RANK, std::min(p->n[0], std::min(p->n[1], p->n[2])))
                                            : DEMAG_CP_MAX_RANK;
    if (rank < 1 || rank > rmax) return fail(DEMAG_EINVAL, "rank %d outside [1, %d]", rank, rmax);
    if (sweeps < 1 || sweeps > 100000) return fail(DEMAG_EINVAL, "sweeps must be in [1, 100000]");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    rc = p->dtype == DEMAG_F32 ? run_compress<float>(p, st, format, rank, sweeps, (const float*)m, (float*)core,
                                                     (float*)U, relerr)
                               : run_compress<double>(p, st, format, rank, sweeps, (const double*)m, (double*)core,
                                                      (double*)U, relerr);
    if (rc) return rc;
    return leave(p, st);
}

int demag_tg_lowrank_info(demag_plan_t p, int64_t* out) {
    if (!p || !out) return fail(DEMAG_EINVAL, "NULL argument");
    if (!p->lr) return fail(DEMAG_ESTATE, "low-rank tensor grid not prepared");
    out[0] = p->lr->R;
    out[1] = (int64_t)p->lr->bytes;
    double hm = std::max(p->d[0], std::max(p->d[1], p->d[2]));
    std::memcpy(&out[2], &hm, sizeof(double));
    return DEMAG_OK;
}

int demag_tg_sinc_nodes(double rmin, double rmax, double step, double* tau, double* w, int cap) {
    std::vector<double> t, ww;
    const int R = tg_sinc_nodes(rmin, rmax, step, t, ww);
    if (R < 0) return fail(DEMAG_EINVAL, "need 0 < rmin <= rmax and step > 0");
    if (tau && w) {
        if (cap < R) return fail(DEMAG_EINVAL, "capacity %d below the %d nodes", cap, R);
        for (int l = 0; l < R; ++l) {
            tau[l] = t[l];
            w[l] = ww[l];
        }
    }
    return R;
}

int demag_plan_describe(demag_plan_t p, char* buf, int len) {
    if (!p || !buf || len < 1) return fail(DEMAG_EINVAL, "NULL argument");
    const char* names[5] = {"x_r2c", "y_fwd", "z_conv", "y_inv", "x_c2r"};
    std::string out;
    for (int w = 0; w < 5; ++w) {
        const LaunchCfg& c = pass_cfg(p->cfg, w);
        char b[160];
        if (c.p2) {
            const int P = p->P[w == 0 || w == 4 ? 0 : w == 2 ? 2 : 1];
            std::string rad;
            if (p2_num_schedules(P) > 1 || (P & (P - 1)) == 0) {
                for (int st = 0; st < p2::schedule_stages(P); ++st)
                    rad += (st ? "." : "") + std::to_string(p2::schedule_radix(P, c.sched, st));
            } else {
                rad = "3x" + std::to_string(P / 3);
            }
            snprintf(b, sizeof b, "%s:pow2(threads=%d,log2 tiles=%d,%d,radix=%s) ", names[w], c.threads, c.t0, c.t1,
                     rad.c_str());
        } else {
            snprintf(b, sizeof b, "%s:generic(threads=%d,E=%d,tiles=%d,%d) ", names[w], c.threads, c.E, c.t0, c.t1);
        }
        out += b;
    }
    if (!out.empty()) out.pop_back();
    snprintf(buf, (size_t)len, "%s", out.c_str());
    return (int)out.size() < len ? DEMAG_OK : fail(DEMAG_EINVAL, "buffer too small (%zu bytes needed)", out.size() + 1);
}

int demag_plan_pass_times(demag_plan_t p, double* ms, int64_t* count) {
    if (!p || !ms || !count) return fail(DEMAG_EINVAL, "NULL argument");
    for (int k = 0; k < kPassMarks - 1; ++k) ms[k] = 0.0;
    const long n = std::min<long>(p->tcount, p->tcap);
    *count = n;
    if (n == 0) return DEMAG_OK;
    HIP_TRY(hipDeviceSynchronize());
    for (long s = 0; s < n; ++s)
        for (int k = 0; k < kPassMarks - 1; ++k) {
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, p->tev[s * kPassMarks + k], p->tev[s * kPassMarks + k + 1]));
            ms[k] += t;
        }
    for (int k = 0; k < kPassMarks - 1; ++k) ms[k] /= (double)n;
    p->tcount = 0;
    return DEMAG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner
namespace {

std::vector<LaunchCfg> candidates_rows(const demag_plan_s* p) {
    std::vector<LaunchCfg> out;
    const size_t cb = csize(p->dtype);
    for (int threads : {128, 256})
        for (int Ty : {2, 4, 8, 16, 32, 64}) {
            if (Ty > p->n[1] + (p->n[1] & 1) && Ty != 2) continue;
            LaunchCfg c;
            c.threads = threads;
            c.t0 = Ty;
            c.E = pick_E((long)(Ty / 2) * p->P[0], threads);
            if (cfg_ok(c, Ty / 2, p->P[0], cb)) out.push_back(c);
        }
    return out;
}

std::vector<LaunchCfg> candidates_pencils(const demag_plan_s* p) {
    std::vector<LaunchCfg> out;
    const size_t cb = csize(p->dtype);
    for (int threads : {128, 256})
        for (int Tz : {1, 2, 4, 8, 16, 32, 64})
            for (int Tx : {1, 2, 4, 8, 16}) {
                if (Tz > p->n[2] && Tz != 1) continue;
                if (Tx > p->Kx && Tx != 1) continue;
                LaunchCfg c;
                c.threads = threads;
                c.t0 = Tx;
                c.t1 = Tz;
                c.E = pick_E((long)Tx * Tz * p->P[1], threads);
                if (cfg_ok(c, (long)Tx * Tz, p->P[1], cb)) out.push_back(c);
            }
    return out;
}

std::vector<LaunchCfg> candidates_z(const demag_plan_s* p) {
    std::vector<LaunchCfg> out;
    const size_t cb = csize(p->dtype);
    for (int threads : {128, 256})
        for (int Tx : {1, 2, 3, 4, 6, 8, 12, 16}) {
            if (Tx > p->Kx && Tx != 1) continue;
            LaunchCfg c;
            c.threads = threads;
            c.t0 = Tx;
            c.E = pick_E(6L * Tx * p->P[2], threads);
            if (cfg_ok(c, 6L * Tx, p->P[2], cb)) out.push_back(c);
        }
    return out;
}

// power-of-two candidates: every tile whose workgroup and LDS fit
void add_p2_candidates(const demag_plan_s* p, int kind, std::vector<LaunchCfg>& out) {
    const int P = p->P[kind == 0 ? 0 : kind == 1 ? 1 : 2];
    if (!p2_supported(P) || (kind == 2 && (!p2_z_supported(P, csize(p->dtype)) || !p2_z_ranges_ok(p)))) return;
    const size_t cb = csize(p->dtype);
    const int TP = p2_threads_per_pencil(P);
    for (int a = 0; a <= 10; ++a)
        for (int b = kind == 2 ? 1 : 0; b <= (kind == 1 ? 10 : kind == 2 ? 2 : 0); ++b) {
            // the fused Z pass pairs each row with its mirror whenever the pair fits a workgroup
            if (kind == 2 && b != (2 * TP <= kP2MaxThreadsZ ? 2 : 1)) continue;
            LaunchCfg c;
            c.p2 = 1;
            if (kind == 0) {
                if (a < 1 || a > pow2_ceil_log(p->n[1]) + 1) continue;
                c.t0 = a;
                c.threads = TP << (a - 1);
            } else if (kind == 1) {
                if (a > pow2_ceil_log(p->Kx) || b > pow2_ceil_log(p->n[2])) continue;
                c.t0 = a;
                c.t1 = b;
                c.threads = TP << (a + b);
            } else {
                if (a > pow2_ceil_log(p->P[1] / 2 + 1)) continue;
                c.t0 = a;  // log2 of the consecutive ky' rows of a tile
                c.t1 = b;  // 2: each row with its mirror, 1: single rows
                c.threads = b * TP << a;
            }
            if (c.threads < 64 && c.threads < TP * 2) continue;
            for (int sc = 0; sc < p2_num_schedules(P); ++sc) {  // every radix schedule of the length
                c.sched = sc;
                if (p2_cfg_ok(c, P, cb, kind)) out.push_back(c);
            }
        }
}

std::string cfg_str(const LaunchCfg& c) {
    char b[64];
    snprintf(b, sizeof b, "%d,%d,%d,%d,%d,%d", c.threads, c.E, c.t0, c.t1, c.p2, c.sched);
    return b;
}

bool cfg_parse(const std::string& s, LaunchCfg& c) {
    return sscanf(s.c_str(), "%d,%d,%d,%d,%d,%d", &c.threads, &c.E, &c.t0, &c.t1, &c.p2, &c.sched) == 6;
}

std::string cache_key(const demag_plan_s* p) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    char b[160];
    snprintf(b, sizeof b, "v5|%s|%s|%d,%d,%d", arch.c_str(), p->dtype == DEMAG_F32 ? "f32" : "f64", p->n[0],
             p->n[1], p->n[2]);
    return b;
}

// Cache file: one line per plan key, "key xf yf zc yi xi" (each
// threads,E,t0,t1,p2,sched).
std::map<std::string, std::string> read_cache(const char* path) {
    std::map<std::string, std::string> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        auto sp = line.find(' ');
        if (sp == std::string::npos || line.rfind("v5|", 0) != 0) continue;
        m[line.substr(0, sp)] = line.substr(sp + 1);
    }
    return m;
}

bool parse_cfgs(const std::string& s, PassCfgs& c) {
    std::istringstream is(s);
    std::string a[5];
    for (auto& x : a)
        if (!(is >> x)) return false;
    return cfg_parse(a[0], c.xf) && cfg_parse(a[1], c.yf) && cfg_parse(a[2], c.zc) && cfg_parse(a[3], c.yi) &&
           cfg_parse(a[4], c.xi);
}

// Time of a whole evaluation with candidate `lc` in pass `which` and the
// plan's current shapes elsewhere.  A pass timed alone in a loop finds its
// working set (up to a few hundred MB) still in the last-level cache, which
// the other passes of an evaluation evict; inside the whole sequence each pass
// meets the cache state it has in use, and the effect of its shape on the
// passes around it is counted too.
template <typename T>
int time_pass(demag_plan_s* p, int which, const LaunchCfg& lc, hipStream_t st, const T* m, T* H, float* ms_out) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    PassCfgs c = p->cfg;
    LaunchCfg* slot[5] = {&c.xf, &c.yf, &c.zc, &c.yi, &c.xi};
    *slot[which] = lc;
    auto launch = [&]() {
        for (int w = 0; w < 5; ++w)
            if (hipError_t e = launch_pass<T>(p, w, pass_cfg(c, w), st, m, 1.0, H, nullptr, nullptr, 0)) return e;
        return hipSuccess;
    };
    hipError_t err = hipSuccess;
    for (int r = 0; r < 3 && err == hipSuccess; ++r) err = launch();
    const int reps = 10;
    float best = 1e30f;
    for (int trial = 0; trial < 3 && err == hipSuccess; ++trial) {
        err = hipEventRecord(e0, st);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, ms / reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "autotune timing");
    *ms_out = best;
    return DEMAG_OK;
}

template <typename T>
int autotune_impl(demag_plan_s* p, hipStream_t st) {
    const size_t nvec = 3ull * p->n[0] * p->n[1] * p->n[2];
    T *m = nullptr, *H = nullptr;
    auto release = [&]() {
        (void)hipFree(m);
        (void)hipFree(H);
    };
    if (dev_malloc(&m, nvec * sizeof(T)) != hipSuccess || dev_malloc(&H, nvec * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(DEMAG_ENOMEM, "autotune: cannot allocate %zu bytes of input and output", 2 * nvec * sizeof(T));
    }
    if (hipError_t e = hipMemsetAsync(m, 0, nvec * sizeof(T), st)) {
        release();
        return hip_fail(e, "hipMemsetAsync");
    }
    int rc = DEMAG_OK;
    std::vector<LaunchCfg> cand[5] = {candidates_rows(p), candidates_pencils(p), candidates_z(p),
                                      candidates_pencils(p), candidates_rows(p)};
    const int kinds[5] = {0, 1, 2, 1, 0};
    for (int w = 0; w < 5; ++w) add_p2_candidates(p, kinds[w], cand[w]);
    LaunchCfg* slot[5] = {&p->cfg.xf, &p->cfg.yf, &p->cfg.zc, &p->cfg.yi, &p->cfg.xi};
    for (int which = 0; which < 5 && !rc; ++which) {
        float best = 1e30f;
        LaunchCfg bestc = *slot[which];
        for (const auto& lc : cand[which]) {
            float ms = 0;
            rc = time_pass<T>(p, which, lc, st, m, H, &ms);
            if (rc) break;
            if (ms < best) {
                best = ms;
                bestc = lc;
            }
        }
        *slot[which] = bestc;
    }
    (void)hipStreamSynchronize(st);  // the timed launches have finished with m and H
    release();
    return rc;
}

}  // namespace

extern "C" int demag_autotune(demag_plan_t p, void* stream) {
    const Range range_("demag_autotune");
    if (!p) return fail(DEMAG_EINVAL, "NULL plan");
    hipStream_t st = (hipStream_t)stream;
    int rc = enter(p, st);
    if (rc) return rc;
    const char* path = getenv("DEMAG_AUTOTUNE_CACHE");
    const std::string key = cache_key(p);
    if (path) {
        auto cache = read_cache(path);
        auto it = cache.find(key);
        PassCfgs c;
        if (it != cache.end() && parse_cfgs(it->second, c) && plan_cfgs_ok(p, c)) {
            p->cfg = c;  // a valid cached entry; a corrupt one falls through to tuning
            return DEMAG_OK;
        }
    }
    const PassCfgs before = p->cfg;  // shapes the plan has verified (defaults, generic_kernels, a cache)
    rc = p->dtype == DEMAG_F32 ? autotune_impl<float>(p, st) : autotune_impl<double>(p, st);
    if (rc) {
        p->cfg = before;
        (void)leave(p, st);  // the busy marker covers what was enqueued before the failure
        return rc;
    }
    if (path) {
        auto cache = read_cache(path);
        cache[key] = cfg_str(p->cfg.xf) + " " + cfg_str(p->cfg.yf) + " " + cfg_str(p->cfg.zc) + " " +
                     cfg_str(p->cfg.yi) + " " + cfg_str(p->cfg.xi);
        std::string tmp = std::string(path) + ".tmp";
        std::ofstream f(tmp);
        for (auto& kv : cache) f << kv.first << " " << kv.second << "\n";
        f.close();
        if (f) std::rename(tmp.c_str(), path);
    }
    return leave(p, st);
}

// ---------------------------------------------------------------------------
// batch: the plans are grouped by geometry; each group runs each pass as one
// launch over all its members (pointer lists), and the five launches of every
// group are recorded once into a HIP graph, groups on forked capture streams
// so that they overlap.  One replay of the graph evaluates the whole batch.
namespace {
constexpr int kBranches = 8;

// Hardware queues the runtime gives a process (HIP's GPU_MAX_HW_QUEUES,
// default 4): capture streams beyond this share a queue, and the groups on a
// shared queue run one after the other.
int hw_queues() {
    const char* e = std::getenv("GPU_MAX_HW_QUEUES");
    int q = e ? std::atoi(e) : 4;
    return std::max(1, std::min(q, kBranches));
}

bool same_geometry(const demag_plan_s* a, const demag_plan_s* b) {
    return a->dtype == b->dtype && a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2] &&
           a->d[0] == b->d[0] && a->d[1] == b->d[1] && a->d[2] == b->d[2] && a->bands.far_cut == b->bands.far_cut &&
           a->bands.fg_cut == b->bands.fg_cut;
}

// per-pass pointer lists of a group: m -> B1 -> B2 -> B2 -> B1 -> H
void group_io(const BatchGroup& grp, BatchIO io[5]) {
    const int n = grp.count;
    void** L = grp.lists;  // device array: [0,n) m, [n,2n) H, [2n,3n) B1, [3n,4n) B2
    io[0].in = (const void* const*)(L);
    io[0].out = L + 2 * n;
    io[1].in = (const void* const*)(L + 2 * n);
    io[1].out = L + 3 * n;
    io[2].in = (const void* const*)(L + 3 * n);
    io[2].out = L + 3 * n;
    io[3].in = (const void* const*)(L + 3 * n);
    io[3].out = L + 2 * n;
    io[4].in = (const void* const*)(L + 2 * n);
    io[4].out = L + n;
    for (int w = 0; w < 5; ++w) io[w].count = n;
}

template <typename T>
int enqueue_group(const BatchGroup& grp, double Ms, hipStream_t st) {
    BatchIO io[5];
    group_io(grp, io);
    for (int w = 0; w < 5; ++w)
        HIP_TRY(launch_pass<T>(grp.lead, w, pass_cfg(grp.cfg, w), st, nullptr, Ms, nullptr, nullptr, nullptr, 0, io[w]));
    return DEMAG_OK;
}

// Record every group's launches into the batch's graph (replacing an earlier
// one): the groups are spread over `lanes` forked capture streams, joined at
// the end, longest first onto the least loaded lane (by group cost), each
// lane running its groups longest first.
int record_graph(demag_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    int rc = DEMAG_OK;
    const int ng = (int)b->groups.size();
    const int nb = std::min(b->lanes > 0 ? std::min(b->lanes, kBranches) : hw_queues(), ng);
    b->used_lanes = nb;
    std::vector<int> order(ng), lane_of(ng);
    for (int i = 0; i < ng; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->groups[a].cost > b->groups[c].cost; });
    {
        std::vector<double> load(nb, 0.0);
        for (int gi : order) {
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            lane_of[gi] = l;
            load[l] += b->groups[gi].cost;
        }
    }
    hipStream_t cs[kBranches] = {};
    hipEvent_t ev[kBranches + 1] = {};
    for (int k = 0; k < nb && !rc; ++k)
        if (hipStreamCreateWithFlags(&cs[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess)
            rc = fail(DEMAG_EHIP, "cannot create capture streams");
    if (!rc && hipEventCreateWithFlags(&ev[kBranches], hipEventDisableTiming) != hipSuccess)
        rc = fail(DEMAG_EHIP, "cannot create capture event");
    bool capturing = false;
    if (!rc) {
        if (hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = fail(DEMAG_EHIP, "hipStreamBeginCapture failed");
        else
            capturing = true;
    }
    // the fork and join of the capture streams: a failed record or wait would
    // leave a dependency out of the graph, so each is checked
    auto chk = [&](hipError_t e, const char* what) {
        if (!rc && e != hipSuccess) rc = hip_fail(e, what);
    };
    if (!rc) {
        chk(hipEventRecord(ev[kBranches], cs[0]), "hipEventRecord (capture fork)");
        for (int k = 1; k < nb; ++k)
            chk(hipStreamWaitEvent(cs[k], ev[kBranches], 0), "hipStreamWaitEvent (capture fork)");
        for (int k = 0; k < ng && !rc; ++k) {
            const BatchGroup& g = b->groups[order[k]];
            hipStream_t lst = cs[lane_of[order[k]]];
            rc = g.lead->dtype == DEMAG_F32 ? enqueue_group<float>(g, b->Ms, lst) : enqueue_group<double>(g, b->Ms, lst);
        }
        for (int k = 1; k < nb; ++k) {
            chk(hipEventRecord(ev[k], cs[k]), "hipEventRecord (capture join)");
            chk(hipStreamWaitEvent(cs[0], ev[k], 0), "hipStreamWaitEvent (capture join)");
        }
    }
    if (capturing) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs[0], &g);
        if (!rc && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        if (!rc && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess)
            rc = fail(DEMAG_EHIP, "hipGraphInstantiate failed");
    }
    for (int k = 0; k < nb; ++k) {
        if (cs[k]) (void)hipStreamDestroy(cs[k]);
        if (ev[k]) (void)hipEventDestroy(ev[k]);
    }
    if (ev[kBranches]) (void)hipEventDestroy(ev[kBranches]);
    return rc;
}

// Time candidate launch shapes of each pass of one group on the group's own
// buffers (one launch covers all members) and keep the fastest.
template <typename T>
int tune_group(BatchGroup& g, hipStream_t st) {
    demag_plan_s* p = g.lead;
    BatchIO io[5];
    group_io(g, io);
    std::vector<LaunchCfg> cand[5] = {candidates_rows(p), candidates_pencils(p), candidates_z(p),
                                      candidates_pencils(p), candidates_rows(p)};
    const int kinds[5] = {0, 1, 2, 1, 0};
    for (int w = 0; w < 5; ++w) add_p2_candidates(p, kinds[w], cand[w]);
    LaunchCfg* slot[5] = {&g.cfg.xf, &g.cfg.yf, &g.cfg.zc, &g.cfg.yi, &g.cfg.xi};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    hipError_t err = hipSuccess;
    for (int w = 0; w < 5 && err == hipSuccess; ++w) {
        float best = 1e30f;
        LaunchCfg bestc = *slot[w];
        for (const auto& lc : cand[w]) {
            // the group's whole evaluation with the candidate in pass w (as the
            // plan autotuner: the cache state of the real sequence)
            auto launch = [&]() {
                for (int ww = 0; ww < 5; ++ww) {
                    const LaunchCfg& c = ww == w ? lc : *slot[ww];
                    if (hipError_t e = launch_pass<T>(p, ww, c, st, nullptr, 1.0, nullptr, nullptr, nullptr, 0, io[ww]))
                        return e;
                }
                return hipSuccess;
            };
            for (int r = 0; r < 2 && err == hipSuccess; ++r) err = launch();
            float t_best = 1e30f;
            for (int trial = 0; trial < 3 && err == hipSuccess; ++trial) {
                err = hipEventRecord(e0, st);
                for (int r = 0; r < 5 && err == hipSuccess; ++r) err = launch();
                if (err == hipSuccess) err = hipEventRecord(e1, st);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                float ms = 0;
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                t_best = std::min(t_best, ms);
            }
            if (err != hipSuccess) break;
            if (t_best < best) {
                best = t_best;
                bestc = lc;
            }
        }
        *slot[w] = bestc;
        g.cost = best;  // after the last pass: the group's evaluation with every chosen shape
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "batch autotune timing");
    return DEMAG_OK;
}

// Average time of one replay of the batch's graph (after warm-up replays).
int time_replays(demag_batch_s* b, hipStream_t st, float* us) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(DEMAG_EHIP, "hipEventCreate failed");
    }
    hipError_t err = hipSuccess;
    for (int r = 0; r < 4 && err == hipSuccess; ++r) err = hipGraphLaunch(b->exec, st);
    float best = 1e30f;  // best of 5 regions of 16 replays (replay times vary by several percent)
    for (int trial = 0; trial < 5 && err == hipSuccess; ++trial) {
        err = hipEventRecord(e0, st);
        for (int r = 0; r < 16 && err == hipSuccess; ++r) err = hipGraphLaunch(b->exec, st);
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        best = std::min(best, 1e3f * ms / 16);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "batch replay timing");
    *us = best;
    return DEMAG_OK;
}
}  // namespace

extern "C" int demag_batch_create(demag_batch_t* out, const demag_plan_t* plans, int count, const void* const* m,
                                  void* const* H, double Ms, void* stream) {
    const Range range_("demag_batch_create");
    if (!out || !plans || !m || !H || count < 1) return fail(DEMAG_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (!std::isfinite(Ms)) return fail(DEMAG_EINVAL, "Ms must be finite");
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !m[i] || !H[i]) return fail(DEMAG_EINVAL, "NULL plan or buffer at batch index %d", i);
        if (plans[i]->dtype != plans[0]->dtype) return fail(DEMAG_EINVAL, "mixed precisions in one batch");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(DEMAG_EINVAL, "plan repeated at batch indices %d and %d", j, i);
    }
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    auto* b = new demag_batch_s();
    b->plans.assign(plans, plans + count);
    // group by geometry, members in batch order
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
        size_t gi = 0;
        while (gi < members.size() && !same_geometry(plans[members[gi][0]], plans[i])) ++gi;
        if (gi == members.size()) members.emplace_back();
        members[gi].push_back(i);
    }
    std::vector<void*> host_lists;
    for (auto& mem : members) {
        const int n = (int)mem.size();
        for (int k = 0; k < n; ++k) host_lists.push_back(const_cast<void*>(m[mem[k]]));
        for (int k = 0; k < n; ++k) host_lists.push_back(H[mem[k]]);
        for (int k = 0; k < n; ++k) host_lists.push_back(plans[mem[k]]->B1);
        for (int k = 0; k < n; ++k) host_lists.push_back(plans[mem[k]]->B2);
    }
    int rc = DEMAG_OK;
    if (dev_malloc(&b->dev_lists, host_lists.size() * sizeof(void*)) != hipSuccess) {
        (void)hipGetLastError();
        b->dev_lists = nullptr;
        rc = fail(DEMAG_ENOMEM, "cannot allocate batch pointer lists");
    } else if (hipMemcpy(b->dev_lists, host_lists.data(), host_lists.size() * sizeof(void*), hipMemcpyHostToDevice) !=
               hipSuccess) {
        rc = fail(DEMAG_EHIP, "cannot upload batch pointer lists");
    }
    size_t off = 0;
    for (auto& mem : members) {
        BatchGroup g;
        g.lead = plans[mem[0]];
        g.count = (int)mem.size();
        g.lists = (void**)b->dev_lists + off;
        g.cfg = g.lead->cfg;
        g.cost = (double)g.count * g.lead->P[0] * g.lead->P[1] * g.lead->P[2];
        off += 4 * (size_t)g.count;
        b->groups.push_back(g);
    }
    b->Ms = Ms;
    if (!rc && hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        b->done = nullptr;
        rc = fail(DEMAG_EHIP, "hipEventCreate failed");
    }
    if (!rc) rc = record_graph(b);
    if (rc) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        if (b->done) (void)hipEventDestroy(b->done);
        (void)hipFree(b->dev_lists);
        delete b;
        return rc;
    }
    *out = b;
    return DEMAG_OK;
}

extern "C" int demag_batch_autotune(demag_batch_t b, void* stream) {
    const Range range_("demag_batch_autotune");
    if (!b || !b->exec) return fail(DEMAG_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    for (auto p : b->plans) {
        int rc = enter(p, st);
        if (rc) return rc;
    }
    int rc = DEMAG_OK;
    for (auto& g : b->groups) {
        rc = g.lead->dtype == DEMAG_F32 ? tune_group<float>(g, st) : tune_group<double>(g, st);
        if (rc) break;
    }
    // then the number of lanes, up to one per hardware queue, by whole replays
    const int maxl = std::min(hw_queues(), (int)b->groups.size());
    int best_l = maxl;
    float best_us = 1e30f;
    for (int l = 1; l <= maxl && !rc; ++l) {
        b->lanes = l;
        rc = record_graph(b);
        float us = 0;
        if (!rc) rc = time_replays(b, st, &us);
        if (!rc && us < best_us) {
            best_us = us;
            best_l = l;
        }
    }
    b->lanes = best_l;
    {  // re-record in every case: a failed timing may have left no graph
        const int r2 = record_graph(b);
        if (!rc) rc = r2;
    }
    for (auto p : b->plans) {
        int r2 = leave(p, st);
        if (!rc) rc = r2;
    }
    return rc;
}

// One event for the whole replay (not one per member: the host cost of the
// per-member bookkeeping would exceed the replay itself for small grids).
extern "C" int demag_batch_launch(demag_batch_t b, void* stream) {
    const Range range_("demag_batch_launch");
    if (!b || !b->exec) return fail(DEMAG_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    for (auto p : b->plans) {
        int rc = enter(p, st);
        if (rc) return rc;
    }
    HIP_TRY(hipGraphLaunch(b->exec, st));
    HIP_TRY(hipEventRecord(b->done, st));
    for (auto p : b->plans) {
        p->busy = b->done;
        p->last_stream = st;
        p->used = true;
    }
    return DEMAG_OK;
}

extern "C" int demag_batch_info(demag_batch_t b, int64_t* out) {
    if (!b || !out) return fail(DEMAG_EINVAL, "NULL argument");
    out[0] = (int64_t)b->plans.size();
    out[1] = (int64_t)b->groups.size();
    out[2] = b->used_lanes;
    return DEMAG_OK;
}

int demag_batch_destroy(demag_batch_t b) {
    if (!b) return fail(DEMAG_EINVAL, "NULL batch");
    (void)hipDeviceSynchronize();
    for (auto p : b->plans)  // the replays are complete: drop the reference to the batch's event
        if (p->busy == b->done) p->busy = nullptr;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->done) (void)hipEventDestroy(b->done);
    (void)hipFree(b->dev_lists);
    delete b;
    return DEMAG_OK;
}
