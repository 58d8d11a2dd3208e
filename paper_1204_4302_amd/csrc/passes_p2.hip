// The five passes of one field evaluation for power-of-two padded lengths
// (compile-time P), on the register-resident FFT of fft_reg.hpp.  Same data
// layouts and arithmetic as the generic passes (passes.hip):
//   m [C][nz][ny][nx] -> B1 [C][nz][Kx][ny] -> B2 [C][Kx][Py][nz] -> (x Nhat)
//   -> B2 -> B1 -> H [C][nz][ny][nx].
// The side of a pass whose pencils are contiguous in memory moves directly
// between HBM and registers (input positions of the first stage, output
// positions of the last); the transposed side goes through the padded LDS
// slabs.  Tile extents are powers of two, passed as log2.
#include <algorithm>
#include <vector>

#include "fft_reg.hpp"
#include "internal.hpp"

namespace demag {
namespace {

template <typename T>
__device__ __forceinline__ cx<T>* lds_base() {
    extern __shared__ __align__(16) unsigned char smem_p2[];
    return reinterpret_cast<cx<T>*>(smem_p2);
}

template <typename T>
__device__ __forceinline__ cx<T> czero() { return mk(T(0), T(0)); }

// Several grids per launch (BatchIO): the tiles of grid g are the logical
// tiles [g T, (g+1) T), T = gridDim.x / count.  Returns the tile within the
// grid and sets g.
__device__ __forceinline__ int batch_tile(int L, const BatchIO& bio, int* g) {
    *g = 0;
    if (!bio.in) return L;
    const int tiles = gridDim.x / bio.count;
    *g = L / tiles;
    return L - *g * tiles;
}

// Logical tile index of this workgroup.  The hardware hands consecutive
// workgroups of a 1-D grid to the XCDs in turn (workgroup b to XCD b mod
// nxcd); renumbering so that XCD x runs one contiguous range of logical tiles
// keeps neighbouring tiles -- which share 128-byte lines of the strided side
// of a pass -- in the same L2.  A bijection on [0, gridDim.x).
__device__ __forceinline__ int xcd_tile(int nxcd) {
    const int b = blockIdx.x, nb = gridDim.x;
    if (nxcd <= 1 || nb < nxcd) return b;
    const int x = b % nxcd, q = b / nxcd;
    const int per = nb / nxcd, rem = nb % nxcd;
    return x * per + min(x, rem) + q;
}

// Twiddle source of a p2 kernel.  A table of at most kP2TwLdsMax bytes is
// copied once per workgroup into LDS after the pencils' slabs, so that each
// thread's twiddle loads are LDS reads instead of vector-memory instructions
// (one per thread for the copy instead of one per twiddle); the caller's next
// workgroup barrier publishes it.  Larger tables are read from global memory.
template <typename T, int P>
__host__ __device__ constexpr bool tw_in_lds() {
    return p2::Len<P>::table_size() * sizeof(cx<T>) <= kP2TwLdsMax;
}
template <typename T, int P>
__device__ __forceinline__ const cx<T>* twiddle_source(cx<T>* lds, int npencils, const cx<T>* __restrict__ twt,
                                                       int tid, int nthr) {
    if constexpr (tw_in_lds<T, P>()) {
        constexpr int TS = p2::Len<P>::table_size();
        cx<T>* dst = lds + npencils * p2::Len<P>::PS;
        for (int i = tid; i < TS; i += nthr) dst[i] = twt[i];
        return dst;
    } else {
        return twt;
    }
}

// One transform of a pencil (length traits LT: length and radix schedule)
// with this thread's twiddles loaded from `src` (thread-major table, in LDS or
// global memory).
template <typename LT, int DIR, bool LO = false, typename T>
__device__ __forceinline__ void run_fft(cx<T>* v, cx<T>* slab, int t, const cx<T>* __restrict__ src) {
    LT::template fft_src<DIR, LO>(v, slab, t, src);
}

// Workgroup size bound of the X and Y kernels: 1024 threads for power-of-two
// lengths; 512 for 3 * 2^a, whose threads hold three times the slots (up to
// 256 registers then).
template <int P>
constexpr int xy_max_threads() { return p2::is_pow2(P) ? 1024 : 512; }

// Global-memory views of pointers (per-grid pointers of a batch are read from
// memory, where the compiler could not tell their address space).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T* p) { return (gptr<T>)p; }

// complex element access through global pointers as one 2-wide vector
template <typename T>
struct vec2 {
    typedef T type __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ cx<T> gld(gptr<const cx<T>> p, size_t i) {
    const typename vec2<T>::type v = ((gptr<const typename vec2<T>::type>)p)[i];
    return mk(v.x, v.y);
}
// Load p[i] if `valid`, else zero, without a branch: the load always goes to
// p[valid ? i : 0] (callers guarantee p[0] is in bounds) and the value is
// selected afterwards, so no exec-masked block forces an early wait.
template <typename T>
__device__ __forceinline__ cx<T> gld_if(gptr<const cx<T>> p, size_t i, bool valid) {
    const cx<T> v = gld(p, valid ? i : 0);
    return valid ? v : czero<T>();
}
// The same for a spectrum that its last reader takes: loaded non-temporally.
template <typename T>
__device__ __forceinline__ cx<T> gld_last_if(gptr<const cx<T>> p, size_t i, bool valid) {
    const typename vec2<T>::type v =
        __builtin_nontemporal_load(&((gptr<const typename vec2<T>::type>)p)[valid ? i : 0]);
    return valid ? mk(v.x, v.y) : czero<T>();
}
// (real values: the magnetization, read once per evaluation, is loaded
// non-temporally, so that it does not displace the spectrum in the caches)
template <typename T>
__device__ __forceinline__ T gldr_if(gptr<const T> p, size_t i, bool valid) {
    const T v = __builtin_nontemporal_load(&p[valid ? i : 0]);
    return valid ? v : T(0);
}

template <typename T>
__device__ __forceinline__ void gst(gptr<cx<T>> p, size_t i, cx<T> c) {
    typename vec2<T>::type v;
    v.x = c.re;
    v.y = c.im;
    ((gptr<typename vec2<T>::type>)p)[i] = v;
}

// 16-byte vectors of reals: VR = 4 floats or 2 doubles.
template <typename T>
__host__ __device__ constexpr int vr() { return 16 / (int)sizeof(T); }
template <typename T>
struct vecN {
    typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};
// X-C2R moves rows as 16-byte vectors when each thread's contiguous share of
// the kept half (EPT/2 positions) is a whole number of them.
template <typename T, int P>
__host__ __device__ constexpr bool vec_rows() {
    return p2::Len<P>::EPT >= 8 && (p2::Len<P>::EPT / 2) % vr<T>() == 0;
}
// Row vector at real index x (a multiple of VR; rows start 16-byte aligned),
// zero if not valid (the load then goes to p[0]); non-temporal: the
// magnetization is read once per evaluation.
template <typename T>
__device__ __forceinline__ typename vecN<T>::type gldv_nt_if(gptr<const T> p, int x, bool valid) {
    using V = typename vecN<T>::type;
    const V v = __builtin_nontemporal_load((gptr<const V>)(p + (valid ? x : 0)));
    return valid ? v : V{};
}
// Two adjacent complex values c0, c1 at p[i], p[i + 1] (i even; FP32: one
// 16-byte store).
template <typename T>
__device__ __forceinline__ void gst2(gptr<cx<T>> p, size_t i, cx<T> c0, cx<T> c1) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 v;
        v.x = c0.re;
        v.y = c0.im;
        v.z = c1.re;
        v.w = c1.im;
        *(gptr<f4>)(p + i) = v;
    } else {
        gst(p, i, c0);
        gst(p, i + 1, c1);
    }
}
// ... and the matching load (FP32: one 16-byte load); zero if not valid.
template <typename T>
__device__ __forceinline__ void gld2_if(gptr<const cx<T>> p, size_t i, bool valid, cx<T>& c0, cx<T>& c1) {
    if constexpr (sizeof(T) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 v = *(gptr<const f4>)(p + (valid ? i : 0));
        c0 = valid ? mk(v.x, v.y) : czero<T>();
        c1 = valid ? mk(v.z, v.w) : czero<T>();
    } else {
        c0 = gld_if(p, i, valid);
        c1 = gld_if(p, i + 1, valid);
    }
}
// Order a pencil's slab accesses among its own threads (see p2::pencil_sync).
template <int P>
__device__ __forceinline__ void pencil_sync_p() { p2::pencil_sync<p2::Len<P>::TP>(); }

// Raw buffer access: a resource (base address and byte range, uniform across
// the wavefront, so held in scalar registers) plus a 32-bit per-lane byte
// offset, with compile-time parts folded into the instruction's immediate.
// The hardware range-checks every access: a load at or beyond the range
// returns zero and a store there is dropped, so lanes outside the data (zero
// padding, ragged tiles) take the offset kOob instead of a branch.  Ranges are
// below kOob (the host keeps such shapes on the generic kernels), and kOob plus
// any immediate stays below 2^32.
constexpr unsigned kOob = 0xFFFFF000u;
constexpr unsigned kBufWord3 = 0x00020000u;  // 32-bit data format, as raw buffers on this family expect

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ Buf make_buf(const void* base, size_t bytes) {
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(unsigned)bytes, (int)kBufWord3)};
}

template <typename T, int POL = 0>  // POL: cache policy bits of the load
__device__ __forceinline__ cx<T> bld(Buf b, unsigned off, unsigned soff = 0) {
    if constexpr (sizeof(T) == 4) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(b.r, off, soff, POL);
        const typename vec2<T>::type v = __builtin_bit_cast(typename vec2<T>::type, u);
        return mk(v.x, v.y);
    } else {
        const auto u = __builtin_amdgcn_raw_buffer_load_b128(b.r, off, soff, POL);
        const typename vec2<T>::type v = __builtin_bit_cast(typename vec2<T>::type, u);
        return mk(v.x, v.y);
    }
}
// Cache policy of the staged (16-byte) loads of the tensor and kernel
// spectra of a single evaluation: non-temporal (read once per evaluation,
// they would otherwise displace the spectrum that the next pass reads from
// the 256 MB memory-side cache; the fused Z pass's TNT instances).  The
// members of a batch group share one tensor spectrum, which they re-read from
// the caches: there the loads are plain, and so are the per-frequency loads
// of the unstaged forms (split form, 3 * 2^a).
constexpr int kNt = 2;

template <typename T>
__device__ __forceinline__ T bldr(Buf b, unsigned off, unsigned soff = 0) {  // (kernel spectrum: streamed)
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(b.r, off, soff, kNt));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(b.r, off, soff, kNt));
    }
}
template <typename T>
__device__ __forceinline__ void bst(Buf b, unsigned off, cx<T> c) {
    typename vec2<T>::type v;
    v.x = c.re;
    v.y = c.im;
    if constexpr (sizeof(T) == 4) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), b.r, off, 0, 0);
    } else {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), b.r, off, 0, 0);
    }
}
// The six tensor components of one frequency (stored side by side): FP32 as
// three 2-dword loads, FP64 as three 4-dword loads (natural alignment: the
// frequency stride is 24 resp. 48 bytes).
template <typename T>
__device__ __forceinline__ void bld6(Buf b, unsigned off, T* o) {
    if constexpr (sizeof(T) == 4) {
        typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const f2 v = __builtin_bit_cast(f2, __builtin_amdgcn_raw_buffer_load_b64(b.r, off + 8 * i, 0, 0));
            o[2 * i] = (T)v.x;
            o[2 * i + 1] = (T)v.y;
        }
    } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const d2 v = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(b.r, off + 16 * i, 0, 0));
            o[2 * i] = (T)v.x;
            o[2 * i + 1] = (T)v.y;
        }
    }
}
// byte offset `base + d` of a lane's element, or an out-of-range offset when
// the element is not valid (d is a compile-time constant after unrolling)
__device__ __forceinline__ unsigned boff(bool valid, unsigned base, unsigned d) {
    return (valid ? base : kOob - d) + d;
}

// ---------------------------------------------------------------------------
// X forward (R2C of two rows per complex pencil).  1-D grid of
// ceil(ny/Ty) * nz * C (* batch) tiles, block (Ty/2) * TP threads.
// Output: thread (pair q, frequency k) forms X_even[k] and X_odd[k] of rows
// 2q and 2q+1 from one pair of slab reads and, when ny is even (rows 2q and
// 2q+1 then lie side by side in B1 and are both inside the tile or both
// outside), writes them with one 16-byte store (FP32).  (Loading the rows as
// 16-byte vectors staged through the slab measured slower than the direct
// first-stage loads.)
template <typename T, int P, int S>
__global__ void __launch_bounds__(xy_max_threads<P>()) kx_fwd(const T* __restrict__ in, cx<T>* __restrict__ out, int nx, int ny,
                                               int nz, int lgTy, int nxcd, const cx<T>* __restrict__ twt,
                                               BatchIO bio) {
    using LT = p2::Len<P, S>;
    constexpr int Kx = P / 2 + 1;
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int p = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Ty = 1 << lgTy;
    const int nyt = (ny + Ty - 1) >> lgTy;
    int g;
    const int L = batch_tile(xcd_tile(nxcd), bio, &g), yt = L % nyt, zc = L / nyt;
    if (bio.in) {
        in = (const T*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int y0 = yt << lgTy, z = zc % nz, c = zc / nz;
    const int ty = min(Ty, ny - y0);
    const bool ok0 = 2 * p < ty, ok1 = 2 * p + 1 < ty;
    const T* rb = in + (((size_t)c * nz + z) * ny + y0) * (size_t)nx;
    const gptr<const T> row0 = gmem(ok0 ? rb + (size_t)(2 * p) * nx : in);
    const gptr<const T> row1 = gmem(ok1 ? rb + (size_t)(2 * p + 1) * nx : in);
    cx<T> v[LT::EPT];
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) {
        const int k = LT::fin_k(j);
        const int x = t + k * LT::TP;
        if (k < LT::EPT / 2) {  // the padded half is never read
            v[j] = mk(gldr_if(row0, x, ok0 && x < nx), gldr_if(row1, x, ok1 && x < nx));
        } else {
            v[j] = czero<T>();
        }
    }
    cx<T>* slab = lds + p * LT::PS;
    const cx<T>* tws = twiddle_source<T, P>(lds, nthr >> LT::LOG_TP, twt, tid, nthr);
    if constexpr (tw_in_lds<T, P>()) __syncthreads();
    run_fft<LT, -1, true>(v, slab, t, tws);
    __syncthreads();
    const int pt = LT::pad(t);
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) slab[LT::fout_slab(pt, t, j)] = v[j];
    __syncthreads();
    // spectra of the two rows: X_even = (Z_k + conj Z_{P-k})/2, X_odd = (Z_k - conj Z_{P-k})/(2i),
    // written y-contiguous; thread (q, k0 + i TP), q = tid mod (Ty/2)
    constexpr int KI = (Kx + LT::TP - 1) / LT::TP;
    const int lgB = lgTy - 1;
    const int q = tid & ((1 << lgB) - 1), k0 = tid >> lgB;
    const bool okq0 = 2 * q < ty, okq1 = 2 * q + 1 < ty;
    if (okq0) {
        const cx<T>* pen = lds + q * LT::PS;
        cx<T> xe[KI], xo[KI];
#pragma unroll
        for (int i = 0; i < KI; ++i) {
            const int k = k0 + i * LT::TP;
            if (i + 1 < KI || k < Kx) {
                const cx<T> a = pen[LT::pad(k)], b = pen[LT::pad(k == 0 ? 0 : P - k)];
                xe[i] = mk(T(0.5) * (a.re + b.re), T(0.5) * (a.im - b.im));
                xo[i] = mk(T(0.5) * (a.im + b.im), T(0.5) * (b.re - a.re));
            }
        }
        const gptr<cx<T>> dst = gmem(out + ((size_t)c * nz + z) * (size_t)Kx * ny + y0 + 2 * q);
        if ((ny & 1) == 0) {  // okq1 == okq0
#pragma unroll
            for (int i = 0; i < KI; ++i) {
                const int k = k0 + i * LT::TP;
                if (i + 1 < KI || k < Kx) gst2(dst, (size_t)k * ny, xe[i], xo[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < KI; ++i) {
                const int k = k0 + i * LT::TP;
                if (i + 1 < KI || k < Kx) {
                    gst(dst, (size_t)k * ny, xe[i]);
                    if (okq1) gst(dst, (size_t)k * ny + 1, xo[i]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// X inverse (C2R of two rows per pencil), first nx outputs, optional
// accumulate and energy partial (one FP64 value per workgroup).
//
// Input: thread (pair q, frequency k) loads B1 at rows 2q and 2q+1 -- one
// 16-byte load (FP32) when ny is even -- and writes the packed pencil
// Z_k = X_even[k] + i X_odd[k] and its mirror to the slab.  Output: when nx is
// a multiple of the 16-byte vector width, the pencil's kept half goes through
// its slab once more so that each thread holds the contiguous positions
// [HALF t, HALF t + HALF) of both rows and writes them (and reads m for the
// energy) as 16-byte vectors (FP32); otherwise each thread writes the
// positions its last stage holds.
template <typename T, int P, int S>
__global__ void __launch_bounds__(xy_max_threads<P>()) kx_inv(const cx<T>* __restrict__ in, T* __restrict__ out,
                                               const T* __restrict__ m, double* __restrict__ partials, int nx,
                                               int ny, int nz, int lgTy, int accumulate, int nxcd,
                                               const cx<T>* __restrict__ twt, BatchIO bio) {
    using LT = p2::Len<P, S>;
    using V = typename vecN<T>::type;
    constexpr int Kx = P / 2 + 1, Lx = P / 2;
    // (FP64 keeps the direct output: its registers would spill)
    constexpr bool kVec = vec_rows<T, P>() && sizeof(T) == 4;
    constexpr int HALF = LT::EPT / 2, VR = vr<T>(), NV = kVec ? HALF / VR : 1;
    __shared__ double red[16];
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int p = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Ty = 1 << lgTy, lgB = lgTy - 1, Bp = Ty >> 1;
    const int nyt = (ny + Ty - 1) >> lgTy;
    int g;
    const int L = batch_tile(xcd_tile(nxcd), bio, &g), yt = L % nyt, zc = L / nyt;
    if (bio.in) {  // batches carry no energy
        in = (const cx<T>*)bio.in[g];
        out = (T*)bio.out[g];
        m = nullptr;
        partials = nullptr;
    }
    const int y0 = yt << lgTy, z = zc % nz, c = zc / nz;
    const int ty = min(Ty, ny - y0);
    const size_t rowbase = (((size_t)c * nz + z) * ny + y0 + 2 * p) * (size_t)nx;
    const bool ok0 = 2 * p < ty, ok1 = 2 * p + 1 < ty;
    const bool vec = kVec && nx % VR == 0;  // uniform
    // energy: the magnetization at this thread's outputs, loaded first so that
    // its latency overlaps the transposition and the transform
    T m0[LT::EPT], m1[LT::EPT];
    V mv0[NV], mv1[NV];
    if (m) {
        const gptr<const T> msrc = gmem(ok0 ? m + rowbase : m);  // rows past the tile read m[0], discarded
        if (vec) {
            const gptr<const T> msrc1 = gmem(ok1 ? m + rowbase + nx : m);
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int x = HALF * t + VR * u;
                mv0[u] = gldv_nt_if(msrc, x, ok0 && x < nx);
                mv1[u] = gldv_nt_if(msrc1, x, ok1 && x < nx);
            }
        } else {
#pragma unroll
            for (int j = 0; j < LT::EPT; ++j) {
                const int k = LT::iout_k(j);
                const int x = t + k * LT::TP;
                if (k < LT::EPT / 2) {
                    m0[j] = gldr_if(msrc, x, ok0 && x < nx);
                    m1[j] = gldr_if(msrc, x + nx, ok1 && x < nx);
                }
            }
        }
    }
    // pair q = tid mod Bp, frequencies k = tid / Bp + i TP: every load of the
    // thread is issued before the first LDS write
    {
        constexpr int KI = (Kx + LT::TP - 1) / LT::TP;
        const int q = tid & (Bp - 1), k0 = tid >> lgB;
        const bool okq0 = 2 * q < ty, okq1 = 2 * q + 1 < ty;
        const cx<T>* qb = in + ((size_t)c * nz + z) * (size_t)Kx * ny + y0 + 2 * q;
        cx<T> xe[KI], xo[KI];
        if ((ny & 1) == 0) {  // rows 2q, 2q+1 side by side, okq1 == okq0
            const gptr<const cx<T>> s0 = gmem(okq0 ? qb : in);
#pragma unroll
            for (int i = 0; i < KI; ++i) {
                const int k = k0 + i * LT::TP;
                gld2_if(s0, (size_t)k * ny, (i + 1 < KI || k < Kx) && okq0, xe[i], xo[i]);
            }
        } else {
            const gptr<const cx<T>> s0 = gmem(okq0 ? qb : in), s1 = gmem(okq1 ? qb + 1 : in);
#pragma unroll
            for (int i = 0; i < KI; ++i) {
                const int k = k0 + i * LT::TP;
                xe[i] = gld_if(s0, (size_t)k * ny, (i + 1 < KI || k < Kx) && okq0);
                xo[i] = gld_if(s1, (size_t)k * ny, (i + 1 < KI || k < Kx) && okq1);
            }
        }
        cx<T>* pq = lds + q * LT::PS;
#pragma unroll
        for (int i = 0; i < KI; ++i) {
            const int k = k0 + i * LT::TP;
            if (i + 1 < KI || k < Kx) {
                cx<T> a = xe[i], b = xo[i];
                if (k == 0 || k == Lx) {  // C2R ignores the imaginary parts of DC and Nyquist
                    a.im = T(0);
                    b.im = T(0);
                }
                pq[LT::pad(k)] = mk(a.re - b.im, a.im + b.re);                           // xe + i xo
                if (k > 0 && k < Lx) pq[LT::pad(P - k)] = mk(a.re + b.im, b.re - a.im);  // conj(xe) + i conj(xo)
            }
        }
    }
    const cx<T>* tws = twiddle_source<T, P>(lds, nthr >> LT::LOG_TP, twt, tid, nthr);
    __syncthreads();
    cx<T>* slab = lds + p * LT::PS;
    cx<T> v[LT::EPT];
    const int pt = LT::pad(t);
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) v[j] = slab[LT::iin_slab(pt, t, j)];
    run_fft<LT, +1>(v, slab, t, tws);
    const gptr<T> dst = out ? gmem(out + rowbase) : nullptr;
    double acc = 0.0;
    if (vec) {
        // the kept half through the slab: position x of row 2p (re) and 2p+1 (im)
        pencil_sync_p<P>();
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::iout_k(j);
            if (k < LT::EPT / 2) slab[LT::pad(t + k * LT::TP)] = v[j];
        }
        pencil_sync_p<P>();
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int x = HALF * t + VR * u;
            V h0, h1;
#pragma unroll
            for (int e = 0; e < VR; ++e) {
                const cx<T> w = slab[LT::pad(x + e)];
                h0[e] = w.re;
                h1[e] = w.im;
            }
            if (x < nx) {  // whole vectors: nx is a multiple of VR
                if (ok0) {
                    if (m) {
#pragma unroll
                        for (int e = 0; e < VR; ++e) acc += (double)(mv0[u][e] * h0[e]);
                    }
                    if (dst) {  // the field is not read again by the evaluation: streamed unless accumulating
                        const gptr<V> d0 = (gptr<V>)(dst + x);
                        if (accumulate) *d0 = *d0 + h0;
                        else __builtin_nontemporal_store(h0, d0);
                    }
                }
                if (ok1) {
                    if (m) {
#pragma unroll
                        for (int e = 0; e < VR; ++e) acc += (double)(mv1[u][e] * h1[e]);
                    }
                    if (dst) {
                        const gptr<V> d1 = (gptr<V>)(dst + nx + x);
                        if (accumulate) *d1 = *d1 + h1;
                        else __builtin_nontemporal_store(h1, d1);
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::iout_k(j);
            const int x = t + k * LT::TP;
            if (k < LT::EPT / 2 && x < nx) {  // the discarded half is never written
                if (ok0) {
                    const T h = v[j].re;
                    if (m) acc += (double)(m0[j] * h);
                    if (dst) {
                        if (accumulate) dst[x] = dst[x] + h;
                        else __builtin_nontemporal_store(h, &dst[x]);
                    }
                }
                if (ok1) {
                    const T h = v[j].im;
                    if (m) acc += (double)(m1[j] * h);
                    if (dst) {
                        if (accumulate) dst[x + nx] = dst[x + nx] + h;
                        else __builtin_nontemporal_store(h, &dst[x + nx]);
                    }
                }
            }
        }
    }
    if (partials) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < (nthr + 63) / 64; ++w) sum += red[w];
            partials[L] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Y forward.  Tile Tz x Tx pencils (z, kx); pencil p = zi * Tx + xi.
// 1-D grid of ceil(nz/Tz) * ceil(Kx/Tx) * C tiles, block Tz * Tx * TP.
//
// FP32 with an even nz and z tiles of at least two: each thread writes two
// adjacent z pencils at a frequency with one 16-byte store (the strided side).
template <typename T, int P, int S>
__global__ void __launch_bounds__(xy_max_threads<P>()) ky_fwd(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int ny,
                                               int nz, int Kx, int lgTz, int lgTx, int nxcd,
                                               const cx<T>* __restrict__ twt, BatchIO bio) {
    using LT = p2::Len<P, S>;
    constexpr bool kVec = sizeof(T) == 4 && LT::EPT >= 8;
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x;
    const int p = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Tx = 1 << lgTx, Tz = 1 << lgTz;
    const int nzt = (nz + Tz - 1) >> lgTz, nxt = (Kx + Tx - 1) >> lgTx;
    int g;
    const int L = batch_tile(xcd_tile(nxcd), bio, &g), zt = L % nzt, xc = L / nzt;
    if (bio.in) {
        in = (const cx<T>*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int kx0 = (xc % nxt) << lgTx, z0 = zt << lgTz, c = xc / nxt;
    const int tx = min(Tx, Kx - kx0), tz = min(Tz, nz - z0);
    const int xi = p & (Tx - 1), zi = p >> lgTx;
    const bool ok = xi < tx && zi < tz;
    const gptr<const cx<T>> src = gmem(ok ? in + (((size_t)c * nz + z0 + zi) * Kx + kx0 + xi) * (size_t)ny : in);
    cx<T> v[LT::EPT];
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) {
        const int k = LT::fin_k(j);
        const int y = t + k * LT::TP;
        v[j] = k < LT::EPT / 2 ? gld_if(src, y, ok && y < ny) : czero<T>();
    }
    cx<T>* slab = lds + p * LT::PS;
    const cx<T>* tws = twiddle_source<T, P>(lds, (int)blockDim.x >> LT::LOG_TP, twt, tid, blockDim.x);
    if constexpr (tw_in_lds<T, P>()) __syncthreads();
    run_fft<LT, -1, true>(v, slab, t, tws);
    __syncthreads();
    const int pt = LT::pad(t);
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) slab[LT::fout_slab(pt, t, j)] = v[j];
    __syncthreads();
    const int lgB = lgTz + lgTx;
    const size_t step = (size_t)LT::TP * nz;  // B2 offset of TP frequencies ky
    if (kVec && lgTz >= 1 && (nz & 1) == 0) {
        // pair (zq, xj) = tid mod (Tz/2 Tx) writes pencils z0 + 2 zq and z0 + 2 zq + 1
        // (both inside the tile or both outside: tz is even), ky = tid / (Tz/2 Tx) + i 2 TP
        const int zq = tid & ((Tz >> 1) - 1), xj = (tid >> (lgTz - 1)) & (Tx - 1), ky0 = tid >> (lgB - 1);
        if (2 * zq < tz && xj < tx) {
            const cx<T>* pj = lds + (((2 * zq) << lgTx) + xj) * LT::PS;
            const int pk = LT::pad(ky0);
            cx<T> lo[LT::EPT / 2], hi[LT::EPT / 2];
#pragma unroll
            for (int i = 0; i < LT::EPT / 2; ++i) {
                lo[i] = pj[LT::pad_add(pk, ky0, 2 * i * LT::TP)];
                hi[i] = pj[Tx * LT::PS + LT::pad_add(pk, ky0, 2 * i * LT::TP)];
            }
            const gptr<cx<T>> dst = gmem(out + (((size_t)c * Kx + kx0 + xj) * P + ky0) * (size_t)nz + z0 + 2 * zq);
#pragma unroll
            for (int i = 0; i < LT::EPT / 2; ++i) gst2(dst, 2 * i * step, lo[i], hi[i]);
        }
    } else {
        // (zj, xj) = tid mod (Tz Tx), ky = tid / (Tz Tx) + i TP; z-contiguous runs
        const int zj = tid & (Tz - 1), xj = (tid >> lgTz) & (Tx - 1), ky0 = tid >> lgB;
        if (zj < tz && xj < tx) {
            const cx<T>* pj = lds + ((zj << lgTx) + xj) * LT::PS;
            const int pk = LT::pad(ky0);
            cx<T> r[LT::EPT];
#pragma unroll
            for (int i = 0; i < LT::EPT; ++i) r[i] = pj[LT::pad_add(pk, ky0, i * LT::TP)];
            const gptr<cx<T>> dst = gmem(out + (((size_t)c * Kx + kx0 + xj) * P + ky0) * (size_t)nz + z0 + zj);
#pragma unroll
            for (int i = 0; i < LT::EPT; ++i) gst(dst, i * step, r[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// Y inverse: first ny outputs, written y-contiguous.
template <typename T, int P, int S>
__global__ void __launch_bounds__(xy_max_threads<P>()) ky_inv(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int ny,
                                               int nz, int Kx, int lgTz, int lgTx, int nxcd,
                                               const cx<T>* __restrict__ twt, BatchIO bio) {
    using LT = p2::Len<P, S>;
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x;
    const int p = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Tx = 1 << lgTx, Tz = 1 << lgTz;
    const int nzt = (nz + Tz - 1) >> lgTz, nxt = (Kx + Tx - 1) >> lgTx;
    int g;
    const int L = batch_tile(xcd_tile(nxcd), bio, &g), zt = L % nzt, xc = L / nzt;
    if (bio.in) {
        in = (const cx<T>*)bio.in[g];
        out = (cx<T>*)bio.out[g];
    }
    const int kx0 = (xc % nxt) << lgTx, z0 = zt << lgTz, c = xc / nxt;
    const int tx = min(Tx, Kx - kx0), tz = min(Tz, nz - z0);
    const int lgB = lgTz + lgTx;
    {
        // (zj, xj) = tid mod (Tz Tx), ky = tid / (Tz Tx) + i TP: all EPT loads of
        // the thread are issued before its LDS writes
        const int zj = tid & (Tz - 1), xj = (tid >> lgTz) & (Tx - 1), ky0 = tid >> lgB;
        const bool okj = zj < tz && xj < tx;
        const gptr<const cx<T>> src =
            gmem(okj ? in + (((size_t)c * Kx + kx0 + xj) * P + ky0) * (size_t)nz + z0 + zj : in);
        const size_t step = (size_t)LT::TP * nz;  // B2 offset of TP frequencies ky
        cx<T> ld[LT::EPT];
#pragma unroll
        for (int i = 0; i < LT::EPT; ++i) ld[i] = gld_last_if(src, i * step, okj);
        cx<T>* pj = lds + ((zj << lgTx) + xj) * LT::PS;
        const int pk = LT::pad(ky0);
#pragma unroll
        for (int i = 0; i < LT::EPT; ++i) pj[LT::pad_add(pk, ky0, i * LT::TP)] = ld[i];
    }
    const cx<T>* tws = twiddle_source<T, P>(lds, (int)blockDim.x >> LT::LOG_TP, twt, tid, blockDim.x);
    __syncthreads();
    cx<T>* slab = lds + p * LT::PS;
    cx<T> v[LT::EPT];
    const int pt = LT::pad(t);
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) v[j] = slab[LT::iin_slab(pt, t, j)];
    run_fft<LT, +1>(v, slab, t, tws);
    const int xi = p & (Tx - 1), zi = p >> lgTx;
    if (xi < tx && zi < tz) {
        const gptr<cx<T>> dst = gmem(out + (((size_t)c * nz + z0 + zi) * Kx + kx0 + xi) * (size_t)ny);
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::iout_k(j);
            const int y = t + k * LT::TP;
            if (k < LT::EPT / 2 && y < ny) gst(dst, y, v[j]);
        }
    }
}

// ---------------------------------------------------------------------------
// Fused Z pass.  A tile is Tx consecutive rows of one kx (B2 and the tensor
// octant are kx-major, so its pencils and tensor rows are contiguous runs, and
// consecutive tiles continue them).  Group g = s * Tx + xi handles the three
// component pencils at (kx, ky_s), ky_0 = ky' = r0 + xi, ky_1 = Py - ky'; each
// thread keeps all three components in registers, so the tensor product needs
// no exchange and the forward output slots hand over to the inverse input
// slots in registers.  Paired form (rows = 2): 1-D grid of
// Kx * ceil((Py/2 + 1)/Tx) tiles, block 2 * Tx * TP; a row and its mirror share
// the tensor octant row ky' (ky' = 0 and Py/2 have no mirror).  Split form
// (rows = 1, for lengths whose pair would exceed the workgroup): rows ky =
// r0 + xi of the whole range, Kx * ceil(Py/Tx) tiles, block Tx * TP,
// s = (ky > Py/2).
// Every B2 and tensor access is a raw buffer access (one resource per B2
// component, one for the tensor octant with the component in the scalar
// offset); the host guarantees that each range is below kOob.
//
// Register budget.  FP32 power-of-two lengths keep the thread's twiddles in
// registers for all six transforms; FP64 (twice the registers) and lengths
// 3 * 2^a (three times the slots) read them per transform from the
// workgroup's LDS copy of the table (from memory if it is larger than
// kP2TwLdsMax).  Power-of-two lengths in the paired form copy the tile's
// tensor rows into LDS with 16-byte loads issued together with the data loads
// and read each frequency's six values from LDS right before its product; the
// split form at 4096 (FP32) loads them into registers up front, and lengths
// 3 * 2^a (24 values per component in a thread) load each frequency's six
// values from memory right before its product, which keeps them within the
// register file (loaded together after the forward transforms they spilled).
template <typename T, int P>
__host__ __device__ constexpr bool z_keep_twiddles() {
    return sizeof(T) == 4 && p2::is_pow2(P);
}
// For power-of-two lengths in the paired form the tile's tensor rows (one
// contiguous run of the kx-major octant) are staged in LDS and each
// frequency's six values are read right before its product, instead of
// holding all of the thread's tensor values in registers: FP32 P = 128
// 142 -> 97 VGPRs (3 -> 4 waves per SIMD), fused Z pass 109 -> 100 us at
// 256x256x64; FP64 P = 128 182 -> 165 VGPRs, 220 -> 210 us.  (For lengths
// 3 * 2^a, whose threads hold 24 frequencies, the staging measured slower:
// the 96-grid batch 499 -> 527 us.)  The staging area follows the slabs and
// the LDS copy of the twiddle table, 16-byte aligned.
template <typename T, int P>
__host__ __device__ constexpr size_t z_stage_offset(int G) {
    const size_t tw = z_keep_twiddles<T, P>() || !tw_in_lds<T, P>() ? 0 : p2::Len<P>::table_size() * sizeof(cx<T>);
    return ((size_t)G * p2::Len<P>::PS * sizeof(cx<T>) + tw + 15) & ~(size_t)15;
}

template <typename T, int P, int S, bool EN = false, bool TNT = false>
__global__ void __launch_bounds__(kP2MaxThreadsZ) kz_conv(cx<T>* __restrict__ B2, const T* __restrict__ nhat, T Ms, int nz,
                                                int Py, int Kx, int lgTx, int rows, int nxcd,
                                                const cx<T>* __restrict__ twt, BatchIO bio,
                                                double* __restrict__ epart = nullptr) {
    using LT = p2::Len<P, S>;
    constexpr bool kPow2 = p2::is_pow2(P);
    constexpr bool kKeep = z_keep_twiddles<T, P>();
    constexpr int Lz = P / 2;
    constexpr unsigned CB = sizeof(cx<T>), RB = sizeof(T);
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x;
    const int g = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Tx = 1 << lgTx, Ly = Py >> 1;
    const int xi = g & (Tx - 1);
    int gb;
    const int tile = batch_tile(xcd_tile(nxcd), bio, &gb);
    if (bio.in) B2 = (cx<T>*)bio.out[gb];
    // a tile: Tx consecutive rows ky' (and their mirrors) of one kx
    const int nrow = rows == 2 ? (Ly + Tx) >> lgTx : (Py + Tx - 1) >> lgTx;
    const int kx = tile / nrow, r0 = (tile % nrow) << lgTx;
    int s, kyp, ky;
    bool ok;
    if (rows == 2) {
        s = g >> lgTx;
        kyp = r0 + xi;
        ok = kyp <= Ly && (s == 0 || (kyp != 0 && kyp != Ly));
        ky = s ? Py - kyp : kyp;
    } else {
        ky = r0 + xi;
        ok = ky < Py;
        s = ky > Ly;
        kyp = s ? Py - ky : ky;
    }
    const size_t cstride = (size_t)Py * Kx * nz;  // component stride of B2 (elements)
    const Buf bc[3] = {make_buf(B2, cstride * CB), make_buf(B2 + cstride, cstride * CB),
                       make_buf(B2 + 2 * cstride, cstride * CB)};
    // byte offset of this lane's first element; zz = t + k TP adds k TP CB
    const unsigned row = (unsigned)((((size_t)kx * Py + ky) * nz + t) * CB);
    // the energy alone is the spectrum's last reader: its loads are non-temporal
    cx<T> v[3][LT::EPT];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::fin_k(j);
            const int zz = t + k * LT::TP;
            v[comp][j] = k < LT::EPT / 2 ? bld<T, EN ? kNt : 0>(bc[comp], boff(ok && zz < nz, row, k * LT::TP * CB))
                                         : czero<T>();
        }
    }
    // Tensor values of this thread's frequencies kz (forward output slots);
    // octant index kz' = kz for kz <= Lz, else P - kz; lanes outside the tile
    // read row 0 (their results are never stored).
    // octant [Kx][Ly+1][Lz+1][6]: the six components of a frequency side by side
    constexpr unsigned FB = 6 * RB;  // bytes per frequency
    const Buf bt = make_buf(nhat, (size_t)Kx * (Ly + 1) * (Lz + 1) * FB);
    const unsigned trow = ok ? (unsigned)((((size_t)kx * (Ly + 1) + kyp) * (Lz + 1)) * FB) : 0u;
    T nt[LT::EPT][6];
    auto load_tensor = [&]() {
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            unsigned off;
            if constexpr (kPow2) {
                // kz = t + k TP; for k >= EPT/2, P - kz = (TP - 1 - t) + P - (k + 1) TP + 1
                const int k = LT::F::slot_out(j);
                off = k < LT::EPT / 2 ? trow + (t + k * LT::TP) * FB : trow + ((LT::TP - 1 - t) + P - (k + 1) * LT::TP + 1) * FB;
            } else {
                const int kz = LT::fout(t, j);
                off = trow + (kz <= Lz ? kz : P - kz) * FB;
            }
            bld6<T>(bt, off, nt[j]);
        }
    };
    constexpr bool kStage = kPow2 && 2 * LT::TP <= kP2MaxThreadsZ;  // power-of-two lengths, paired form
    // kStage: the tile's octant rows (kx, r0 .. r0 + Tx - 1) are one contiguous
    // run; it is copied into LDS (after the slabs) with 16-byte loads from a
    // 16-byte-aligned start, and each frequency's six values are read from there
    // right before its product.
    const T* tls = nullptr;
    unsigned tmis = 0;
    if constexpr (kStage) {
        const int nthr = blockDim.x;
        const int G = rows << lgTx;
        const unsigned tb0 = (unsigned)((((size_t)kx * (Ly + 1) + r0) * (Lz + 1)) * FB);
        const unsigned tal = tb0 & ~15u;
        tmis = tb0 - tal;
        const unsigned nbytes = (unsigned)min(Tx, Ly + 1 - r0) * (Lz + 1) * FB + tmis;
        constexpr int NCH = ((Lz + 1) * (int)FB + 16 + 32 * LT::TP - 1) / (32 * LT::TP);
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        u4 ch[NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q)
            ch[q] = __builtin_amdgcn_raw_buffer_load_b128(bt.r, tal + (unsigned)(tid + q * nthr) * 16u, 0, TNT ? kNt : 0);
        unsigned char* sbase = (unsigned char*)lds + z_stage_offset<T, P>(G);
        u4* dstl = (u4*)sbase;
#pragma unroll
        for (int q = 0; q < NCH; ++q)
            if ((unsigned)(tid + q * nthr) * 16u < nbytes) dstl[tid + q * nthr] = ch[q];
        __syncthreads();
        tls = (const T*)(sbase + tmis) + (size_t)xi * (Lz + 1) * 6;
    } else if constexpr (kKeep) {
        load_tensor();
    }
    cx<T>* slab = lds + g * LT::PS;
    const cx<T>* twsrc = twt;
    if constexpr (!kKeep) {
        twsrc = twiddle_source<T, P>(lds, (int)blockDim.x >> LT::LOG_TP, twt, tid, blockDim.x);
        if constexpr (tw_in_lds<T, P>()) __syncthreads();
    }
    typename LT::template Tw<T> tws;
    if constexpr (kKeep) tws.load(t, twsrc);
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        if constexpr (kKeep) LT::template fft<-1, true>(v[comp], slab, t, tws);
        else run_fft<LT, -1, true>(v[comp], slab, t, twsrc);
    }
    constexpr bool kLazy = !kPow2;  // 3 * 2^a: each frequency's six values loaded right before its product
    if constexpr (!kKeep && !kStage && !kLazy) load_tensor();
    // H^ = Nhat(kx, ky, kz) M^ (Ms applied at the store).  Octant lookup with
    // parity signs: xy, yz odd in ky (negative for ky > Ly, i.e. s = 1); xz, yz
    // odd in kz, negative for kz > Lz.  For power-of-two lengths that is slot
    // k >= EPT/2 (a compile-time property) except kz = Lz itself, where the odd
    // components are exactly zero.
    const T sy = s ? T(-1) : T(1);
    double eacc = 0.0;  // EN: sum over this thread's frequencies of Re(M^H N M)
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) {
        bool negz;
        if constexpr (kPow2) negz = LT::F::slot_out(j) >= LT::EPT / 2;
        else negz = LT::fout(t, j) > Lz;
        if constexpr (kLazy && !kStage && !kKeep) {
            const int kz = LT::fout(t, j);
            bld6<T>(bt, trow + (kz <= Lz ? kz : P - kz) * FB, nt[j]);
        }
        if constexpr (kStage) {
            int kzp;
            if constexpr (kPow2) {
                const int k = LT::F::slot_out(j);
                kzp = k < LT::EPT / 2 ? t + k * LT::TP : (LT::TP - 1 - t) + P - (k + 1) * LT::TP + 1;
            } else {
                const int kz = LT::fout(t, j);
                kzp = kz <= Lz ? kz : P - kz;
            }
            typedef T t2 __attribute__((ext_vector_type(2)));
            const t2* e = (const t2*)(tls + kzp * 6);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const t2 u = e[i];
                nt[j][2 * i] = u.x;
                nt[j][2 * i + 1] = u.y;
            }
        }
        const T nxx = nt[j][0], nyy = nt[j][1], nzz = nt[j][2];
        const T nxy = sy * nt[j][3];
        const T nxz = negz ? -nt[j][4] : nt[j][4];
        const T nyz = negz ? -(sy * nt[j][5]) : sy * nt[j][5];
        const cx<T> mx = v[0][j], my = v[1][j], mz = v[2][j];
        const cx<T> hx = mk(nxx * mx.re + nxy * my.re + nxz * mz.re, nxx * mx.im + nxy * my.im + nxz * mz.im);
        const cx<T> hy = mk(nxy * mx.re + nyy * my.re + nyz * mz.re, nxy * mx.im + nyy * my.im + nyz * mz.im);
        const cx<T> hz = mk(nxz * mx.re + nyz * my.re + nzz * mz.re, nxz * mx.im + nyz * my.im + nzz * mz.im);
        if constexpr (EN) {
            eacc += (double)(mx.re * hx.re + mx.im * hx.im + my.re * hy.re + my.im * hy.im + mz.re * hz.re +
                             mz.im * hz.im);
        } else {
            v[0][j] = hx;
            v[1][j] = hy;
            v[2][j] = hz;
        }
    }
    if constexpr (EN) {
        // Parseval: sum_i m_i . (N * m)_i over the padded grid (m zero off the
        // grid) = sum over the full spectrum of Re(M^H Nhat M); the stored half
        // (kx <= Px/2) counts kx = 0 and kx = Px/2 once and the rest twice
        // (Hermitian symmetry).  Per workgroup one FP64 partial, summed in a
        // fixed order (a tree over the threads in LDS; the thread count is a
        // power of two).
        __syncthreads();  // the slabs are no longer read: reuse them
        double* red = (double*)lds;
        red[tid] = ok ? eacc * (kx == 0 || kx == Kx - 1 ? 1.0 : 2.0) : 0.0;
        __syncthreads();
        for (int w = (int)blockDim.x >> 1; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) epart[blockIdx.x] = red[0];
        return;
    }
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        cx<T> w[LT::EPT];
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) w[j] = v[comp][LT::fwd_slot_of_iin(j)];
        if constexpr (kKeep) LT::template fft<+1, false>(w, slab, t, tws);
        else run_fft<LT, +1>(w, slab, t, twsrc);
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::iout_k(j);
            const int zz = t + k * LT::TP;
            if (k < LT::EPT / 2)  // the discarded half is never written
                bst<T>(bc[comp], boff(ok && zz < nz, row, k * LT::TP * CB), mk(Ms * w[j].re, Ms * w[j].im));
        }
    }
}

// ---------------------------------------------------------------------------
// Fused Z pass of the scalar-potential method (Sec. 3.1, eq. (convolution)):
// per (kx, ky) the three component pencils are transformed along z, combined
// with the kernel spectrum S^_a = i s_a (s_a real: Im of the transform of the
// odd kernel, octant [Kx][Py/2+1][3][Pz/2+1], +1/(Px Py Pz) folded in) into
// phi^ = i sum_a s_a M^_a, transformed back, and Ms phi (first nz outputs) is
// written in place to component 0 of B2.  Parity signs: s_y odd in ky (s = 1
// groups), s_z odd in kz; s_x needs none (kx <= Px/2).  Tiles, groups, buffer
// access and register budget as in kz_conv.
template <typename T, int P, int S>
__global__ void __launch_bounds__(kP2MaxThreadsZ) kz_sp(cx<T>* __restrict__ B2, const T* __restrict__ shat, T Ms,
                                                        int nz, int Py, int Kx, int lgTx, int rows, int nxcd,
                                                        const cx<T>* __restrict__ twt) {
    using LT = p2::Len<P, S>;
    constexpr bool kPow2 = p2::is_pow2(P);
    constexpr bool kKeep = z_keep_twiddles<T, P>();
    constexpr int Lz = P / 2;
    constexpr unsigned CB = sizeof(cx<T>), RB = sizeof(T);
    cx<T>* lds = lds_base<T>();
    const int tid = threadIdx.x;
    const int g = tid >> LT::LOG_TP, t = tid & (LT::TP - 1);
    const int Tx = 1 << lgTx, Ly = Py >> 1;
    const int xi = g & (Tx - 1);
    const int tile = xcd_tile(nxcd);
    // a tile: Tx consecutive rows ky' (and their mirrors) of one kx
    const int nrow = rows == 2 ? (Ly + Tx) >> lgTx : (Py + Tx - 1) >> lgTx;
    const int kx = tile / nrow, r0 = (tile % nrow) << lgTx;
    int s, kyp, ky;
    bool ok;
    if (rows == 2) {
        s = g >> lgTx;
        kyp = r0 + xi;
        ok = kyp <= Ly && (s == 0 || (kyp != 0 && kyp != Ly));
        ky = s ? Py - kyp : kyp;
    } else {
        ky = r0 + xi;
        ok = ky < Py;
        s = ky > Ly;
        kyp = s ? Py - ky : ky;
    }
    const size_t cstride = (size_t)Py * Kx * nz;
    const Buf bc[3] = {make_buf(B2, cstride * CB), make_buf(B2 + cstride, cstride * CB),
                       make_buf(B2 + 2 * cstride, cstride * CB)};
    const unsigned row = (unsigned)((((size_t)kx * Py + ky) * nz + t) * CB);
    cx<T> v[3][LT::EPT];
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            const int k = LT::fin_k(j);
            const int zz = t + k * LT::TP;
            v[comp][j] = k < LT::EPT / 2 ? bld<T, kNt>(bc[comp], boff(ok && zz < nz, row, k * LT::TP * CB)) : czero<T>();
        }
    }
    const size_t cs = (size_t)(Lz + 1);  // component stride of the spectrum octant
    const Buf bt = make_buf(shat, (size_t)Kx * (Ly + 1) * 3 * cs * RB);
    const unsigned trow = ok ? (unsigned)((((size_t)kx * (Ly + 1) + kyp) * 3 * (Lz + 1)) * RB) : 0u;
    T sk[LT::EPT][3];
    // kStage (as in kz_conv): the tile's kernel rows (kx, r0 .. r0 + Tx - 1)
    // are one contiguous run, copied into LDS after the slabs with 16-byte
    // loads; each frequency's three values are read from there before use
    // (not in FP64 at 2048, where it spilled more registers than it saved)
    constexpr bool kStage = kPow2 && 2 * LT::TP <= kP2MaxThreadsZ && (sizeof(T) == 4 || P <= 1024);
    const T* tls = nullptr;
    if constexpr (kStage) {
        constexpr unsigned RowB = 3 * (Lz + 1) * RB;  // bytes per octant row
        const int nthr = blockDim.x;
        const int G = rows << lgTx;
        const unsigned tb0 = (unsigned)(((size_t)kx * (Ly + 1) + r0) * RowB);
        const unsigned tal = tb0 & ~15u;
        const unsigned tmis = tb0 - tal;
        const unsigned nbytes = (unsigned)min(Tx, Ly + 1 - r0) * RowB + tmis;
        constexpr int NCH = ((int)RowB + 16 + 32 * LT::TP - 1) / (32 * LT::TP);
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        u4 ch[NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q) ch[q] = __builtin_amdgcn_raw_buffer_load_b128(bt.r, tal + (unsigned)(tid + q * nthr) * 16u, 0, kNt);
        unsigned char* sbase = (unsigned char*)lds + z_stage_offset<T, P>(G);
        u4* dstl = (u4*)sbase;
#pragma unroll
        for (int q = 0; q < NCH; ++q)
            if ((unsigned)(tid + q * nthr) * 16u < nbytes) dstl[tid + q * nthr] = ch[q];
        __syncthreads();
        tls = (const T*)(sbase + tmis) + (size_t)xi * 3 * (Lz + 1);
    }
    auto load_kernel = [&]() {
#pragma unroll
        for (int j = 0; j < LT::EPT; ++j) {
            unsigned off;
            if constexpr (kPow2) {
                const int k = LT::F::slot_out(j);
                off = k < LT::EPT / 2 ? trow + (t + k * LT::TP) * RB : trow + ((LT::TP - 1 - t) + P - (k + 1) * LT::TP + 1) * RB;
            } else {
                const int kz = LT::fout(t, j);
                off = trow + (kz <= Lz ? kz : P - kz) * RB;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) sk[j][a] = bldr<T>(bt, off, (unsigned)(a * cs * RB));
        }
    };
    if constexpr (kKeep && !kStage) load_kernel();
    cx<T>* slab = lds + g * LT::PS;
    const cx<T>* twsrc = twt;
    if constexpr (!kKeep) {
        twsrc = twiddle_source<T, P>(lds, (int)blockDim.x >> LT::LOG_TP, twt, tid, blockDim.x);
        if constexpr (tw_in_lds<T, P>()) __syncthreads();
    }
    typename LT::template Tw<T> tws;
    if constexpr (kKeep) tws.load(t, twsrc);
#pragma unroll
    for (int comp = 0; comp < 3; ++comp) {
        if constexpr (kKeep) LT::template fft<-1, true>(v[comp], slab, t, tws);
        else run_fft<LT, -1, true>(v[comp], slab, t, twsrc);
    }
    if constexpr (!kKeep && !kStage) load_kernel();
    const T sy = s ? T(-1) : T(1);
    cx<T> w[LT::EPT];
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) {
        bool negz;
        if constexpr (kPow2) negz = LT::F::slot_out(j) >= LT::EPT / 2;
        else negz = LT::fout(t, j) > Lz;
        if constexpr (kStage) {
            const int k = LT::F::slot_out(j);
            const int kzp = k < LT::EPT / 2 ? t + k * LT::TP : (LT::TP - 1 - t) + P - (k + 1) * LT::TP + 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) sk[j][a] = tls[a * (Lz + 1) + kzp];
        }
        const T ax = sk[j][0], ay = sy * sk[j][1], az = negz ? -sk[j][2] : sk[j][2];
        const cx<T> c = mk(ax * v[0][j].re + ay * v[1][j].re + az * v[2][j].re,
                           ax * v[0][j].im + ay * v[1][j].im + az * v[2][j].im);
        v[0][j] = mk(-c.im, c.re);  // times i
    }
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) w[j] = v[0][LT::fwd_slot_of_iin(j)];
    if constexpr (kKeep) LT::template fft<+1, false>(w, slab, t, tws);
    else run_fft<LT, +1>(w, slab, t, twsrc);
#pragma unroll
    for (int j = 0; j < LT::EPT; ++j) {
        const int k = LT::iout_k(j);
        const int zz = t + k * LT::TP;
        if (k < LT::EPT / 2) bst<T>(bc[0], boff(ok && zz < nz, row, k * LT::TP * CB), mk(Ms * w[j].re, Ms * w[j].im));
    }
}

template <int P>
constexpr int tpp() { return p2::Len<P>::TP; }

// Dynamic LDS above 64 KB must be allowed per kernel before its launch.
template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}


}  // namespace

// ---------------------------------------------------------------------------
// host launchers: switch on the runtime length to the compile-time instance
#define DEMAG_P2_CASES_POW2(CALL)                                                                  \
    case 2: CALL(2); break;                                                                        \
    case 4: CALL(4); break;                                                                        \
    case 8: CALL(8); break;                                                                        \
    case 16: CALL(16); break;                                                                      \
    case 32: CALL(32); break;                                                                      \
    case 64: CALL(64); break;                                                                      \
    case 128: CALL(128); break;                                                                    \
    case 256: CALL(256); break;                                                                    \
    case 512: CALL(512); break;                                                                    \
    case 1024: CALL(1024); break;                                                                  \
    case 2048: CALL(2048); break;                                                                  \
    case 4096: CALL(4096); break;
#define DEMAG_P2_CASES_3POW2(CALL)                                                                 \
    case 6: CALL(6); break;                                                                        \
    case 12: CALL(12); break;                                                                      \
    case 24: CALL(24); break;                                                                      \
    case 48: CALL(48); break;                                                                      \
    case 96: CALL(96); break;                                                                      \
    case 192: CALL(192); break;                                                                    \
    case 384: CALL(384); break;                                                                    \
    case 768: CALL(768); break;                                                                    \
    case 1536: CALL(1536); break;                                                                  \
    case 3072: CALL(3072); break;
#define DEMAG_P2_SWITCH(P, CALL)                                                                   \
    switch (P) {                                                                                   \
        DEMAG_P2_CASES_POW2(CALL)                                                                  \
        DEMAG_P2_CASES_3POW2(CALL)                                                                 \
    default: return hipErrorInvalidValue;                                                          \
    }
// The radix schedule `sched` of length PP as a compile-time instance (CALLS(PP, S)).
#define DEMAG_P2_SCHED(PP, CALLS)                                                                  \
    switch (sched) {                                                                               \
    case 0: CALLS(PP, 0); break;                                                                   \
    case 1:                                                                                        \
        if constexpr (p2::is_pow2(PP) && p2::num_schedules(PP) > 1) { CALLS(PP, 1); }              \
        else { return hipErrorInvalidValue; }                                                      \
        break;                                                                                     \
    case 2:                                                                                        \
        if constexpr (p2::is_pow2(PP) && p2::num_schedules(PP) > 2) { CALLS(PP, 2); }              \
        else { return hipErrorInvalidValue; }                                                      \
        break;                                                                                     \
    default: return hipErrorInvalidValue;                                                          \
    }

int kXcds = 8;  // XCDs of the device (workgroup swizzle); set by the plan runtime

bool p2_supported(int P) { return P <= 4096 && p2::reg_length(P); }
bool p2_z_supported(int P, size_t cbytes) {
    return p2_supported(P) && (p2::is_pow2(P) || cbytes == sizeof(cx<float>));
}
int p2_threads_per_pencil(int P) {
    const int q = p2::is_pow2(P) ? P : P / 3;  // the power-of-two transforms' length
    return q >= 8 ? q / 8 : 1;
}
int p2_slab_elems(int P) { return (P + (P >> 3)) + 1; }
int p2_max_threads(int P) { return p2::is_pow2(P) ? 1024 : 512; }  // xy_max_threads
int p2_num_schedules(int P) { return p2_supported(P) && p2::is_pow2(P) ? p2::num_schedules(P) : (p2_supported(P) ? 1 : 0); }
static size_t table_entries(int P) {
    switch (P) {
#define TS(PP) \
    case PP: return (size_t)p2::Len<PP>::table_size();
        TS(2) TS(4) TS(8) TS(16) TS(32) TS(64) TS(128) TS(256) TS(512) TS(1024) TS(2048) TS(4096)
        TS(6) TS(12) TS(24) TS(48) TS(96) TS(192) TS(384) TS(768) TS(1536) TS(3072)
#undef TS
    default: return 0;
    }
}
size_t p2_twiddle_lds_bytes(int P, size_t cbytes) {
    const size_t n = table_entries(P);
    return n * cbytes <= kP2TwLdsMax ? n * cbytes : 0;
}
size_t p2_z_lds_bytes(int P, int rows, int lgTx, size_t cbytes) {
    size_t lds = (size_t)(rows << lgTx) * p2_slab_elems(P) * cbytes + p2_z_twiddle_lds_bytes(P, cbytes);
    if (p2::is_pow2(P) && 2 * p2_threads_per_pencil(P) <= kP2MaxThreadsZ)  // tensor staging (kz_conv's kStage)
        lds = ((lds + 15) & ~(size_t)15) + (size_t)(1 << lgTx) * (P / 2 + 1) * 3 * cbytes + 16;
    return lds;
}
size_t p2_z_twiddle_lds_bytes(int P, size_t cbytes) {
    const bool keep = cbytes == sizeof(cx<float>) && p2::is_pow2(P);  // z_keep_twiddles
    return keep ? 0 : p2_twiddle_lds_bytes(P, cbytes);
}

template <typename T>
hipError_t launch_x_fwd_p2(int lgTy, int sched, hipStream_t st, const T* in, cx<T>* out, int nx, int ny, int nz, int C,
                           int P, const cx<T>* twt, const BatchIO& bio) {
    if (!twt) return hipErrorInvalidValue;
    const int Bp = 1 << (lgTy - 1);
    dim3 grid((unsigned)(((ny + (1 << lgTy) - 1) >> lgTy) * nz * C * bio.count));
    const size_t lds = (size_t)Bp * p2_slab_elems(P) * sizeof(cx<T>) + p2_twiddle_lds_bytes(P, sizeof(cx<T>));
#define CALLS(PP, SS) \
    if (hipError_t e_ = allow_lds(&kx_fwd<T, PP, SS>, lds)) return e_; \
    hipLaunchKernelGGL((kx_fwd<T, PP, SS>), grid, dim3(Bp * tpp<PP>()), lds, st, in, out, nx, ny, nz, lgTy, kXcds, twt, \
                       bio)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    DEMAG_P2_SWITCH(P, CALL)
#undef CALL
#undef CALLS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_x_inv_p2(int lgTy, int sched, hipStream_t st, const cx<T>* in, T* out, const T* m, double* partials,
                           int nx, int ny, int nz, int C, int accumulate, int P, const cx<T>* twt, const BatchIO& bio) {
    if (!twt) return hipErrorInvalidValue;
    const int Bp = 1 << (lgTy - 1);
    dim3 grid((unsigned)(((ny + (1 << lgTy) - 1) >> lgTy) * nz * C * bio.count));
    const size_t lds = (size_t)Bp * p2_slab_elems(P) * sizeof(cx<T>) + p2_twiddle_lds_bytes(P, sizeof(cx<T>));
#define CALLS(PP, SS)                                                                                       \
    if (hipError_t e_ = allow_lds(&kx_inv<T, PP, SS>, lds)) return e_; \
    hipLaunchKernelGGL((kx_inv<T, PP, SS>), grid, dim3(Bp * tpp<PP>()), lds, st, in, out, m, partials, nx, ny, nz, \
                       lgTy, accumulate, kXcds, twt, bio)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    DEMAG_P2_SWITCH(P, CALL)
#undef CALL
#undef CALLS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_fwd_p2(int lgTz, int lgTx, int sched, hipStream_t st, const cx<T>* in, cx<T>* out, int ny, int nz,
                           int Kx, int C, int P, const cx<T>* twt, const BatchIO& bio) {
    if (!twt) return hipErrorInvalidValue;
    const int B = 1 << (lgTz + lgTx);
    dim3 grid((unsigned)(((Kx + (1 << lgTx) - 1) >> lgTx) * ((nz + (1 << lgTz) - 1) >> lgTz) * C * bio.count));
    const size_t lds = (size_t)B * p2_slab_elems(P) * sizeof(cx<T>) + p2_twiddle_lds_bytes(P, sizeof(cx<T>));
#define CALLS(PP, SS) \
    if (hipError_t e_ = allow_lds(&ky_fwd<T, PP, SS>, lds)) return e_; \
    hipLaunchKernelGGL((ky_fwd<T, PP, SS>), grid, dim3(B * tpp<PP>()), lds, st, in, out, ny, nz, Kx, lgTz, lgTx, kXcds, \
                       twt, bio)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    DEMAG_P2_SWITCH(P, CALL)
#undef CALL
#undef CALLS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_y_inv_p2(int lgTz, int lgTx, int sched, hipStream_t st, const cx<T>* in, cx<T>* out, int ny, int nz,
                           int Kx, int C, int P, const cx<T>* twt, const BatchIO& bio) {
    if (!twt) return hipErrorInvalidValue;
    const int B = 1 << (lgTz + lgTx);
    dim3 grid((unsigned)(((Kx + (1 << lgTx) - 1) >> lgTx) * ((nz + (1 << lgTz) - 1) >> lgTz) * C * bio.count));
    const size_t lds = (size_t)B * p2_slab_elems(P) * sizeof(cx<T>) + p2_twiddle_lds_bytes(P, sizeof(cx<T>));
#define CALLS(PP, SS) \
    if (hipError_t e_ = allow_lds(&ky_inv<T, PP, SS>, lds)) return e_; \
    hipLaunchKernelGGL((ky_inv<T, PP, SS>), grid, dim3(B * tpp<PP>()), lds, st, in, out, ny, nz, Kx, lgTz, lgTx, kXcds, \
                       twt, bio)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    DEMAG_P2_SWITCH(P, CALL)
#undef CALL
#undef CALLS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_z_conv_p2(int lgTx, int rows, int sched, hipStream_t st, cx<T>* B2, const T* nhat, T Ms, int nz,
                            int Py, int Kx, int P, const cx<T>* twt, const BatchIO& bio) {
    if (!twt) return hipErrorInvalidValue;
    if (!p2_z_supported(P, sizeof(cx<T>)) || (rows != 1 && rows != 2)) return hipErrorInvalidValue;
    if (rows != (2 * p2_threads_per_pencil(P) <= kP2MaxThreadsZ ? 2 : 1)) return hipErrorInvalidValue;
    const int G = rows << lgTx;
    dim3 grid((unsigned)(Kx * ((rows == 2 ? Py / 2 + (1 << lgTx) : Py + (1 << lgTx) - 1) >> lgTx) * bio.count));
    const size_t lds = p2_z_lds_bytes(P, rows, lgTx, sizeof(cx<T>));
#define CALLS(PP, SS) \
    if (bio.in) { /* a batch group: its members re-read one tensor spectrum from the caches */ \
        if (hipError_t e_ = allow_lds(&kz_conv<T, PP, SS>, lds)) return e_; \
        hipLaunchKernelGGL((kz_conv<T, PP, SS>), grid, dim3(G * tpp<PP>()), lds, st, B2, nhat, Ms, nz, Py, Kx, lgTx, \
                           rows, kXcds, twt, bio); \
    } else { \
        if (hipError_t e_ = allow_lds(&kz_conv<T, PP, SS, false, true>, lds)) return e_; \
        hipLaunchKernelGGL((kz_conv<T, PP, SS, false, true>), grid, dim3(G * tpp<PP>()), lds, st, B2, nhat, Ms, nz, Py, \
                           Kx, lgTx, rows, kXcds, twt, bio); \
    }
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    if constexpr (sizeof(T) == 4) {
        DEMAG_P2_SWITCH(P, CALL)
    } else {  // FP64 lengths 3 * 2^a would not fit the registers: generic kernels
        switch (P) {
            DEMAG_P2_CASES_POW2(CALL)
        default: return hipErrorInvalidValue;
        }
    }
#undef CALL
#undef CALLS
    return hipGetLastError();
}

// The fused Z pass's forward half with the energy's quadratic form in place of
// the product and the inverse transforms: one FP64 partial per workgroup into
// epart (*nparts of them; B2 is only read).
template <typename T>
hipError_t launch_z_energy_p2(int lgTx, int rows, int sched, hipStream_t st, cx<T>* B2, const T* nhat, int nz, int Py,
                              int Kx, int P, const cx<T>* twt, double* epart, int* nparts) {
    if (!twt || !epart || !nparts) return hipErrorInvalidValue;
    if (!p2_z_supported(P, sizeof(cx<T>)) || (rows != 1 && rows != 2)) return hipErrorInvalidValue;
    if (rows != (2 * p2_threads_per_pencil(P) <= kP2MaxThreadsZ ? 2 : 1)) return hipErrorInvalidValue;
    const int G = rows << lgTx;
    dim3 grid((unsigned)(Kx * ((rows == 2 ? Py / 2 + (1 << lgTx) : Py + (1 << lgTx) - 1) >> lgTx)));
    *nparts = (int)grid.x;
    // the slabs (P values per pencil) hold the reduction's one double per thread
    const size_t lds = p2_z_lds_bytes(P, rows, lgTx, sizeof(cx<T>));
    const BatchIO none;
#define CALLS(PP, SS) \
    if (hipError_t e_ = allow_lds(&kz_conv<T, PP, SS, true, true>, lds)) return e_; \
    hipLaunchKernelGGL((kz_conv<T, PP, SS, true, true>), grid, dim3(G * tpp<PP>()), lds, st, B2, nhat, T(1), nz, Py, Kx, \
                       lgTx, rows, kXcds, twt, none, epart)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    if constexpr (sizeof(T) == 4) {
        DEMAG_P2_SWITCH(P, CALL)
    } else {
        switch (P) {
            DEMAG_P2_CASES_POW2(CALL)
        default: return hipErrorInvalidValue;
        }
    }
#undef CALL
#undef CALLS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_z_sp_p2(int lgTx, int rows, int sched, hipStream_t st, cx<T>* B2, const T* shat, T Ms, int nz,
                          int Py, int Kx, int P, const cx<T>* twt) {
    if (!twt) return hipErrorInvalidValue;
    if (!p2_z_supported(P, sizeof(cx<T>)) || (rows != 1 && rows != 2)) return hipErrorInvalidValue;
    const int G = rows << lgTx;
    dim3 grid((unsigned)(Kx * ((rows == 2 ? Py / 2 + (1 << lgTx) : Py + (1 << lgTx) - 1) >> lgTx)));
    // slabs, twiddles and the staged kernel rows (fewer bytes than kz_conv's tensor rows)
    const size_t lds = p2_z_lds_bytes(P, rows, lgTx, sizeof(cx<T>));
#define CALLS(PP, SS) \
    if (hipError_t e_ = allow_lds(&kz_sp<T, PP, SS>, lds)) return e_; \
    hipLaunchKernelGGL((kz_sp<T, PP, SS>), grid, dim3(G * tpp<PP>()), lds, st, B2, shat, Ms, nz, Py, Kx, lgTx, rows, \
                       kXcds, twt)
#define CALL(PP) DEMAG_P2_SCHED(PP, CALLS)
    if constexpr (sizeof(T) == 4) {
        DEMAG_P2_SWITCH(P, CALL)
    } else {
        switch (P) {
            DEMAG_P2_CASES_POW2(CALL)
        default: return hipErrorInvalidValue;
        }
    }
#undef CALL
#undef CALLS
    return hipGetLastError();
}

// The table of length P and schedule S (nothing for a schedule the length has not).
template <typename T, int P, int S>
void fill_table(const std::vector<cx<T>>& tw, std::vector<cx<T>>& out) {
    if constexpr (S == 0 || (p2::is_pow2(P) && S < p2::num_schedules(P))) {
        using LT = p2::Len<P, S>;
        out.resize(LT::table_size());
        LT::fill(tw.data(), out.data());
    }
}

template <typename T>
std::vector<cx<T>> p2_thread_twiddles(int P, int sched, const std::vector<cx<T>>& tw) {
    std::vector<cx<T>> out;
    if ((int)tw.size() != P || sched < 0 || sched >= p2_num_schedules(P)) return out;
    switch (P) {
#define FILL(PP)                                                         \
    case PP:                                                             \
        if (sched == 0) fill_table<T, PP, 0>(tw, out);                   \
        else if (sched == 1) fill_table<T, PP, 1>(tw, out);              \
        else fill_table<T, PP, 2>(tw, out);                              \
        break;
        FILL(2) FILL(4) FILL(8) FILL(16) FILL(32) FILL(64) FILL(128) FILL(256) FILL(512) FILL(1024) FILL(2048) FILL(4096)
        FILL(6) FILL(12) FILL(24) FILL(48) FILL(96) FILL(192) FILL(384) FILL(768) FILL(1536) FILL(3072)
#undef FILL
    default: break;
    }
    return out;
}

#define DEMAG_P2_INSTANTIATE(T)                                                                                    \
    template hipError_t launch_x_fwd_p2<T>(int, int, hipStream_t, const T*, cx<T>*, int, int, int, int, int,      \
                                           const cx<T>*, const BatchIO&);                                          \
    template hipError_t launch_x_inv_p2<T>(int, int, hipStream_t, const cx<T>*, T*, const T*, double*, int, int,  \
                                           int, int, int, int, const cx<T>*, const BatchIO&);                      \
    template hipError_t launch_y_fwd_p2<T>(int, int, int, hipStream_t, const cx<T>*, cx<T>*, int, int, int, int, \
                                           int, const cx<T>*, const BatchIO&);                                     \
    template hipError_t launch_y_inv_p2<T>(int, int, int, hipStream_t, const cx<T>*, cx<T>*, int, int, int, int, \
                                           int, const cx<T>*, const BatchIO&);                                     \
    template hipError_t launch_z_conv_p2<T>(int, int, int, hipStream_t, cx<T>*, const T*, T, int, int, int, int,  \
                                            const cx<T>*, const BatchIO&);                                         \
    template hipError_t launch_z_sp_p2<T>(int, int, int, hipStream_t, cx<T>*, const T*, T, int, int, int, int,    \
                                          const cx<T>*);                                                           \
    template hipError_t launch_z_energy_p2<T>(int, int, int, hipStream_t, cx<T>*, const T*, int, int, int, int,     \
                                              const cx<T>*, double*, int*);

DEMAG_P2_INSTANTIATE(float)
DEMAG_P2_INSTANTIATE(double)
template std::vector<cx<float>> p2_thread_twiddles<float>(int, int, const std::vector<cx<float>>&);
template std::vector<cx<double>> p2_thread_twiddles<double>(int, int, const std::vector<cx<double>>&);

}  // namespace demag
