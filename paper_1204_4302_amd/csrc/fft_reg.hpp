// Register-resident FFT of compile-time power-of-two length P (gfx950).
//
// A pencil of P complex values is held by TP = P / EPT threads, EPT = 8
// values per thread (EPT = P for P < 8).  The transform is a Stockham
// sequence of radix-8 stages followed by at most one radix-2 or radix-4 stage;
// each stage works on registers, and consecutive stages exchange data through
// the pencil's LDS slab (for pencils of up to 64 threads, i.e. P <= 512,
// within one wavefront and without workgroup barriers).  LDS positions are padded
// with one slot per eight (pad(i) = i + i/8) so that the strided writes of the
// first stages do not collide on banks; slabs are PS = pad(P) + 1 apart (odd in
// 8-byte units) so that reads across pencils at one position do not collide
// either.  All index arithmetic is on compile-time powers of two (shifts and
// masks).  Twiddles are the generic engine's values, tw[t] = exp(-2 pi i t / P)
// rounded once from long double, rearranged thread-major (see Twiddles).
//
// Register slot j of thread t:
//   before the first stage it must hold input element  in_pos(t, j),
//   after the last stage it holds output element       out_pos(t, j).
// Both position sets equal { t + k TP : k = 0..EPT-1 }; slot_in(j), slot_out(j)
// give k.  For P >= 8, positions < P/2 are exactly the slots with k < EPT/2,
// which is what the zero-skip (forward) and pruning (inverse) use.
#pragma once
#include "fft_lds.hpp"

namespace demag {
namespace p2 {

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

template <int P>
struct Fft {
    static_assert(P >= 2 && (P & (P - 1)) == 0, "power-of-two length");
    static constexpr int L2 = ilog2(P);
    static constexpr int N8 = L2 / 3;
    static constexpr int RLAST = 1 << (L2 % 3);  // 1, 2 or 4
    static constexpr int NST = N8 + (RLAST > 1 ? 1 : 0);
    static constexpr int EPT = P >= 8 ? 8 : P;
    static constexpr int TP = P / EPT;
    static constexpr int LOG_TP = ilog2(TP);
    __host__ __device__ static constexpr int radix(int s) { return s < N8 ? 8 : RLAST; }
    __host__ __device__ static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * radix(s - 1); }
    __host__ __device__ static constexpr int pad(int i) { return i + (i >> 3); }
    // pad(a + c) from pt = pad(a): exact when c is a multiple of 8, or when a
    // is and 0 <= c < 8 (no carry out of the low three bits); c is a
    // compile-time constant after unrolling, so the test folds away.
    __host__ __device__ static constexpr int pad_add(int pt, int a, int c) {
        return (c & 7) == 0 ? pt + c + (c >> 3) : pad(a + c);
    }
    static constexpr int PS = pad(P) + 1;  // LDS slab stride of one pencil (elements)
    // slot j = i * R + r of a radix-R stage holds element t + i TP + r (P/R)
    __host__ __device__ static constexpr int slot_k(int j, int R) { return j / R + (j % R) * (EPT / R); }
    __host__ __device__ static constexpr int slot_in(int j) { return slot_k(j, radix(0)); }
    __host__ __device__ static constexpr int slot_out(int j) { return slot_k(j, radix(NST - 1)); }
};

// Make one pencil's LDS writes visible to its own threads.  A pencil of
// TP <= 64 threads lies inside one wavefront (TP divides 64 and pencils start
// at multiples of TP), whose LDS instructions execute in program order, so a
// wavefront-scope fence (a compiler barrier for memory operations) suffices;
// longer pencils span several wavefronts and need the workgroup barrier.
template <int TP>
__device__ __forceinline__ void pencil_sync() {
    if constexpr (TP <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// The twiddles one thread applies, per stage S >= 1: entry [S][e], e =
// i (R-1) + r-1, is tw[r k P/(NS R)] for its butterfly i (k = butterfly index
// mod NS).  They depend on the thread only, so a thread that runs several
// transforms loads them once; the inverse uses their conjugates.  They are
// read from a thread-major table, twt[((S-1) 7 + e) TP + t] (thread_twiddle
// below), so that the threads of a pencil load consecutive addresses.
template <int P, typename T>
struct Twiddles {
    cx<T> w[Fft<P>::NST > 1 ? Fft<P>::NST : 1][7];

    __device__ __forceinline__ void load(int t, const cx<T>* __restrict__ twt) { load_from<1>(t, twt); }

    template <int S>
    __device__ __forceinline__ void load_from(int t, const cx<T>* __restrict__ twt) {
        using F = Fft<P>;
        if constexpr (S < F::NST) {
            constexpr int R = F::radix(S), NB = F::EPT / R;
#pragma unroll
            for (int e = 0; e < NB * (R - 1); ++e) w[S][e] = twt[((S - 1) * 7 + e) * F::TP + t];
            load_from<S + 1>(t, twt);
        }
    }
};

// Table position of entry [S][e] of thread t, and the index into tw[] it
// holds; table_size() entries in all.  Host-side builder of the table.
template <int P>
struct TwiddleTable {
    using F = Fft<P>;
    static constexpr int table_size() { return (F::NST > 1 ? F::NST - 1 : 1) * 7 * F::TP; }
    template <typename T>
    static void fill(const cx<T>* tw, cx<T>* twt) {
        for (int i = 0; i < table_size(); ++i) twt[i] = tw[0];
        for (int S = 1; S < F::NST; ++S) {
            const int R = F::radix(S), NS = F::ns(S), NB = F::EPT / R;
            for (int t = 0; t < F::TP; ++t)
                for (int i = 0; i < NB; ++i) {
                    const int k = (t + i * F::TP) & (NS - 1);
                    for (int r = 1; r < R; ++r)
                        twt[((S - 1) * 7 + i * (R - 1) + r - 1) * F::TP + t] = tw[r * k * (P / (NS * R))];
                }
        }
    }
};

// LO: the transform's upper half of inputs (positions >= P/2, i.e. slots
// j >= EPT/2 of the first stage, whose radix equals EPT) is zero and unread.
template <int P, int S, int DIR, bool LO, typename T>
__device__ __forceinline__ void stage_compute(cx<T>* v, const Twiddles<P, T>& tws) {
    using F = Fft<P>;
    constexpr int R = F::radix(S), NS = F::ns(S), NB = F::EPT / R;
    if constexpr (S == 0 && LO) {
        static_assert(NB == 1 && NS == 1, "first stage spans the thread's slots");
        dftR_lo<R, DIR>(v);
        return;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tws.w[S][i * (R - 1) + r - 1];
                if (DIR > 0) w.im = -w.im;
                v[i * R + r] = mul(v[i * R + r], w);
            }
        }
        dftR<R, DIR>(v + i * R);
    }
}

// Stage S and every later one.  Caller: slots hold stage-S inputs.
template <int P, int S, int DIR, bool LO, typename T>
__device__ __forceinline__ void stages_from(cx<T>* v, cx<T>* slab, int t, const Twiddles<P, T>& tws) {
    using F = Fft<P>;
    stage_compute<P, S, DIR, LO>(v, tws);
    if constexpr (S + 1 < F::NST) {
        constexpr int R = F::radix(S), NS = F::ns(S), NB = F::EPT / R;
        // every thread of the pencil has consumed the slab's previous contents
        // (automatic inside one wavefront, which executes in lockstep)
        pencil_sync<F::TP>();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int b = t + i * F::TP;
            const int k = b & (NS - 1);
            // base = (b - k) R + k is a multiple of 8 when NS = 1 (R = 8 there),
            // and r NS is one when NS >= 8: pad(base + r NS) = pad(base) + r NS (9/8)
            const int pb = F::pad((b - k) * R + k);
#pragma unroll
            for (int r = 0; r < R; ++r) slab[pb + r * NS + ((r * NS) >> 3)] = v[i * R + r];
        }
        pencil_sync<F::TP>();
        constexpr int R2 = F::radix(S + 1), NB2 = F::EPT / R2;
        const int pt = F::pad(t);
#pragma unroll
        for (int i = 0; i < NB2; ++i)
#pragma unroll
            for (int r = 0; r < R2; ++r) v[i * R2 + r] = slab[F::pad_add(pt, t, i * F::TP + r * (P / R2))];
        stages_from<P, S + 1, DIR, LO>(v, slab, t, tws);
    }
}

// Full transform.  Every thread of the workgroup must call it (for TP > 64 it
// contains workgroup barriers).  The slab belongs to this pencil alone; the
// caller orders any access by other threads (a workgroup barrier) before.
// LO = true: input positions >= P/2 are zero (zero-padded data) and the slots
// holding them are not read.
template <int P, int DIR, bool LO = false, typename T>
__device__ __forceinline__ void fft(cx<T>* v, cx<T>* slab, int t, const Twiddles<P, T>& tws) {
    stages_from<P, 0, DIR, LO>(v, slab, t, tws);
}

template <int P, int DIR, bool LO = false, typename T>
__device__ __forceinline__ void fft(cx<T>* v, cx<T>* slab, int t, const cx<T>* __restrict__ twt) {
    Twiddles<P, T> tws;
    tws.load(t, twt);
    stages_from<P, 0, DIR, LO>(v, slab, t, tws);
}

}  // namespace p2
}  // namespace demag
