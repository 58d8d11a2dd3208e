// Register-resident FFT of compile-time power-of-two length P (gfx950).
//
// A pencil of P complex values is held by TP = P / EPT threads, EPT = 8
// values per thread (EPT = P for P < 8).  The transform is a Stockham
// sequence of radix-8, -4 and -2 stages in one of a few radix schedules (see
// Fft); each stage works on registers, and consecutive stages exchange data through
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

// Radix schedules of a power-of-two length P = 8^N8 r (r = 1, 2 or 4).  Stage
// 0 is always radix 8 (it spans the thread's eight slots; the zero-skip of a
// padded input reads half of them), and every schedule has the same number of
// stages, i.e. of LDS exchanges:
//   S = 0: 8, 8, ..., 8, r         (the remaining factor last)
//   S = 1: 8, r, 8, ..., 8         (N8 >= 2, r > 1: the remaining factor second)
//   S = 2: 8, ..., 8, 4, 4         (N8 >= 2, r = 2: the last 8 x 2 as 4 x 4)
// They differ in the twiddles a thread holds per stage and in the butterflies'
// arithmetic and register use; the autotuner chooses one per axis.
__host__ __device__ constexpr int num_schedules(int P) {
    const int L2 = ilog2(P), N8 = L2 / 3, r = 1 << (L2 % 3);
    return 1 + (N8 >= 2 && r > 1 ? 1 : 0) + (N8 >= 2 && r == 2 ? 1 : 0);
}
// Radix of stage s of schedule S (stages: N8, plus one when r > 1).
__host__ __device__ constexpr int schedule_radix(int P, int S, int s) {
    const int L2 = ilog2(P), N8 = L2 / 3, r = 1 << (L2 % 3);
    return S == 0 ? (s < N8 ? 8 : r) : S == 1 ? (s == 1 ? r : 8) : (s < N8 - 1 ? 8 : 4);
}
__host__ __device__ constexpr int schedule_stages(int P) {
    return ilog2(P) / 3 + ((ilog2(P) % 3) ? 1 : 0);
}

template <int P, int S = 0>
struct Fft {
    static_assert(P >= 2 && (P & (P - 1)) == 0, "power-of-two length");
    static_assert(S >= 0 && S < num_schedules(P), "radix schedule of this length");
    static constexpr int L2 = ilog2(P);
    static constexpr int N8 = L2 / 3;
    static constexpr int RLAST = 1 << (L2 % 3);  // 1, 2 or 4
    static constexpr int NST = N8 + (RLAST > 1 ? 1 : 0);
    static constexpr int EPT = P >= 8 ? 8 : P;
    static constexpr int TP = P / EPT;
    static constexpr int LOG_TP = ilog2(TP);
    __host__ __device__ static constexpr int radix(int s) { return schedule_radix(P, S, s); }
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
template <int P, typename T, int SCH = 0>
struct Twiddles {
    cx<T> w[Fft<P, SCH>::NST > 1 ? Fft<P, SCH>::NST : 1][7];

    __device__ __forceinline__ void load(int t, const cx<T>* __restrict__ twt) { load_from<1>(t, twt); }

    template <int S>
    __device__ __forceinline__ void load_from(int t, const cx<T>* __restrict__ twt) {
        using F = Fft<P, SCH>;
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
template <int P, int SCH = 0>
struct TwiddleTable {
    using F = Fft<P, SCH>;
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
template <int P, int SCH, int S, int DIR, bool LO, typename T>
__device__ __forceinline__ void stage_compute(cx<T>* v, const Twiddles<P, T, SCH>& tws) {
    using F = Fft<P, SCH>;
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
template <int P, int SCH, int S, int DIR, bool LO, typename T>
__device__ __forceinline__ void stages_from(cx<T>* v, cx<T>* slab, int t, const Twiddles<P, T, SCH>& tws) {
    using F = Fft<P, SCH>;
    stage_compute<P, SCH, S, DIR, LO>(v, tws);
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
        stages_from<P, SCH, S + 1, DIR, LO>(v, slab, t, tws);
    }
}

// Full transform.  Every thread of the workgroup must call it (for TP > 64 it
// contains workgroup barriers).  The slab belongs to this pencil alone; the
// caller orders any access by other threads (a workgroup barrier) before.
// LO = true: input positions >= P/2 are zero (zero-padded data) and the slots
// holding them are not read.
template <int P, int DIR, bool LO = false, typename T, int SCH>
__device__ __forceinline__ void fft(cx<T>* v, cx<T>* slab, int t, const Twiddles<P, T, SCH>& tws) {
    stages_from<P, SCH, 0, DIR, LO>(v, slab, t, tws);
}

// ---------------------------------------------------------------------------
// Length traits over the lengths the register transforms handle: P = 2^a and
// P = 3 Q with Q = 2^a (a >= 1).  The pass kernels are written against these:
//   EPT, TP, LOG_TP, PS, pad()     registers per thread, threads per pencil,
//                                  LDS slab stride of one pencil of length P
//   fin_k(j)   forward input slot j holds position  t + fin_k(j) TP
//   iout_k(j)  inverse output slot j holds position t + iout_k(j) TP
//   fout(t,j)  frequency held by forward output slot j
//   iin(t,j)   frequency the inverse input slot j must hold
//   fout_slab / iin_slab   their padded LDS positions
//   fwd_slot_of_iin(j)     forward output slot with the frequency of inverse
//                          input slot j (register hand-over in the Z pass)
//   Tw<T>      one thread's twiddles (load from the thread-major table)
//   fft<DIR, LO>(v, slab, t, tw)
// In both cases positions >= P/2 are exactly the slots with fin_k or iout_k
// >= EPT/2 (zero-skip of the forward input, pruning of the inverse output).
constexpr bool is_pow2(int v) { return v >= 1 && (v & (v - 1)) == 0; }
constexpr bool reg_length(int P) { return P >= 2 && (is_pow2(P) || (P % 3 == 0 && P >= 6 && is_pow2(P / 3))); }

template <int P, int S = 0, bool POW2 = is_pow2(P)>
struct Len;

template <int P, int S>
struct Len<P, S, true> {
    using F = Fft<P, S>;
    static constexpr int EPT = F::EPT, TP = F::TP, LOG_TP = F::LOG_TP, PS = F::PS;
    __host__ __device__ static constexpr int pad(int i) { return F::pad(i); }
    __host__ __device__ static constexpr int pad_add(int pt, int a, int c) { return F::pad_add(pt, a, c); }
    __host__ __device__ static constexpr int fin_k(int j) { return F::slot_in(j); }
    __host__ __device__ static constexpr int iout_k(int j) { return F::slot_out(j); }
    __device__ static int fout(int t, int j) { return t + F::slot_out(j) * TP; }
    __device__ static int iin(int t, int j) { return t + F::slot_in(j) * TP; }
    __device__ static int fout_slab(int pt, int t, int j) { return F::pad_add(pt, t, F::slot_out(j) * TP); }
    __device__ static int iin_slab(int pt, int t, int j) { return F::pad_add(pt, t, F::slot_in(j) * TP); }
    __host__ __device__ static constexpr int fwd_slot_of_iin(int j) {
        for (int jj = 0; jj < EPT; ++jj)
            if (F::slot_out(jj) == F::slot_in(j)) return jj;
        return -1;
    }
    template <typename T>
    using Tw = Twiddles<P, T, S>;
    template <int DIR, bool LO, typename T>
    __device__ static void fft(cx<T>* v, cx<T>* slab, int t, const Tw<T>& tw) {
        p2::fft<P, DIR, LO>(v, slab, t, tw);
    }
    // the same with the twiddles read from the table `src` when needed
    template <int DIR, bool LO, typename T>
    __device__ static void fft_src(cx<T>* v, cx<T>* slab, int t, const cx<T>* __restrict__ src) {
        Tw<T> tw;
        tw.load(t, src);
        p2::fft<P, DIR, LO>(v, slab, t, tw);
    }
    static constexpr int table_size() { return TwiddleTable<P, S>::table_size(); }
    template <typename T>
    static void fill(const cx<T>* tw, cx<T>* twt) {
        TwiddleTable<P, S>::fill(tw, twt);
    }
};

// P = 3 Q.  Position n = n1 + Q n2 (n1 < Q, n2 < 3), frequency k = 3 k1 + k2.
// Forward: a radix-3 DFT over n2 for every n1, the twiddle W_P^(n1 k2), then
// one Q-point transform per k2 (its output k1 is frequency 3 k1 + k2).
// Inverse: the Q-point transforms first, the conjugate twiddle, then the
// radix-3 DFT, whose output n2 is position n1 + Q n2.  Thread t keeps the
// three Q-transforms' slots side by side: slot j = g EPTQ + jj, g = n2 (input
// side) or k2 (frequency side).  The Q-transforms use the pencil's slab in
// turn.  Twiddle table: the Q-transform's, then W_P^(m (t + k TPQ)) for m = 1,
// 2 and k < EPTQ, thread-major.
template <int P, int S>
struct Len<P, S, false> {
    static_assert(P % 3 == 0 && is_pow2(P / 3) && P >= 6, "length 3 * 2^a");
    static_assert(S == 0, "lengths 3 * 2^a have one schedule");
    static constexpr int Q = P / 3;
    using FQ = Fft<Q>;
    static constexpr int EQ = FQ::EPT;
    static constexpr int EPT = 3 * EQ, TP = FQ::TP, LOG_TP = FQ::LOG_TP;
    __host__ __device__ static constexpr int pad(int i) { return i + (i >> 3); }
    __host__ __device__ static constexpr int pad_add(int pt, int a, int c) { return FQ::pad_add(pt, a, c); }
    static constexpr int PS = pad(P) + 1;
    __host__ __device__ static constexpr int fin_k(int j) { return FQ::slot_in(j % EQ) + (j / EQ) * EQ; }
    __host__ __device__ static constexpr int iout_k(int j) { return FQ::slot_out(j % EQ) + (j / EQ) * EQ; }
    __device__ static int fout(int t, int j) { return 3 * (t + FQ::slot_out(j % EQ) * TP) + j / EQ; }
    __device__ static int iin(int t, int j) { return 3 * (t + FQ::slot_in(j % EQ) * TP) + j / EQ; }
    __device__ static int fout_slab(int, int t, int j) { return pad(fout(t, j)); }
    __device__ static int iin_slab(int, int t, int j) { return pad(iin(t, j)); }
    __host__ __device__ static constexpr int fwd_slot_of_iin(int j) {
        for (int jj = 0; jj < EQ; ++jj)
            if (FQ::slot_out(jj) == FQ::slot_in(j % EQ)) return (j / EQ) * EQ + jj;
        return -1;
    }
    template <typename T>
    struct Tw {
        Twiddles<Q, T> q;
        cx<T> w3[2][EQ];  // W_P^(m (t + k TP)), m = 1, 2
        __device__ __forceinline__ void load(int t, const cx<T>* __restrict__ twt) {
            q.load(t, twt);
            constexpr int TSQ = TwiddleTable<Q>::table_size();
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int k = 0; k < EQ; ++k) w3[m][k] = twt[TSQ + (m * EQ + k) * TP + t];
        }
    };
    template <int DIR, bool LO, typename T>
    __device__ static void fft(cx<T>* v, cx<T>* slab, int t, const Tw<T>& tw) {
        if constexpr (DIR < 0) {
#pragma unroll
            for (int jj = 0; jj < EQ; ++jj) {
                const int k = FQ::slot_in(jj);  // n1 = t + k TP
                cx<T> y[3] = {v[jj], v[EQ + jj], v[2 * EQ + jj]};
                // LO: positions >= P/2 are zero, i.e. n2 = 2 always and n2 = 1 for n1 >= Q/2
                if constexpr (LO) {
                    if (k >= EQ / 2) {  // a compile-time constant after unrolling
                        y[1] = y[0];
                        y[2] = y[0];
                    } else {
                        dft3_lo<DIR>(y);
                    }
                } else {
                    dft3<DIR>(y);
                }
                v[jj] = y[0];
                v[EQ + jj] = mul(y[1], tw.w3[0][k]);
                v[2 * EQ + jj] = mul(y[2], tw.w3[1][k]);
            }
#pragma unroll
            for (int g = 0; g < 3; ++g) p2::fft<Q, DIR, false>(v + g * EQ, slab, t, tw.q);
        } else {
#pragma unroll
            for (int g = 0; g < 3; ++g) p2::fft<Q, DIR, false>(v + g * EQ, slab, t, tw.q);
#pragma unroll
            for (int jj = 0; jj < EQ; ++jj) {
                const int k = FQ::slot_out(jj);  // n1 = t + k TP
                cx<T> y[3] = {v[jj], mul(v[EQ + jj], conj_(tw.w3[0][k])), mul(v[2 * EQ + jj], conj_(tw.w3[1][k]))};
                dft3<DIR>(y);
                v[jj] = y[0];
                v[EQ + jj] = y[1];
                v[2 * EQ + jj] = y[2];
            }
        }
    }
    // The same with the twiddles read from the table `src` when needed: the
    // radix-3 twiddles of one slot right before its radix-3 DFT, the
    // Q-transforms' right before them (fewer live registers).
    template <int DIR, bool LO, typename T>
    __device__ static void fft_src(cx<T>* v, cx<T>* slab, int t, const cx<T>* __restrict__ src) {
        constexpr int TSQ = TwiddleTable<Q>::table_size();
        if constexpr (DIR < 0) {
#pragma unroll
            for (int jj = 0; jj < EQ; ++jj) {
                const int k = FQ::slot_in(jj);
                cx<T> y[3] = {v[jj], v[EQ + jj], v[2 * EQ + jj]};
                if constexpr (LO) {
                    if (k >= EQ / 2) {  // a compile-time constant after unrolling
                        y[1] = y[0];
                        y[2] = y[0];
                    } else {
                        dft3_lo<DIR>(y);
                    }
                } else {
                    dft3<DIR>(y);
                }
                v[jj] = y[0];
                v[EQ + jj] = mul(y[1], src[TSQ + k * TP + t]);
                v[2 * EQ + jj] = mul(y[2], src[TSQ + (EQ + k) * TP + t]);
            }
            Twiddles<Q, T> q;
            q.load(t, src);
#pragma unroll
            for (int g = 0; g < 3; ++g) p2::fft<Q, DIR, false>(v + g * EQ, slab, t, q);
        } else {
            {
                Twiddles<Q, T> q;
                q.load(t, src);
#pragma unroll
                for (int g = 0; g < 3; ++g) p2::fft<Q, DIR, false>(v + g * EQ, slab, t, q);
            }
#pragma unroll
            for (int jj = 0; jj < EQ; ++jj) {
                const int k = FQ::slot_out(jj);
                cx<T> y[3] = {v[jj], mul(v[EQ + jj], conj_(src[TSQ + k * TP + t])),
                              mul(v[2 * EQ + jj], conj_(src[TSQ + (EQ + k) * TP + t]))};
                dft3<DIR>(y);
                v[jj] = y[0];
                v[EQ + jj] = y[1];
                v[2 * EQ + jj] = y[2];
            }
        }
    }
    static constexpr int table_size() { return TwiddleTable<Q>::table_size() + 2 * Q; }
    template <typename T>
    static void fill(const cx<T>* tw, cx<T>* twt) {
        cx<T> twq[Q];  // exp(-2 pi i t / Q) = tw[3 t]
        for (int i = 0; i < Q; ++i) twq[i] = tw[3 * i];
        TwiddleTable<Q>::fill(twq, twt);
        constexpr int TSQ = TwiddleTable<Q>::table_size();
        for (int m = 0; m < 2; ++m)
            for (int k = 0; k < EQ; ++k)
                for (int t = 0; t < TP; ++t) twt[TSQ + (m * EQ + k) * TP + t] = tw[((m + 1) * (t + k * TP)) % P];
    }
};

}  // namespace p2
}  // namespace demag
