// LDS-resident batched complex FFT for gfx950 (device code only).
//
// A workgroup holds B pencils of length P (complex, real type T = float or
// double) in LDS, pencil b at offset b * PS.  The transform runs as a
// Stockham auto-sort sequence of radix-R stages (R in {2,3,4,5,8}); each
// stage reads R values per butterfly into registers, barriers, twiddles,
// applies the radix-R DFT and writes back in place.  Output is in natural
// order.  Twiddles come from a table tw[t] = exp(-2 pi i t / P), built in FP64
// on the host and rounded once to T; no recurrences and no fast-math sin/cos.
//
// Forward: X_k = sum_j x_j exp(-2 pi i jk/P).  Inverse: the + sign, no 1/P.
#pragma once
#include <hip/hip_runtime.h>

namespace demag {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { cx<T> c; c.re = r; c.im = i; return c; }
template <typename T>
__device__ __forceinline__ cx<T> add(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> sub(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> mul(cx<T> a, cx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cx<T> conj_(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
// multiply by -i (forward, DIR = -1) or +i (inverse, DIR = +1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
    return DIR < 0 ? mk(a.im, -a.re) : mk(-a.im, a.re);
}

// ---- radix-R DFTs in registers (sign of the exponent = DIR) -------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = add(a, b);
    v[1] = sub(a, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
    cx<T> t0 = add(v[0], v[2]), t1 = sub(v[0], v[2]);
    cx<T> t2 = add(v[1], v[3]), t3 = rot90<DIR>(sub(v[1], v[3]));
    v[0] = add(t0, t2);
    v[2] = sub(t0, t2);
    v[1] = add(t1, t3);
    v[3] = sub(t1, t3);
}

// The same DFTs when the upper half of the inputs is known to be zero (the
// first stage of a transform of zero-padded data): v[R/2..R-1] are not read.
template <int DIR, typename T>
__device__ __forceinline__ void dft2_lo(cx<T>* v) {
    v[1] = v[0];
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4_lo(cx<T>* v) {
    const cx<T> a = v[0], b = v[1], rb = rot90<DIR>(b);
    v[0] = add(a, b);
    v[2] = sub(a, b);
    v[1] = add(a, rb);
    v[3] = sub(a, rb);
}

template <int DIR, typename T, bool LO = false>
__device__ __forceinline__ void dft8(cx<T>* v) {
    const T h = T(0.70710678118654752440084436210484903928);
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    if constexpr (LO) {
        dft4_lo<DIR>(e);
        dft4_lo<DIR>(o);
    } else {
        dft4<DIR>(e);
        dft4<DIR>(o);
    }
    // o[k] *= exp(DIR * 2 pi i k / 8)
    o[1] = DIR < 0 ? mk(h * (o[1].re + o[1].im), h * (o[1].im - o[1].re))
                   : mk(h * (o[1].re - o[1].im), h * (o[1].im + o[1].re));
    o[2] = rot90<DIR>(o[2]);
    o[3] = DIR < 0 ? mk(h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im))
                   : mk(-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im));
    for (int k = 0; k < 4; ++k) {
        v[k] = add(e[k], o[k]);
        v[k + 4] = sub(e[k], o[k]);
    }
}

// radix-3 DFT of (v[0], v[1], 0): v[2] is not read
template <int DIR, typename T>
__device__ __forceinline__ void dft3_lo(cx<T>* v) {
    const T s = T(0.86602540378443864676372317075293618347);  // sin(2 pi / 3)
    const cx<T> a = v[0], b = v[1];
    const cx<T> m = mk(a.re - T(0.5) * b.re, a.im - T(0.5) * b.im);
    const cx<T> r = rot90<DIR>(scale(b, s));
    v[0] = add(a, b);
    v[1] = add(m, r);
    v[2] = sub(m, r);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cx<T>* v) {
    const T s = T(0.86602540378443864676372317075293618347);  // sin(2 pi / 3)
    cx<T> t1 = add(v[1], v[2]), t2 = sub(v[1], v[2]);
    cx<T> m = mk(v[0].re - T(0.5) * t1.re, v[0].im - T(0.5) * t1.im);
    cx<T> r = rot90<DIR>(scale(t2, s));  // DIR * i * s * t2
    v[0] = add(v[0], t1);
    v[1] = add(m, r);
    v[2] = sub(m, r);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft5(cx<T>* v) {
    const T c1 = T(0.30901699437494742410229341718281905886);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410229341718281905886);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357211643933337938214340);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312916870595463907276860);   // sin(4 pi/5)
    cx<T> b1 = add(v[1], v[4]), d1 = sub(v[1], v[4]);
    cx<T> b2 = add(v[2], v[3]), d2 = sub(v[2], v[3]);
    cx<T> a0 = v[0];
    cx<T> p1 = mk(a0.re + c1 * b1.re + c2 * b2.re, a0.im + c1 * b1.im + c2 * b2.im);
    cx<T> p2 = mk(a0.re + c2 * b1.re + c1 * b2.re, a0.im + c2 * b1.im + c1 * b2.im);
    cx<T> q1 = rot90<DIR>(mk(s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im));
    cx<T> q2 = rot90<DIR>(mk(s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im));
    v[0] = add(a0, add(b1, b2));
    v[1] = add(p1, q1);
    v[4] = sub(p1, q1);
    v[2] = add(p2, q2);
    v[3] = sub(p2, q2);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(cx<T>* v) {
    if constexpr (R == 2) dft2<DIR>(v);
    else if constexpr (R == 3) dft3<DIR>(v);
    else if constexpr (R == 4) dft4<DIR>(v);
    else if constexpr (R == 5) dft5<DIR>(v);
    else dft8<DIR>(v);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR_lo(cx<T>* v) {
    static_assert(R == 2 || R == 4 || R == 8, "power-of-two radix");
    if constexpr (R == 2) dft2_lo<DIR>(v);
    else if constexpr (R == 4) dft4_lo<DIR>(v);
    else dft8<DIR, T, true>(v);
}

// Stage schedule of one transform length: radices in execution order.
struct FftPlanDev {
    int P;          // transform length
    int nstages;
    int radix[16];
};

// One Stockham stage over B pencils (pencil stride PS) held in LDS.
// E is the compile-time bound on elements per thread: B * P <= nthr * E.
template <int R, int DIR, int E, typename T>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int B, int PS, int P, int Ns,
                                          const cx<T>* __restrict__ tw) {
    constexpr int MAXB = (E + R - 1) / R;
    const int nthr = blockDim.x;
    const int tid = threadIdx.x;
    const int PR = P / R;
    const int total = B * PR;
    const int twstep = P / (Ns * R);
    cx<T> v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        int u = tid + i * nthr;
        if (u < total) {
            int b = u / PR, j = u - b * PR;
            const cx<T>* src = buf + b * PS + j;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = src[r * PR];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        int u = tid + i * nthr;
        if (u < total) {
            int b = u / PR, j = u - b * PR;
            int k = j % Ns;
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = tw[r * k * twstep];
                    if (DIR > 0) w.im = -w.im;
                    v[i][r] = mul(v[i][r], w);
                }
            }
            dftR<R, DIR>(v[i]);
            cx<T>* dst = buf + b * PS + (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r * Ns] = v[i][r];
        }
    }
    __syncthreads();
}

// Full transform of B pencils in LDS.  Must be called by every thread of the
// workgroup (it contains barriers); the caller barriers before the call.
template <int DIR, int E, typename T>
__device__ void fft_lds(cx<T>* buf, int B, int PS, const FftPlanDev& pl,
                        const cx<T>* __restrict__ tw) {
    int Ns = 1;
    for (int s = 0; s < pl.nstages; ++s) {
        const int R = pl.radix[s];
        switch (R) {
        case 8: fft_stage<8, DIR, E>(buf, B, PS, pl.P, Ns, tw); break;
        case 4: fft_stage<4, DIR, E>(buf, B, PS, pl.P, Ns, tw); break;
        case 2: fft_stage<2, DIR, E>(buf, B, PS, pl.P, Ns, tw); break;
        case 3: fft_stage<3, DIR, E>(buf, B, PS, pl.P, Ns, tw); break;
        default: fft_stage<5, DIR, E>(buf, B, PS, pl.P, Ns, tw); break;
        }
        Ns *= R;
    }
}

}  // namespace demag
