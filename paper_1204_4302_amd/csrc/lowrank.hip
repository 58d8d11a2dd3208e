// Tensor-grid method on low-rank magnetization (Sec. 3.2, "Low-Rank
// Magnetization"; Tables 1 and 2, TG Tucker / TG CP rows; Appendix, eqs. (CP),
// (tucker)).
//
// Each component M_p of the magnetization (p = x, y, z) is given in Tucker
// format, M_p = C_p x_1 U_1^p x_2 U_2^p x_3 U_3^p (core r x r x r, factors
// n_q x r), or in CP format, M_p = sum_s lambda_p(s) u_1s^p o u_2s^p o u_3s^p
// (a Tucker tensor with a superdiagonal core).  Inserting this into the
// block-CP sum of eq. (sumpot) moves every Gaussian matrix onto a factor:
//
//     Phi = sum_p sum_l alpha c_l  C_p x_1 F_1^{pl} x_2 F_2^{pl} x_3 F_3^{pl},
//     F_q^{pl} = D_q^{l,p} U_q^p                       (n_q x r)
//
// (D_q^{l,p} the odd Gaussian matrix of node l when q = p, else the even one;
// c_l the Sinc weight; alpha = Ms h_max, lengths in units of h_max), i.e. the
// potential is again a block-CP tensor whose factors cost R n_q^2 r each, and
// no dense tensor is formed.  A difference operator along axis a acts on the
// mode-a factor only, so the field component H_a = -d_a Phi is the same sum
// with F_a replaced by G_a^{pl} = -delta_a F_a^{pl}.
//
// The factor product is a dense contraction: in FP32 it runs on MFMA
// (v_mfma_f32_16x16x4f32) over Gaussian matrices stored in the instruction's
// operand order, one launch for all axes, nodes and components, and the field
// factors follow from a small difference kernel; in FP64 the difference rows
// are folded into the matrices at set-up ([D; -delta D] stacked) and a VALU
// kernel produces both factors from one pass over the matrices.
//
// The energy -mu0/2 Ms V sum_a <M_a, H_a> is a sum of inner products of
// Tucker (CP) tensors, taken on the factors: with the r x r Gram matrices
// Gamma_q = (U_q^a)^T X_q (X_q = G_q or F_q),
//     <C x_q U_q, C' x_q X_q> = sum_{s,s'} C(s) C'(s') prod_q Gamma_q(s_q, s'_q)
// (Tucker: r^4 per term; CP: r^2), so the energy is sub-linear in N too; the
// Gram matrices (27 R of them) and the contractions (9 R) are two launches.
//
// The dense field on the grid, when asked for, is one GEMM per component
// with K = 3 R r:  H_a(i1, (i2, i3)) = sum_{p,l,s1} A_1(i1, s1) W(s1, i2, i3),
// W = alpha c_l C_p x_2 A_2 x_3 A_3 formed per (p, l, i3) by a small kernel.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>

#include "blas.hpp"
#include "internal.hpp"
#include "tg_gauss.hpp"

namespace demag {

namespace {

// The stacked Gaussian matrices of the three axes (kernel argument).
template <typename T>
struct LrStacks {
    const T* E[3];
    const T* O[3];
};

// -d/dx of the values v(j) = f(j) along an axis of n cells at row j (spacing h):
// central inside, second-order one-sided on the two faces, first order for
// two cells, zero for one cell.
template <typename F>
__device__ double minus_diff(F f, int j, int n, double h) {
    if (n == 1) return 0.0;
    if (n == 2) return -(f(1) - f(0)) / h;
    if (j == 0) return -(-3.0 * f(0) + 4.0 * f(1) - f(2)) / (2.0 * h);
    if (j == n - 1) return -(3.0 * f(n - 1) - 4.0 * f(n - 2) + f(n - 3)) / (2.0 * h);
    return -(f(j + 1) - f(j - 1)) / (2.0 * h);
}

// Stacked Gaussian matrices of one axis (n cells, reduced edge d, physical
// edge h): for node l, S[l] is 2n x n column-major, rows [0, n) the Gaussian
// matrix D(i', i) (target i', source i), rows [n, 2n) its negative
// difference -delta D along i' with spacing h.  E: even, O: odd kind.
template <typename T>
__global__ void __launch_bounds__(256) k_lr_axis(int n, double d, double h, int R, const double* __restrict__ tau,
                                                 T* __restrict__ E, T* __restrict__ O) {
    const size_t per = (size_t)2 * n * n;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per * R) return;
    const int l = (int)(t / per);
    const size_t e = t - (size_t)l * per;
    const int row = (int)(e % (2 * n)), i = (int)(e / (2 * n));
    const double s = tau[l], c = (i + 0.5) * d;
    auto even = [&](int j) { return gauss_even((j + 0.5) * d, c, d, s); };
    auto odd = [&](int j) { return gauss_odd((j + 0.5) * d, c, d, s); };
    if (row < n) {
        E[t] = (T)even(row);
        O[t] = (T)odd(row);
    } else {
        E[t] = (T)minus_diff(even, row - n, n, h);
        O[t] = (T)minus_diff(odd, row - n, n, h);
    }
}

// Potential and field factors of all three components in one launch:
//     FG_q(:, (p R + l) r + s) = S_q^{l,p} U_q^p(:, s),
// S_q^{l,p} the stacked (2 n_q x n_q) even matrix for p != q, the odd one for
// p = q.  Each matrix element is read once and used for every column (p, s)
// of the thread's column group.  Grid: x = row tiles of the three axes one
// after another, y = node l, z = column group (COLS of the 3 r columns);
// one thread per stacked row; the factors staged in LDS by row chunks.
constexpr int kLrRows = 128;   // stacked rows (threads) per workgroup
constexpr int kLrChunk = 64;   // factor rows per staged chunk
// matrix columns loaded ahead of their products (64 resp. 32 loads in flight per thread)
template <typename T>
constexpr int lr_batch() { return sizeof(T) == 4 ? 32 : 16; }

template <typename T, int COLS>
__global__ void __launch_bounds__(kLrRows) k_lr_factors(int n1, int n2, int n3, int R, int r, LrStacks<T> S,
                                                        const T* __restrict__ U, T* __restrict__ FG) {
    __shared__ T Us[kLrChunk][COLS];
    const int t1 = (2 * n1 + kLrRows - 1) / kLrRows, t2 = (2 * n2 + kLrRows - 1) / kLrRows;
    const int bx = blockIdx.x, l = blockIdx.y, c0 = blockIdx.z * COLS;
    const int q = bx < t1 ? 0 : bx < t1 + t2 ? 1 : 2;
    const int tile = q == 0 ? bx : q == 1 ? bx - t1 : bx - t1 - t2;
    const int nq = q == 0 ? n1 : q == 1 ? n2 : n3;
    const size_t uoff = q == 0 ? 0 : q == 1 ? (size_t)3 * r * n1 : (size_t)3 * r * (n1 + n2);
    const size_t foff = q == 0 ? 0 : q == 1 ? (size_t)6 * R * r * n1 : (size_t)6 * R * r * (n1 + n2);
    const size_t ld = (size_t)2 * nq;
    const T* __restrict__ E = S.E[q] + (size_t)l * ld * nq;
    const T* __restrict__ O = S.O[q] + (size_t)l * ld * nq;
    const int row = tile * kLrRows + (int)threadIdx.x;
    const bool live = row < 2 * nq;
    const int ncol = 3 * r;
    bool odd[COLS];
#pragma unroll
    for (int k = 0; k < COLS; ++k) odd[k] = (c0 + k) / r == q;
    T acc[COLS];
#pragma unroll
    for (int k = 0; k < COLS; ++k) acc[k] = T(0);
    for (int j0 = 0; j0 < nq; j0 += kLrChunk) {
        const int rows = nq - j0 < kLrChunk ? nq - j0 : kLrChunk;
        __syncthreads();
        for (int v = threadIdx.x; v < kLrChunk * COLS; v += kLrRows) {
            const int jj = v % kLrChunk, k = v / kLrChunk, c = c0 + k;
            Us[jj][k] = (jj < rows && c < ncol) ? U[uoff + (size_t)(j0 + jj) + (size_t)c * nq] : T(0);
        }
        __syncthreads();
        if (live) {
            const T* e_col = E + row + (size_t)j0 * ld;
            const T* o_col = O + row + (size_t)j0 * ld;
            // JB columns of both matrices in flight before the products
            // (the staged factor rows past `rows` are zero)
            constexpr int JB = lr_batch<T>();
            for (int jb = 0; jb < rows; jb += JB) {
                T e[JB], o[JB];
#pragma unroll
                for (int u = 0; u < JB; ++u) {
                    const bool ok = jb + u < rows;
                    e[u] = ok ? e_col[(size_t)(jb + u) * ld] : T(0);
                    o[u] = ok ? o_col[(size_t)(jb + u) * ld] : T(0);
                }
#pragma unroll
                for (int u = 0; u < JB; ++u)
#pragma unroll
                    for (int k = 0; k < COLS; ++k) acc[k] += (odd[k] ? o[u] : e[u]) * Us[jb + u][k];
            }
        }
    }
    if (live) {
#pragma unroll
        for (int k = 0; k < COLS; ++k) {
            const int c = c0 + k;
            if (c < ncol) {
                const int pp = c / r, ss = c - pp * r;
                FG[foff + ((size_t)(pp * R + l) * r + ss) * ld + row] = acc[k];
            }
        }
    }
}

// ---- FP32: the factor product on MFMA ------------------------------------------
constexpr int kMfChunk = 128;  // factor rows staged per chunk (8 tiles of 16)
constexpr int kMfGroups = kMfChunk / 16;

// Tiles of 16 columns per row block in the swizzled layout: ceil(n / 16)
// rounded up to whole chunks (the padding is zero).
__host__ __device__ inline int lr_sw_cols(int n) {
    const int nb = (n + 15) / 16;
    return (nb + kMfGroups - 1) / kMfGroups * kMfGroups;
}

// Swizzled Gaussian matrices (FP32): per node l, for the 16 x 16 tile (row
// block rb, column group kg) of D, the 256 values in the operand order of
// v_mfma_f32_16x16x4f32 over four k-steps: entry ((rb nc + kg) 64 + lane) 4 + v
// = D(16 rb + lane % 16, 16 kg + 4 v + lane / 16), zero outside n x n
// (nb = ceil(n / 16) row blocks, nc = lr_sw_cols(n) column groups).  A wave
// then loads each 16 x 16 tile as one 1 KB run.
__global__ void __launch_bounds__(256) k_lr_axis_sw(int n, double d, int R, const double* __restrict__ tau,
                                                    float* __restrict__ E, float* __restrict__ O) {
    const int nb = (n + 15) / 16, nc = lr_sw_cols(n);
    const size_t per = (size_t)nb * nc * 256;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per * R) return;
    const int l = (int)(t / per);
    const size_t e = t - (size_t)l * per;
    const int v = (int)(e & 3), lane = (int)((e >> 2) & 63);
    const size_t blk = e >> 8;
    const int rb = (int)(blk / nc), kg = (int)(blk % nc);
    const int row = 16 * rb + (lane & 15), k = 16 * kg + 4 * v + (lane >> 4);
    float ev = 0.f, ov = 0.f;
    if (row < n && k < n) {
        const double s = tau[l];
        ev = (float)gauss_even((row + 0.5) * d, (k + 0.5) * d, d, s);
        ov = (float)gauss_odd((row + 0.5) * d, (k + 0.5) * d, d, s);
    }
    E[t] = ev;
    O[t] = ov;
}

struct LrSwizzled {
    const float* E[3];
    const float* O[3];
};

typedef float lr_f32x4 __attribute__((ext_vector_type(4)));

// F_q^{pl} for FP32 on MFMA.  Columns of axis q: even blocks of 16 hold the
// two components p != q (2r columns), odd blocks component q (r columns); a
// workgroup takes NE even and NO odd blocks (column group = grid z; blocks
// past the last are zero and not written) and 4 row blocks of 16 (one per
// wave; grid x over the three axes), node l = grid y.  Per 16 x 16 tile a
// wave issues four MFMAs per block (K = 4 each): A from the swizzled matrix
// (all tiles of a chunk in flight before the chunk's factor rows are staged),
// B from LDS.  Accumulator layout: lane holds rows 4 (lane / 16) + v, column
// lane % 16.  No control flow inside the product loop: idle waves compute on
// a valid tile and do not store.
template <int NE, int NO>
__global__ void __launch_bounds__(256) k_lr_factors_mfma(int n1, int n2, int n3, int R, int r, LrSwizzled S,
                                                         const float* __restrict__ U, float* __restrict__ FG) {
    constexpr int NB = NE + NO;
    __shared__ float Us[kMfChunk][NB * 16 + 1];
    const int nb1 = (n1 + 15) / 16, nb2 = (n2 + 15) / 16, nb3 = (n3 + 15) / 16;
    const int t1 = (nb1 + 3) / 4, t2 = (nb2 + 3) / 4;
    const int bx = blockIdx.x, l = blockIdx.y, z = blockIdx.z;
    const int q = bx < t1 ? 0 : bx < t1 + t2 ? 1 : 2;
    const int tile = q == 0 ? bx : q == 1 ? bx - t1 : bx - t1 - t2;
    const int n = q == 0 ? n1 : q == 1 ? n2 : n3;
    const int nb = q == 0 ? nb1 : q == 1 ? nb2 : nb3;
    const int nc = lr_sw_cols(n);
    const size_t uoff = q == 0 ? 0 : q == 1 ? (size_t)3 * r * n1 : (size_t)3 * r * (n1 + n2);
    const size_t foff = q == 0 ? 0 : q == 1 ? (size_t)6 * R * r * n1 : (size_t)6 * R * r * (n1 + n2);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int rb = tile * 4 + wave;
    const bool live = rb < nb;
    const int rbc = live ? rb : nb - 1;
    const size_t per = (size_t)nb * nc * 256;
    const float* Esw = S.E[q] + (size_t)l * per + (size_t)rbc * nc * 256 + lane * 4;
    const float* Osw = S.O[q] + (size_t)l * per + (size_t)rbc * nc * 256 + lane * 4;
    // (component, column) of block j, column c; -1 for padding
    auto col_of = [&](int j, int c, int& p) {
        if (j < NE) {
            const int cc = 16 * (z * NE + j) + c;
            if (cc >= 2 * r) return -1;
            const int i = cc / r;
            p = i < q ? i : i + 1;
            return cc - i * r;
        }
        const int cc = 16 * (z * NO + j - NE) + c;
        if (cc >= r) return -1;
        p = q;
        return cc;
    };
    lr_f32x4 acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = lr_f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nc * 16; k0 += kMfChunk) {
        lr_f32x4 aE[NE > 0 ? kMfGroups : 1], aO[NO > 0 ? kMfGroups : 1];
#pragma unroll
        for (int g = 0; g < kMfGroups; ++g) {
            const size_t off = (size_t)((k0 >> 4) + g) * 256;
            if constexpr (NE > 0) aE[g] = *(const lr_f32x4*)(Esw + off);
            if constexpr (NO > 0) aO[g] = *(const lr_f32x4*)(Osw + off);
        }
        // the chunk's factor rows: every load issued before the first LDS store
        constexpr int kPer = kMfChunk * NB * 16 / 256;
        float uv[kPer];
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = tid + 256 * e;
            const int kk = idx % kMfChunk, cl = idx / kMfChunk;
            int p = 0;
            const int s = col_of(cl >> 4, cl & 15, p);
            const int k = k0 + kk;
            uv[e] = (s >= 0 && k < n) ? U[uoff + (size_t)k + (size_t)n * (p * r + s)] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int idx = tid + 256 * e;
            Us[idx % kMfChunk][idx / kMfChunk] = uv[e];
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < kMfGroups; ++g) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk = 16 * g + 4 * v + (lane >> 4);
                float bv[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) bv[j] = Us[kk][16 * j + (lane & 15)];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    float a;
                    if constexpr (NE > 0) a = j < NE ? aE[g][v] : aO[NO > 0 ? g : 0][v];
                    else a = aO[g][v];
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[j], acc[j], 0, 0, 0);
                }
            }
        }
    }
    if (live) {
        const size_t ld = (size_t)2 * n;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            int p = 0;
            const int s = col_of(j, lane & 15, p);
            if (s >= 0) {
                float* col = FG + foff + ((size_t)(p * R + l) * r + s) * ld;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rb + 4 * (lane >> 4) + v;
                    if (row < n) col[row] = acc[j][v];
                }
            }
        }
    }
}

// Field factors from potential factors: G_q = -delta_q F_q (rows [n_q, 2 n_q)
// of every column of FG), the difference stencils of the field, FP64 arithmetic.
__global__ void __launch_bounds__(256) k_lr_grad(int n1, int n2, int n3, int R, int r, double h1, double h2,
                                                 double h3, float* __restrict__ FG) {
    const size_t cols = (size_t)3 * R * r;
    const size_t c1 = cols * n1, c2 = cols * n2, c3 = cols * n3;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= c1 + c2 + c3) return;
    int n;
    double h;
    size_t foff;
    if (t < c1) {
        n = n1, h = h1, foff = 0;
    } else if (t < c1 + c2) {
        t -= c1;
        n = n2, h = h2, foff = (size_t)6 * R * r * n1;
    } else {
        t -= c1 + c2;
        n = n3, h = h3, foff = (size_t)6 * R * r * (n1 + n2);
    }
    const size_t col = t / n;
    const int row = (int)(t - col * n);
    float* F = FG + foff + col * 2 * n;
    auto f = [&](int j) { return (double)F[j]; };
    F[n + row] = (float)minus_diff(f, row, n, h);
}

// Energy, step 1: the Gram matrices Gamma_q = (U_q^a)^T X_q (r x r, X_q the
// field factor G_q^{pl} when q = a, else the potential factor F_q^{pl}), one
// workgroup per (a, p, l, q), blockIdx.x = ((a * 3 + p) * R + l) * 3 + q.
// Rows are summed over chunks staged in LDS; when the r^2 entries are fewer
// than 256 the rows of a chunk are split over 256 / r^2 thread groups.
// gram[blockIdx.x][s + r s'] (FP64).
constexpr int kLrStage = 2048;  // staged values per operand (rows x r)

template <typename T>
__global__ void __launch_bounds__(256) k_lr_gram(int n1, int n2, int n3, int R, int r, const T* __restrict__ U,
                                                 const T* __restrict__ FG, double* __restrict__ gram) {
    extern __shared__ double lds[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int q = b % 3, l = (b / 3) % R, p = (b / (3 * R)) % 3, a = b / (9 * R);
    const int rr = r * r;
    const int nq = q == 0 ? n1 : q == 1 ? n2 : n3;
    const size_t uoff = q == 0 ? 0 : q == 1 ? (size_t)3 * r * n1 : (size_t)3 * r * (n1 + n2);
    const size_t foff = q == 0 ? 0 : q == 1 ? (size_t)6 * R * r * n1 : (size_t)6 * R * r * (n1 + n2);
    const T* Ua = U + uoff + (size_t)a * r * nq;                                   // n_q x r, ld n_q
    const T* X = FG + foff + (size_t)(p * R + l) * r * 2 * nq + (q == a ? nq : 0);  // n_q x r, ld 2 n_q
    const int CH = kLrStage / r;  // rows per chunk
    const int ldc = CH + 1;       // padded stride of a staged column
    double* Us = lds;
    double* Xs = lds + (size_t)ldc * r;
    double* out = gram + (size_t)b * rr;
    const int G = rr >= 256 ? 1 : 256 / rr;  // row groups when the entries are few
    const int e1 = tid % rr, g1 = tid / rr;
    double acc = 0.0;
    for (int e = tid; e < rr; e += blockDim.x) out[e] = 0.0;
    for (int i0 = 0; i0 < nq; i0 += CH) {
        const int rows = nq - i0 < CH ? nq - i0 : CH;
        __syncthreads();
        for (int j = tid; j < rows * r; j += blockDim.x) {
            const int i = j % rows, s = j / rows;
            Us[i + ldc * s] = (double)Ua[i0 + i + (size_t)s * nq];
            Xs[i + ldc * s] = (double)X[i0 + i + (size_t)s * 2 * nq];
        }
        __syncthreads();
        if (G > 1) {
            if (g1 < G) {
                const double* u = Us + ldc * (e1 % r);
                const double* x = Xs + ldc * (e1 / r);
                for (int i = g1; i < rows; i += G) acc += u[i] * x[i];
            }
        } else {
            for (int e = tid; e < rr; e += blockDim.x) {
                const double* u = Us + ldc * (e % r);
                const double* x = Xs + ldc * (e / r);
                double v = 0.0;
                for (int i = 0; i < rows; ++i) v += u[i] * x[i];
                out[e] += v;  // each entry owned by one thread
            }
        }
    }
    if (G > 1) {
        __syncthreads();
        if (g1 < G) lds[tid] = acc;  // staging is free: reuse it for the group sums
        __syncthreads();
        if (tid < rr) {
            double v = 0.0;
            for (int g = 0; g < G; ++g) v += lds[g * rr + tid];
            out[tid] = v;
        }
    }
}

// Energy, step 2: one workgroup per (a, p, l), blockIdx.x = (a * 3 + p) * R + l:
// partials[b] = alpha c_l sum_{s,s'} C_a(s) C_p(s') prod_q Gamma_q(s_q, s'_q)
// (Tucker: one mode at a time, r^4 per mode; CP: lambda_a(s) lambda_p(s')
// prod_q Gamma_q(s, s'), r^2).  LDS (doubles): Gram [3 r^2], Tucker buffers
// [2 r^3].
template <typename T, bool TUCKER>
__global__ void __launch_bounds__(256) k_lr_contract(int R, int r, const T* __restrict__ core,
                                                     const double* __restrict__ gram, const double* __restrict__ c,
                                                     double alpha, double* __restrict__ partials) {
    extern __shared__ double lds[];
    __shared__ double red[4];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int l = b % R, p = (b / R) % 3, a = b / (3 * R);
    const int rr = r * r;
    double* gam = lds;  // [q][s][s'] at q r^2 + s + r s'
    for (int e = tid; e < 3 * rr; e += blockDim.x) gam[e] = gram[(size_t)b * 3 * rr + e];
    double acc = 0.0;
    if constexpr (TUCKER) {
        const int r3 = rr * r;
        double* A = lds + 3 * rr;
        double* B = A + r3;
        const T* Ca = core + (size_t)a * r3;
        const T* Cp = core + (size_t)p * r3;
        for (int e = tid; e < r3; e += blockDim.x) A[e] = (double)Ca[e];
        __syncthreads();
        // B(s1', s2, s3) = sum_s1 Gamma_1(s1, s1') A(s1, s2, s3)
        for (int e = tid; e < r3; e += blockDim.x) {
            const int x = e % r, yz = e / r;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[k + r * x] * A[k + r * yz];
            B[e] = v;
        }
        __syncthreads();
        // A(s1', s2', s3) = sum_s2 Gamma_2(s2, s2') B(s1', s2, s3)
        for (int e = tid; e < r3; e += blockDim.x) {
            const int x = e % r, y = (e / r) % r, z = e / rr;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[rr + k + r * y] * B[x + r * k + rr * z];
            A[e] = v;
        }
        __syncthreads();
        // sum_{s'} C_p(s') sum_s3 Gamma_3(s3, s3') A(s1', s2', s3)
        for (int e = tid; e < r3; e += blockDim.x) {
            const int xy = e % rr, z = e / rr;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[2 * rr + k + r * z] * A[xy + rr * k];
            acc += v * (double)Cp[e];
        }
    } else {
        __syncthreads();
        const T* la = core + (size_t)a * r;
        const T* lp = core + (size_t)p * r;
        for (int e = tid; e < rr; e += blockDim.x) {
            const int s = e % r, sp = e / r;
            acc += (double)la[s] * (double)lp[sp] * gam[e] * gam[rr + e] * gam[2 * rr + e];
        }
    }
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int w = 0; w < nw; ++w) sum += red[w];
        partials[b] = alpha * c[l] * sum;
    }
}

// Right operand of the dense expansion of H_a over the z slices [k0, k0 + kc):
// Wt (n2 kc x 3 R r, column-major) with
//     Wt((i2, k), (p, l, s1)) = alpha c_l sum_{s2, s3} C_p(s1, s2, s3) A_2(i2, s2) A_3(k0 + k, s3)
// (CP: alpha c_l lambda_p(s1) A_2(i2, s1) A_3(k0 + k, s1)), A_q the field
// factor G_q when q = a, else F_q.  One workgroup per (p, l, k).
template <typename T, bool TUCKER>
__global__ void __launch_bounds__(256) k_lr_expand(int n1, int n2, int n3, int R, int r, int a, int k0, int kc,
                                                   const T* __restrict__ core, const T* __restrict__ FG,
                                                   const double* __restrict__ c, double alpha, T* __restrict__ Wt) {
    extern __shared__ double lds[];
    const int b = blockIdx.x;
    const int k = b % kc, pl = b / kc;
    const int p = pl / R, l = pl % R;
    const int rr = r * r;
    double* a3 = lds;      // r
    double* Z = lds + r;   // Tucker: r x r; CP: r
    const size_t f2off = (size_t)2 * n1 * 3 * R * r, f3off = f2off + (size_t)2 * n2 * 3 * R * r;
    const T* A2 = FG + f2off + (size_t)pl * r * 2 * n2 + (a == 1 ? n2 : 0);  // n2 x r, ld 2 n2
    const T* A3 = FG + f3off + (size_t)pl * r * 2 * n3 + (a == 2 ? n3 : 0);  // n3 x r, ld 2 n3
    const int i3 = k0 + k;
    for (int s = threadIdx.x; s < r; s += blockDim.x) a3[s] = (double)A3[i3 + (size_t)s * 2 * n3];
    __syncthreads();
    const double w = alpha * c[l];
    if constexpr (TUCKER) {
        const T* C = core + (size_t)p * rr * r;
        for (int e = threadIdx.x; e < rr; e += blockDim.x) {
            double v = 0.0;
            for (int s3 = 0; s3 < r; ++s3) v += (double)C[e + (size_t)rr * s3] * a3[s3];
            Z[e] = w * v;  // Z(s1, s2) at s1 + r s2
        }
    } else {
        for (int s = threadIdx.x; s < r; s += blockDim.x) Z[s] = w * (double)core[(size_t)p * r + s] * a3[s];
    }
    __syncthreads();
    const size_t ld = (size_t)n2 * kc;
    for (int e = threadIdx.x; e < r * n2; e += blockDim.x) {
        const int i2 = e % n2, s1 = e / n2;
        double v;
        if constexpr (TUCKER) {
            v = 0.0;
            for (int s2 = 0; s2 < r; ++s2) v += Z[s1 + r * s2] * (double)A2[i2 + (size_t)s2 * 2 * n2];
        } else {
            v = Z[s1] * (double)A2[i2 + (size_t)s1 * 2 * n2];
        }
        Wt[(size_t)i2 + (size_t)n2 * k + ld * ((size_t)pl * r + s1)] = (T)v;
    }
}

}  // namespace

template <typename T>
hipError_t launch_lr_axis(hipStream_t st, int n, double d, double h, int R, const double* tau, T* E, T* O) {
    const size_t total = (size_t)2 * n * n * R;
    hipLaunchKernelGGL((k_lr_axis<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, d, h, R, tau, E, O);
    return hipGetLastError();
}

hipError_t launch_lr_axis_sw(hipStream_t st, int n, double d, int R, const double* tau, float* E, float* O) {
    const size_t total = lr_swizzled_elems(n) * R;
    hipLaunchKernelGGL(k_lr_axis_sw, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, d, R, tau, E, O);
    return hipGetLastError();
}

size_t lr_swizzled_elems(int n) {
    return (size_t)((n + 15) / 16) * lr_sw_cols(n) * 256;
}

size_t lr_gram_lds_bytes(int r) {
    return sizeof(double) * std::max<size_t>(2 * (size_t)(kLrStage / r + 1) * r, 256);
}

size_t lr_contract_lds_bytes(int r, bool tucker) {
    const size_t rr = (size_t)r * r;
    return sizeof(double) * (3 * rr + (tucker ? 2 * rr * r : 0));
}

// The low-rank evaluation: factors (9 GEMMs), then optionally the energy from
// the factors and the dense field.  DE[q], DO[q]: stacked Gaussian matrices
// of axis q ([R][n_q][2 n_q] column-major, ld 2 n_q).
template <typename T>
int lr_evaluate(void* handle, hipStream_t st, const int n[3], const double h[3], int R, int r, bool tucker,
                const T* core, const T* U, const T* const DE[3], const T* const DO[3], const double* c, double alpha,
                T* FG, double* partials, double* gram, T* H, T* W, size_t w_elems) {
    rocblas_handle hd = (rocblas_handle)handle;
    if (rocblas_set_stream(hd, st) != rocblas_status_success) return -1;
    const T one = 1, zero = 0;
    if constexpr (sizeof(T) == 4) {  // FP32: swizzled matrices, MFMA, then the differences
        LrSwizzled S;
        for (int q = 0; q < 3; ++q) {
            S.E[q] = (const float*)DE[q];
            S.O[q] = (const float*)DO[q];
        }
        const int tiles = ((n[0] + 15) / 16 + 3) / 4 + ((n[1] + 15) / 16 + 3) / 4 + ((n[2] + 15) / 16 + 3) / 4;
        const int nbE = (2 * r + 15) / 16, nbO = (r + 15) / 16;
        if (r <= 8) {
            hipLaunchKernelGGL((k_lr_factors_mfma<1, 1>), dim3(tiles, R, 1), dim3(256), 0, st, n[0], n[1], n[2], R, r,
                               S, (const float*)U, (float*)FG);
        } else {
            const int groups = std::max((nbE + 1) / 2, nbO);
            hipLaunchKernelGGL((k_lr_factors_mfma<2, 1>), dim3(tiles, R, groups), dim3(256), 0, st, n[0], n[1], n[2],
                               R, r, S, (const float*)U, (float*)FG);
        }
        if (hipGetLastError() != hipSuccess) return -2;
        const size_t total = (size_t)3 * R * r * (n[0] + n[1] + n[2]);
        hipLaunchKernelGGL(k_lr_grad, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n[0], n[1], n[2], R, r,
                           h[0], h[1], h[2], (float*)FG);
        if (hipGetLastError() != hipSuccess) return -2;
    } else {
        LrStacks<T> S;
        for (int q = 0; q < 3; ++q) {
            S.E[q] = DE[q];
            S.O[q] = DO[q];
        }
        const int tiles = (2 * n[0] + kLrRows - 1) / kLrRows + (2 * n[1] + kLrRows - 1) / kLrRows +
                          (2 * n[2] + kLrRows - 1) / kLrRows;
        if (3 * r <= 24)
            hipLaunchKernelGGL((k_lr_factors<T, 24>), dim3(tiles, R, 1), dim3(kLrRows), 0, st, n[0], n[1], n[2], R, r,
                               S, U, FG);
        else
            hipLaunchKernelGGL((k_lr_factors<T, 48>), dim3(tiles, R, (3 * r + 47) / 48), dim3(kLrRows), 0, st, n[0],
                               n[1], n[2], R, r, S, U, FG);
        if (hipGetLastError() != hipSuccess) return -2;
    }
    if (partials) {
        // partials doubles as [9 R] energy terms; the Gram matrices go to gram
        const size_t lg = lr_gram_lds_bytes(r), lc = lr_contract_lds_bytes(r, tucker);
        hipLaunchKernelGGL((k_lr_gram<T>), dim3(27 * R), dim3(256), lg, st, n[0], n[1], n[2], R, r, U, FG, gram);
        if (hipGetLastError() != hipSuccess) return -3;
        if (lc > 65536) {  // dynamic LDS above 64 KB must be allowed per kernel
            const void* kern = tucker ? (const void*)k_lr_contract<T, true> : (const void*)k_lr_contract<T, false>;
            if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lc) != hipSuccess)
                return -6;
        }
        if (tucker)
            hipLaunchKernelGGL((k_lr_contract<T, true>), dim3(9 * R), dim3(256), lc, st, R, r, core, gram, c, alpha,
                               partials);
        else
            hipLaunchKernelGGL((k_lr_contract<T, false>), dim3(9 * R), dim3(256), lc, st, R, r, core, gram, c, alpha,
                               partials);
        if (hipGetLastError() != hipSuccess) return -3;
    }
    if (H) {
        const int n1 = n[0], n2 = n[1], n3 = n[2];
        const int K = 3 * R * r;
        const size_t N = (size_t)n1 * n2 * n3;
        const int kc = (int)std::max<size_t>(1, std::min<size_t>(n3, w_elems / ((size_t)K * n2)));
        const size_t lds = sizeof(double) * (size_t)(r + (tucker ? r * r : r));
        for (int a = 0; a < 3; ++a) {
            const T* A1 = FG + (a == 0 ? n1 : 0);  // n1 x K, ld 2 n1
            for (int k0 = 0; k0 < n3; k0 += kc) {
                const int kk = std::min(kc, n3 - k0);
                const dim3 grid((unsigned)(3 * R * kk));
                if (tucker)
                    hipLaunchKernelGGL((k_lr_expand<T, true>), grid, dim3(256), lds, st, n1, n2, n3, R, r, a, k0, kk,
                                       core, FG, c, alpha, W);
                else
                    hipLaunchKernelGGL((k_lr_expand<T, false>), grid, dim3(256), lds, st, n1, n2, n3, R, r, a, k0, kk,
                                       core, FG, c, alpha, W);
                if (hipGetLastError() != hipSuccess) return -4;
                // H_a(:, slices k0..) (n1 x n2 kk) = A1 (n1 x K) Wt^T (Wt: n2 kk x K)
                if (gemm(hd, rocblas_operation_none, rocblas_operation_transpose, n1, n2 * kk, K, &one, A1, 2 * n1, W,
                         n2 * kk, &zero, H + (size_t)a * N + (size_t)k0 * n1 * n2, n1) != rocblas_status_success)
                    return -5;
            }
        }
    }
    return 0;
}

template hipError_t launch_lr_axis<float>(hipStream_t, int, double, double, int, const double*, float*, float*);
template hipError_t launch_lr_axis<double>(hipStream_t, int, double, double, int, const double*, double*, double*);
template int lr_evaluate<float>(void*, hipStream_t, const int[3], const double[3], int, int, bool, const float*,
                                const float*, const float* const[3], const float* const[3], const double*, double,
                                float*, double*, double*, float*, float*, size_t);
template int lr_evaluate<double>(void*, hipStream_t, const int[3], const double[3], int, int, bool, const double*,
                                 const double*, const double* const[3], const double* const[3], const double*, double,
                                 double*, double*, double*, double*, double*, size_t);

}  // namespace demag
