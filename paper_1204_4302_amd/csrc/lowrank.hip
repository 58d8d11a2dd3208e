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
// with F_a replaced by G_a^{pl} = -delta_a F_a^{pl}; the difference matrices
// are folded into the Gaussian matrices at set-up ([D; -delta D] stacked), so
// one GEMM per (axis, component) gives both factors for all nodes.
//
// The energy -mu0/2 Ms V sum_a <M_a, H_a> is a sum of inner products of
// Tucker (CP) tensors, taken on the factors: with the r x r Gram matrices
// Gamma_q = (U_q^a)^T X_q (X_q = G_q or F_q),
//     <C x_q U_q, C' x_q X_q> = sum_{s,s'} C(s) C'(s') prod_q Gamma_q(s_q, s'_q)
// (Tucker: r^4 per term; CP: r^2), so the energy is sub-linear in N too.
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

// Energy terms: one workgroup per (a, p, l), blockIdx.x = (a * 3 + p) * R + l.
// partials[b] = alpha c_l <M_a, term (p, l) of H_a>, evaluated on the factors.
// LDS (doubles): three r x r Gram matrices, then two r^3 buffers (Tucker).
template <typename T, bool TUCKER>
__global__ void __launch_bounds__(256) k_lr_energy(int n1, int n2, int n3, int R, int r, const T* __restrict__ core,
                                                   const T* __restrict__ U, const T* __restrict__ FG,
                                                   const double* __restrict__ c, double alpha,
                                                   double* __restrict__ partials) {
    extern __shared__ double lds[];
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int l = b % R, p = (b / R) % 3, a = b / (3 * R);
    const int rr = r * r;
    double* gam = lds;  // [q][s][s'] at q r^2 + s + r s'
    const int n[3] = {n1, n2, n3};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // Gram matrices: one wave per dot product, lanes over the rows
    size_t uoff = 0, foff = 0;
    for (int q = 0; q < 3; ++q) {
        const int nq = n[q];
        const T* Ua = U + uoff + (size_t)a * r * nq;                                   // n_q x r, ld n_q
        const T* X = FG + foff + (size_t)(p * R + l) * r * 2 * nq + (q == a ? nq : 0);  // n_q x r, ld 2 n_q
        for (int e = wave; e < rr; e += nw) {
            const int s = e % r, sp = e / r;
            double acc = 0.0;
            for (int i = lane; i < nq; i += 64) acc += (double)Ua[i + (size_t)s * nq] * (double)X[i + (size_t)sp * 2 * nq];
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
            if (lane == 0) gam[q * rr + e] = acc;
        }
        uoff += (size_t)3 * r * nq;
        foff += (size_t)2 * nq * 3 * R * r;
    }
    __syncthreads();
    double acc = 0.0;
    if constexpr (TUCKER) {
        const int r3 = rr * r;
        double* A = lds + 3 * rr;
        double* B = A + r3;
        const T* Ca = core + (size_t)a * r3;
        const T* Cp = core + (size_t)p * r3;
        for (int e = threadIdx.x; e < r3; e += blockDim.x) A[e] = (double)Ca[e];
        __syncthreads();
        // B(s1', s2, s3) = sum_s1 Gamma_1(s1, s1') A(s1, s2, s3)
        for (int e = threadIdx.x; e < r3; e += blockDim.x) {
            const int x = e % r, yz = e / r;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[k + r * x] * A[k + r * yz];
            B[e] = v;
        }
        __syncthreads();
        // A(s1', s2', s3) = sum_s2 Gamma_2(s2, s2') B(s1', s2, s3)
        for (int e = threadIdx.x; e < r3; e += blockDim.x) {
            const int x = e % r, y = (e / r) % r, z = e / rr;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[rr + k + r * y] * B[x + r * k + rr * z];
            A[e] = v;
        }
        __syncthreads();
        // sum_{s'} C_p(s') sum_s3 Gamma_3(s3, s3') A(s1', s2', s3)
        for (int e = threadIdx.x; e < r3; e += blockDim.x) {
            const int xy = e % rr, z = e / rr;
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += gam[2 * rr + k + r * z] * A[xy + rr * k];
            acc += v * (double)Cp[e];
        }
    } else {
        const T* la = core + (size_t)a * r;
        const T* lp = core + (size_t)p * r;
        for (int e = threadIdx.x; e < rr; e += blockDim.x) {
            const int s = e % r, sp = e / r;
            acc += (double)la[s] * (double)lp[sp] * gam[e] * gam[rr + e] * gam[2 * rr + e];
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w];
        partials[b] = alpha * c[l] * s;
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

size_t lr_energy_lds_bytes(int r, bool tucker) {
    const size_t rr = (size_t)r * r;
    return sizeof(double) * (3 * rr + (tucker ? 2 * rr * r : 0));
}

// The low-rank evaluation: factors (9 GEMMs), then optionally the energy from
// the factors and the dense field.  DE[q], DO[q]: stacked Gaussian matrices
// of axis q ([R][n_q][2 n_q] column-major, ld 2 n_q).
template <typename T>
int lr_evaluate(void* handle, hipStream_t st, const int n[3], int R, int r, bool tucker, const T* core, const T* U,
                const T* const DE[3], const T* const DO[3], const double* c, double alpha, T* FG, double* partials,
                T* H, T* W, size_t w_elems) {
    rocblas_handle hd = (rocblas_handle)handle;
    if (rocblas_set_stream(hd, st) != rocblas_status_success) return -1;
    const T one = 1, zero = 0;
    size_t uoff = 0, foff = 0;
    for (int q = 0; q < 3; ++q) {
        const int nq = n[q];
        for (int p = 0; p < 3; ++p) {
            // [F; G] (2 n_q x r) for every node l = stacked D (2 n_q x n_q) U_q^p (n_q x r)
            const T* S = p == q ? DO[q] : DE[q];
            if (gemm_sb(hd, rocblas_operation_none, rocblas_operation_none, 2 * nq, r, nq, &one, S, 2 * nq,
                        (rocblas_stride)2 * nq * nq, U + uoff + (size_t)p * r * nq, nq, 0, &zero,
                        FG + foff + (size_t)p * R * r * 2 * nq, 2 * nq, (rocblas_stride)r * 2 * nq,
                        R) != rocblas_status_success)
                return -2;
        }
        uoff += (size_t)3 * r * nq;
        foff += (size_t)2 * nq * 3 * R * r;
    }
    if (partials) {
        const size_t lds = lr_energy_lds_bytes(r, tucker);
        if (lds > 65536) {  // dynamic LDS above 64 KB must be allowed per kernel
            const void* kern = tucker ? (const void*)k_lr_energy<T, true> : (const void*)k_lr_energy<T, false>;
            if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                return -6;
        }
        if (tucker)
            hipLaunchKernelGGL((k_lr_energy<T, true>), dim3(9 * R), dim3(256), lds, st, n[0], n[1], n[2], R, r, core,
                               U, FG, c, alpha, partials);
        else
            hipLaunchKernelGGL((k_lr_energy<T, false>), dim3(9 * R), dim3(256), lds, st, n[0], n[1], n[2], R, r, core,
                               U, FG, c, alpha, partials);
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
template int lr_evaluate<float>(void*, hipStream_t, const int[3], int, int, bool, const float*, const float*,
                                const float* const[3], const float* const[3], const double*, double, float*, double*,
                                float*, float*, size_t);
template int lr_evaluate<double>(void*, hipStream_t, const int[3], int, int, bool, const double*, const double*,
                                 const double* const[3], const double* const[3], const double*, double, double*,
                                 double*, double*, double*, size_t);

}  // namespace demag
