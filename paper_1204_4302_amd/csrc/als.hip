// Alternating least squares compression of a dense magnetization into the
// low-rank formats of the tensor-grid method (Sec. 3.2 "Low-Rank
// Magnetization", where the CP and Tucker approximations are computed by ALS
// from random initial guesses; Appendix eqs. (CP), (tucker)).  Each component
// X (n1 x n2 x n3, x fastest) is compressed on its own, from the caller's
// initial factors, for a fixed number of sweeps over the three modes.
//
// Tucker (higher-order orthogonal iteration), mode n of a sweep:
//     Y = X x_{m != n} U_m^T,   U_n <- orth(Y_(n) (Y_(n)^T U_n)),
// i.e. the leading r-dimensional left singular subspace of Y_(n) by one step
// of orthogonal iteration from the current U_n (orth: Gram-Schmidt twice,
// dependent columns completed by unit vectors);
// after the sweeps C = X x_1 U1^T x_2 U2^T x_3 U3^T.
// CP (CP-ALS), mode n of a sweep (b, c the other two modes):
//     U_n <- X_(n) (U_c (.) U_b) V^-1,   V = (U_b^T U_b) * (U_c^T U_c),
//     lambda <- column 2-norms of U_n,   U_n <- U_n / lambda.
// The contractions with the dense component are GEMMs / GEMVs (rocBLAS); the
// r x r algebra (Gram matrices, Cholesky, triangular inverse, Hadamard
// product, normalisation) is FP64 in small kernels of this file.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>

#include "blas.hpp"
#include "internal.hpp"

namespace demag {

namespace {

// Dependence threshold of the orthonormalisation (relative to the largest
// column norm of the orthogonal-iteration product, whose columns scale with
// the squared singular values).
constexpr double kAlsTolF64 = 1e-13;
constexpr double kAlsTolF32 = 1e-6;

// G[s + r s'] = sum_i A(i, s) B(i, s') (FP64); one wave per entry, lanes over
// the rows; four entries per workgroup.
template <typename T>
__global__ void __launch_bounds__(256) k_als_gram(int n, int r, const T* __restrict__ A, int lda,
                                                  const T* __restrict__ B, int ldb, double* __restrict__ G) {
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= r * r) return;
    const int s = e % r, sp = e / r;
    const T* a = A + (size_t)s * lda;
    const T* b = B + (size_t)sp * ldb;
    double acc = 0.0;
    for (int i = lane; i < n; i += 64) acc += (double)a[i] * (double)b[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) G[e] = acc;
}

// From the SPD matrix V = G1 (* G2 elementwise, when G2 is given): its
// Cholesky factor V = R^T R (R upper), X = R^-1, and
//   mode 0: out = X          (orthonormalising factor of Cholesky QR)
//   mode 1: out = X X^T = V^-1.
// out is r x r column-major in T.  A pivot not above 1e-14 of its diagonal
// entry (not positive definite to working accuracy) sets *flag.
// One workgroup; LDS 2 r^2 doubles.
template <typename T>
__global__ void __launch_bounds__(256) k_als_chol_inv(int r, const double* __restrict__ G1,
                                                      const double* __restrict__ G2, int mode, T* __restrict__ out,
                                                      int* __restrict__ flag) {
    extern __shared__ double lds[];
    double* R = lds;           // R[i + r j] = R(i, j), row i, column j
    double* X = lds + r * r;   // X[i + r j]
    const int tid = threadIdx.x;
    for (int e = tid; e < r * r; e += blockDim.x) R[e] = G2 ? G1[e] * G2[e] : G1[e];  // symmetric
    __syncthreads();
    __shared__ int bad;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        if (tid == 0) {
            double d = R[j + r * j];
            const double diag = d;
            for (int k = 0; k < j; ++k) d -= R[k + r * j] * R[k + r * j];
            if (!(d > 1e-14 * diag)) {
                bad = 1;
                d = diag > 0 ? diag : 1.0;  // keep going with finite values; the caller reports the failure
            }
            R[j + r * j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < r; i += blockDim.x) {
            double v = R[j + r * i];  // V(j, i), still unmodified in the upper part
            for (int k = 0; k < j; ++k) v -= R[k + r * j] * R[k + r * i];
            R[j + r * i] = v / R[j + r * j];
        }
        __syncthreads();
    }
    // X = R^-1 (upper): column c by back substitution
    for (int c = tid; c < r; c += blockDim.x) {
        for (int i = r - 1; i >= 0; --i) {
            double v;
            if (i > c) {
                v = 0.0;
            } else {
                v = i == c ? 1.0 : 0.0;
                for (int k = i + 1; k <= c; ++k) v -= R[i + r * k] * X[k + r * c];
                v /= R[i + r * i];
            }
            X[i + r * c] = v;
        }
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += blockDim.x) {
        const int a = e % r, b = e / r;
        if (mode == 0) {
            out[e] = (T)X[e];
        } else {
            double v = 0.0;
            for (int k = 0; k < r; ++k) v += X[a + r * k] * X[b + r * k];
            out[e] = (T)v;
        }
    }
    if (tid == 0 && bad) flag[0] = 1;
}

// Block-wide FP64 sum over the workgroup (256 threads); every thread gets it.
__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    __syncthreads();  // red may still be read from the previous call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// Q (n x r) = orthonormal basis of range(P) (n x r, both ld n) by modified
// Gram-Schmidt applied twice per column.  A column whose remainder is not
// above tol times the largest column norm of P is numerically dependent; it
// is replaced by the unit vector e_i with the largest remainder (the first
// such i), orthogonalised the same way, so Q is always orthonormal (a rank
// deficient Y_(n), e.g. a state invariant along an axis, gets an arbitrary
// completion carrying no weight).  For full-rank P, Q is the Q of the QR
// decomposition with diag(R) > 0.  One workgroup of 256 threads; the column
// being built in LDS (n doubles).
template <typename T>
__global__ void __launch_bounds__(256) k_als_orth(int n, int r, const T* __restrict__ P, T* __restrict__ Q, double tol) {
    extern __shared__ double v[];
    __shared__ double red[4];
    __shared__ double best_val;
    __shared__ int best_idx;
    const int tid = threadIdx.x;
    double pmax = 0.0;
    for (int j = 0; j < r; ++j) {
        double a = 0.0;
        for (int i = tid; i < n; i += blockDim.x) a += (double)P[i + (size_t)j * n] * (double)P[i + (size_t)j * n];
        pmax = fmax(pmax, sqrt(block_sum(a, red)));
    }
    for (int j = 0; j < r; ++j) {
        for (int i = tid; i < n; i += blockDim.x) v[i] = (double)P[i + (size_t)j * n];
        for (int attempt = 0; attempt < 2; ++attempt) {
            for (int pass = 0; pass < 2; ++pass)
                for (int k = 0; k < j; ++k) {
                    const T* q = Q + (size_t)k * n;
                    double a = 0.0;
                    __syncthreads();  // v complete
                    for (int i = tid; i < n; i += blockDim.x) a += (double)q[i] * v[i];
                    const double c = block_sum(a, red);
                    for (int i = tid; i < n; i += blockDim.x) v[i] -= c * (double)q[i];
                }
            __syncthreads();
            double a = 0.0;
            for (int i = tid; i < n; i += blockDim.x) a += v[i] * v[i];
            const double nv = sqrt(block_sum(a, red));
            if (nv > tol * pmax && nv > 0) {
                const double inv = 1.0 / nv;
                for (int i = tid; i < n; i += blockDim.x) Q[i + (size_t)j * n] = (T)(v[i] * inv);
                break;
            }
            // dependent column: the unit vector with the largest remainder
            // 1 - sum_k Q(i, k)^2 (the first index on ties), then orthogonalise it
            double bv = -1.0;
            int bi = n;
            for (int i = tid; i < n; i += blockDim.x) {  // increasing i: strict > keeps the first
                double res = 1.0;
                for (int k = 0; k < j; ++k) res -= (double)Q[i + (size_t)k * n] * (double)Q[i + (size_t)k * n];
                if (res > bv) {
                    bv = res;
                    bi = i;
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_down(bv, off, 64);
                const int oi = __shfl_down(bi, off, 64);
                if (ov > bv || (ov == bv && oi < bi)) {
                    bv = ov;
                    bi = oi;
                }
            }
            __syncthreads();
            if ((tid & 63) == 0) red[tid >> 6] = bv;
            __shared__ int ridx[4];
            if ((tid & 63) == 0) ridx[tid >> 6] = bi;
            __syncthreads();
            if (tid == 0) {
                best_val = red[0];
                best_idx = ridx[0];
                for (int w = 1; w < 4; ++w)
                    if (red[w] > best_val || (red[w] == best_val && ridx[w] < best_idx)) {
                        best_val = red[w];
                        best_idx = ridx[w];
                    }
            }
            __syncthreads();
            for (int i = tid; i < n; i += blockDim.x) v[i] = i == best_idx ? 1.0 : 0.0;
            pmax = 1.0;  // the candidate has unit norm; accept any remainder above tol
        }
        __syncthreads();
    }
}

// Column s of U (n x r, ld n): lambda_s = 2-norm, U(:, s) /= lambda_s (a zero
// column stays zero).  One workgroup per column.
template <typename T>
__global__ void __launch_bounds__(256) k_als_normalize(int n, T* __restrict__ U, T* __restrict__ lambda) {
    __shared__ double red[4];
    __shared__ double norm;
    const int s = blockIdx.x, tid = threadIdx.x;
    T* u = U + (size_t)s * n;
    double acc = 0.0;
    for (int i = tid; i < n; i += blockDim.x) acc += (double)u[i] * (double)u[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w];
        norm = sqrt(v);
        lambda[s] = (T)norm;
    }
    __syncthreads();
    if (norm > 0) {
        const double inv = 1.0 / norm;
        for (int i = tid; i < n; i += blockDim.x) u[i] = (T)((double)u[i] * inv);
    }
}

// FP64 partial sums of squares, one per workgroup (grid-stride).
template <typename T>
__global__ void __launch_bounds__(256) k_als_sumsq(size_t n, const T* __restrict__ x, double* __restrict__ partials) {
    __shared__ double red[4];
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        acc += (double)x[i] * (double)x[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w];
        partials[blockIdx.x] = v;
    }
}

// Tucker core from U3^T Y3: src(s3 + r s2 + r^2 s1) -> dst(s1 + r s2 + r^2 s3).
template <typename T>
__global__ void __launch_bounds__(256) k_als_core(int r, const T* __restrict__ src, T* __restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r * r) return;
    const int s1 = e % r, s2 = (e / r) % r, s3 = e / (r * r);
    dst[e] = src[s3 + r * s2 + r * r * s1];
}

// CP residual ||X - X^||^2 = ||X||^2 - 2 sum_s lambda_s D(s, s)
//     + sum_{s,s'} lambda_s lambda_s' G1 G2 G3 (s, s'),
// D = M3^T U3 (M3 the last mode-3 right-hand side); out[0] = residual^2.
template <typename T>
__global__ void __launch_bounds__(256) k_als_cp_fit(int r, const T* __restrict__ lambda, const double* __restrict__ G1,
                                                    const double* __restrict__ G2, const double* __restrict__ G3,
                                                    const double* __restrict__ D, const double* __restrict__ xx,
                                                    double* __restrict__ out) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int s = e % r, sp = e / r;
        const double ls = (double)lambda[s], lp = (double)lambda[sp];
        acc += ls * lp * G1[e] * G2[e] * G3[e];
        if (s == sp) acc -= 2.0 * ls * D[e];
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = xx[0];
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v += red[w];
        out[0] = v;
    }
}

// Tucker residual: ||X||^2 - ||C||^2 (orthonormal factors).
__global__ void k_als_tucker_fit(const double* __restrict__ xx, const double* __restrict__ cc,
                                 double* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = xx[0] - cc[0];
}

}  // namespace

// ---- host orchestration ----------------------------------------------------------
namespace {

template <typename T>
struct AlsRun {
    rocblas_handle h;
    hipStream_t st;
    const AlsScratch<T>& w;
    int r;
    int rc = 0;

    void check(rocblas_status s) {
        if (s != rocblas_status_success && !rc) rc = -2;
    }
    void check(hipError_t e) {
        if (e != hipSuccess && !rc) rc = -3;
    }
    // G (r x r, FP64) = A^T B, A and B n x r
    void gram(int n, const T* A, int lda, const T* B, int ldb, double* G) {
        hipLaunchKernelGGL((k_als_gram<T>), dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, st, n, r, A, lda, B, ldb,
                           G);
        check(hipGetLastError());
    }
    void chol_inv(const double* G1, const double* G2, int mode, T* out) {
        hipLaunchKernelGGL((k_als_chol_inv<T>), dim3(1), dim3(256), 2 * sizeof(double) * r * r, st, r, G1, G2, mode,
                           out, w.flag);
        check(hipGetLastError());
    }
    // dst = orth(src) (src, dst n x r, ld n; may alias: src is copied first)
    void orth(int n, const T* src, T* dst) {
        const T* in = src;
        if (src == dst) {
            check(hipMemcpyAsync(w.Q, src, sizeof(T) * (size_t)n * r, hipMemcpyDeviceToDevice, st));
            in = w.Q;
        }
        const double tol = sizeof(T) == 4 ? kAlsTolF32 : kAlsTolF64;
        hipLaunchKernelGGL((k_als_orth<T>), dim3(1), dim3(256), sizeof(double) * (size_t)n, st, n, r, in, dst, tol);
        check(hipGetLastError());
    }
    // U (n x r) <- orth(Y Y^T U), Y n x r^2 (ld n)
    void subspace_step(int n, const T* Y, T* U) {
        const T one = 1, zero = 0;
        const int rr = r * r;
        check(gemm(h, rocblas_operation_transpose, rocblas_operation_none, rr, r, n, &one, Y, n, U, n, &zero, w.W, rr));
        check(gemm(h, rocblas_operation_none, rocblas_operation_none, n, r, rr, &one, Y, n, w.W, rr, &zero, w.P, n));
        orth(n, w.P, U);
    }
    // U_n <- M V^-1 normalised, V = (Ub^T Ub) * (Uc^T Uc); M = w.P (n x r)
    void cp_update(int n, int nb, const T* Ub, int nc, const T* Uc, T* Un, T* lambda) {
        const T one = 1, zero = 0;
        gram(nb, Ub, nb, Ub, nb, w.G[0]);
        gram(nc, Uc, nc, Uc, nc, w.G[1]);
        chol_inv(w.G[0], w.G[1], 1, w.Rinv);
        check(gemm(h, rocblas_operation_none, rocblas_operation_none, n, r, r, &one, w.P, n, w.Rinv, r, &zero, Un, n));
        hipLaunchKernelGGL((k_als_normalize<T>), dim3(r), dim3(256), 0, st, n, Un, lambda);
        check(hipGetLastError());
    }
    void sumsq(size_t n, const T* x, double* out) {
        const int blocks = (int)std::min<size_t>(1024, (n + 255) / 256);
        hipLaunchKernelGGL((k_als_sumsq<T>), dim3(blocks), dim3(256), 0, st, n, x, w.partials);
        check(hipGetLastError());
        check(launch_energy_reduce(st, w.partials, blocks, 1.0, out));
    }
};

}  // namespace

template <typename T>
int als_compress(void* handle, hipStream_t st, const int n[3], int r, bool tucker, int sweeps, const T* m, T* core,
                 T* U, double* err2, const AlsScratch<T>& w) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return -1;
    AlsRun<T> run{h, st, w, r};
    const int n1 = n[0], n2 = n[1], n3 = n[2];
    const size_t N = (size_t)n1 * n2 * n3;
    const T one = 1, zero = 0;
    const rocblas_operation NN = rocblas_operation_none, TT = rocblas_operation_transpose;
    // ||X||^2 of every component first: a zero component (CP) is skipped
    double xx[6];
    for (int p = 0; p < 3; ++p) run.sumsq(N, m + (size_t)p * N, err2 + 2 * p + 1);
    run.check(hipMemcpyAsync(xx, err2, sizeof(xx), hipMemcpyDeviceToHost, st));
    run.check(hipStreamSynchronize(st));
    for (int p = 0; p < 3 && !run.rc; ++p) {
        const T* X = m + (size_t)p * N;
        T* U1 = U + (size_t)p * r * n1;
        T* U2 = U + (size_t)3 * r * n1 + (size_t)p * r * n2;
        T* U3 = U + (size_t)3 * r * (n1 + n2) + (size_t)p * r * n3;
        double* e2 = err2 + 2 * p;  // [residual^2, ||X||^2]
        if (!tucker && !(xx[2 * p + 1] > 0)) {  // zero component: weights 0, factors as given
            run.check(hipMemsetAsync(core + (size_t)p * r, 0, sizeof(T) * r, st));
            run.check(hipMemsetAsync(e2, 0, sizeof(double), st));
            continue;
        }
        if (tucker) {
            run.orth(n1, U1, U1);
            run.orth(n2, U2, U2);
            run.orth(n3, U3, U3);
            for (int it = 0; it < sweeps && !run.rc; ++it) {
                // T3 = X x_3 U3^T (n1 n2 x r)
                run.check(gemm(h, NN, NN, n1 * n2, r, n3, &one, X, n1 * n2, U3, n3, &zero, w.Tm, n1 * n2));
                // mode 1: Y(i1, s2 + r s3) = sum_i2 T3(i1, i2, s3) U2(i2, s2)
                run.check(gemm_sb(h, NN, NN, n1, r, n2, &one, w.Tm, n1, (rocblas_stride)n1 * n2, U2, n2, 0, &zero, w.Y,
                                  n1, (rocblas_stride)n1 * r, r));
                run.subspace_step(n1, w.Y, U1);
                // mode 2: Y(i2, s1 + r s3) = sum_i1 T3(i1, i2, s3) U1(i1, s1)
                run.check(gemm_sb(h, TT, NN, n2, r, n1, &one, w.Tm, n1, (rocblas_stride)n1 * n2, U1, n1, 0, &zero, w.Y,
                                  n2, (rocblas_stride)n2 * r, r));
                run.subspace_step(n2, w.Y, U2);
                // mode 3: T1 = X^T U1 (n2 n3 x r); Y(i3, s2 + r s1) = sum_i2 T1(i2, i3, s1) U2(i2, s2)
                run.check(gemm(h, TT, NN, n2 * n3, r, n1, &one, X, n1, U1, n1, &zero, w.Tm, n2 * n3));
                run.check(gemm_sb(h, TT, NN, n3, r, n2, &one, w.Tm, n2, (rocblas_stride)n2 * n3, U2, n2, 0, &zero, w.Y,
                                  n3, (rocblas_stride)n3 * r, r));
                run.subspace_step(n3, w.Y, U3);
            }
            // core: C = X x_1 U1^T x_2 U2^T x_3 U3^T from Y3 with the final factors
            run.check(gemm(h, TT, NN, n2 * n3, r, n1, &one, X, n1, U1, n1, &zero, w.Tm, n2 * n3));
            run.check(gemm_sb(h, TT, NN, n3, r, n2, &one, w.Tm, n2, (rocblas_stride)n2 * n3, U2, n2, 0, &zero, w.Y, n3,
                              (rocblas_stride)n3 * r, r));
            run.check(gemm(h, TT, NN, r, r * r, n3, &one, U3, n3, w.Y, n3, &zero, w.Q, r));
            T* Cp = core + (size_t)p * r * r * r;
            hipLaunchKernelGGL((k_als_core<T>), dim3((unsigned)((r * r * r + 255) / 256)), dim3(256), 0, st, r, w.Q,
                               Cp);
            run.check(hipGetLastError());
            run.sumsq((size_t)r * r * r, Cp, w.scal);
            hipLaunchKernelGGL(k_als_tucker_fit, dim3(1), dim3(64), 0, st, e2 + 1, w.scal, e2);
            run.check(hipGetLastError());
        } else {
            T* lam = core + (size_t)p * r;
            for (int it = 0; it < sweeps && !run.rc; ++it) {
                // T3 = X x_3 U3^T (n1 n2 x r)
                run.check(gemm(h, NN, NN, n1 * n2, r, n3, &one, X, n1 * n2, U3, n3, &zero, w.Tm, n1 * n2));
                // mode 1: M(:, s) = T3(:, :, s) U2(:, s)
                run.check(gemv_sb(h, NN, n1, n2, &one, w.Tm, n1, (rocblas_stride)n1 * n2, U2, 1, n2, &zero, w.P, 1,
                                  n1, r));
                run.cp_update(n1, n2, U2, n3, U3, U1, lam);
                // mode 2: M(:, s) = T3(:, :, s)^T U1(:, s)
                run.check(gemv_sb(h, TT, n1, n2, &one, w.Tm, n1, (rocblas_stride)n1 * n2, U1, 1, n1, &zero, w.P, 1,
                                  n2, r));
                run.cp_update(n2, n1, U1, n3, U3, U2, lam);
                // mode 3: T1 = X^T U1 (n2 n3 x r); M(:, s) = T1(:, :, s)^T U2(:, s)
                run.check(gemm(h, TT, NN, n2 * n3, r, n1, &one, X, n1, U1, n1, &zero, w.Tm, n2 * n3));
                run.check(gemv_sb(h, TT, n2, n3, &one, w.Tm, n2, (rocblas_stride)n2 * n3, U2, 1, n2, &zero, w.P, 1,
                                  n3, r));
                run.cp_update(n3, n1, U1, n2, U2, U3, lam);
            }
            // residual from the last mode-3 right-hand side (final U1, U2) and the final factors
            run.gram(n1, U1, n1, U1, n1, w.G[0]);
            run.gram(n2, U2, n2, U2, n2, w.G[1]);
            run.gram(n3, U3, n3, U3, n3, w.G[2]);
            run.gram(n3, w.P, n3, U3, n3, w.G[3]);
            hipLaunchKernelGGL((k_als_cp_fit<T>), dim3(1), dim3(256), 0, st, r, lam, w.G[0], w.G[1], w.G[2], w.G[3],
                               e2 + 1, e2);
            run.check(hipGetLastError());
        }
    }
    return run.rc;
}

template int als_compress<float>(void*, hipStream_t, const int[3], int, bool, int, const float*, float*, float*,
                                 double*, const AlsScratch<float>&);
template int als_compress<double>(void*, hipStream_t, const int[3], int, bool, int, const double*, double*, double*,
                                  double*, const AlsScratch<double>&);

}  // namespace demag
