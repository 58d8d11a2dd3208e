// Tensor-grid method (TG, Sec. 3.2, eqs. (transform), (gausspot), (sumpot),
// (Dmat), (gs)) in its dense form on the plan's regular grid.
//
// The kernel of eq. (scpot) is written as a Gaussian integral (eq.
// (transform)), 1/r^3 = (4/sqrt(pi)) int_0^inf tau^2 exp(-tau^2 r^2) dtau,
// and the tau integral is taken by a Sinc (trapezoidal) quadrature in
// t = log(tau): tau_l = exp(t0 + l h), l = 0..R-1, weight h tau_l^3.  The cell
// integrals then factor into one-dimensional Gaussian matrices per axis q and
// node l (eq. (Dmat)): for the magnetization component p,
//     q != p:  E(i', i) = int_{cell i} exp(-tau^2 (x_i' - x)^2) dx
//     q == p:  O(i', i) = int_{cell i} (x_i' - x) exp(-tau^2 (x_i' - x)^2) dx
// (x_i' the target cell centre), here in closed form (erf / erfc and exp,
// evaluated in FP64) instead of the paper's Gauss-Legendre quadrature.  The
// potential on the cell centres is the block-CP sum of eq. (sumpot),
//     Phi = Ms h_max sum_p sum_l c_l  M_p x_1 D_1 x_2 D_2 x_3 D_3,
//     c_l = h tau_l^3 / pi^(3/2),
// lengths in units of the largest cell edge h_max.  On the GPU each mode
// product is a GEMM (MFMA through rocBLAS):
//     mode 1: Y1[l] = D_1[l] M_p                (strided-batched over l)
//     mode 2: Y2[l](:,:,k) = Y1[l](:,:,k) D_2[l]^T   (pointer-batched over l, k)
//     mode 3: Phi += [Y2[0] .. Y2[R-1]] [c_l D_3[l]^T stacked]  (one GEMM, K = R n3)
// The field is the finite-difference gradient of the SP method.
#include <rocblas/rocblas.h>

#include <cmath>
#include <vector>

#include "blas.hpp"
#include "internal.hpp"
#include "tg_gauss.hpp"

namespace demag {

namespace {

// Gaussian matrices of one axis (n cells of edge d, reduced units) for every
// node: E[l][i][i'] and O[l][i][i'] column-major (entry (i', i) at i' + i n).
template <typename T>
__global__ void __launch_bounds__(256) k_tg_axis(int n, double d, int R, const double* __restrict__ tau,
                                                 T* __restrict__ E, T* __restrict__ O) {
    const size_t nn = (size_t)n * n;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * R) return;
    const int l = (int)(t / nn);
    const size_t e = t - (size_t)l * nn;
    const int ip = (int)(e % n), i = (int)(e / n);
    const double a = (ip + 0.5) * d, c = (i + 0.5) * d, s = tau[l];
    E[t] = (T)gauss_even(a, c, d, s);
    O[t] = (T)gauss_odd(a, c, d, s);
}

// Mode-3 right factor: B3[(l n3 + k) + k' R n3] = c_l D3[l](k', k).
template <typename T>
__global__ void __launch_bounds__(256) k_tg_stack3(int n3, int R, const double* __restrict__ c,
                                                   const T* __restrict__ D3, T* __restrict__ B3) {
    const size_t K = (size_t)R * n3;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= K * n3) return;
    const size_t row = t % K;
    const int kp = (int)(t / K);
    const int l = (int)(row / n3), k = (int)(row - (size_t)l * n3);
    B3[t] = (T)(c[l] * (double)D3[(size_t)l * n3 * n3 + kp + (size_t)k * n3]);
}

}  // namespace

// Sinc nodes for 1/r^3 on [rmin, rmax] (reduced units): t from
// -log(rmax) - 10 (the part below is under exp(-30) of the smallest term) to
// log(14 / rmin) (exp(-tau^2 rmin^2 / 4) negligible beyond), step h.
int tg_sinc_nodes(double rmin, double rmax, double h, std::vector<double>& tau, std::vector<double>& w) {
    if (!(rmin > 0) || !(rmax >= rmin) || !(h > 0)) return -1;
    const double t0 = -std::log(rmax) - 10.0, t1 = std::log(14.0 / rmin);
    const int R = (int)std::ceil((t1 - t0) / h) + 1;
    tau.resize(R);
    w.resize(R);
    for (int l = 0; l < R; ++l) {
        const double t = t0 + l * h;
        tau[l] = std::exp(t);
        w[l] = h * tau[l] * tau[l] * tau[l] / std::pow(3.14159265358979323846, 1.5);
    }
    return R;
}

template <typename T>
hipError_t launch_tg_axis(hipStream_t st, int n, double d, int R, const double* tau, T* E, T* O) {
    const size_t total = (size_t)n * n * R;
    hipLaunchKernelGGL((k_tg_axis<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, d, R, tau, E, O);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tg_stack3(hipStream_t st, int n3, int R, const double* c, const T* D3, T* B3) {
    const size_t total = (size_t)R * n3 * n3;
    hipLaunchKernelGGL((k_tg_stack3<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n3, R, c, D3, B3);
    return hipGetLastError();
}

template hipError_t launch_tg_axis<float>(hipStream_t, int, double, int, const double*, float*, float*);
template hipError_t launch_tg_axis<double>(hipStream_t, int, double, int, const double*, double*, double*);
template hipError_t launch_tg_stack3<float>(hipStream_t, int, int, const double*, const float*, float*);
template hipError_t launch_tg_stack3<double>(hipStream_t, int, int, const double*, const double*, double*);

// ---- the GEMM chain ----------------------------------------------------------

// Phi (column-major n1 x n2 x n3, i.e. [n3][n2][n1]) for the three components
// of m.  D1E/D1O [R][n1][n1], D2E/D2O [R][n2][n2] column-major, B3[p]
// [n3][R n3] stacked mode-3 factors with c_l folded in; Y1, Y2 [R][N]
// scratch; Y1k/Y2k/D2p device pointer arrays for the mode-2 batch (R n3
// entries each; D2p per component).  alpha = Ms h_max.
template <typename T>
int tg_potential(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const T* m, const T* D1E,
                 const T* D1O, const T* const* D2p[3], const T* const* Y1k, T* const* Y2k, const T* const B3[3], T* Y1,
                 T* Y2, T* phi, double alpha) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return -1;
    const size_t N = (size_t)n1 * n2 * n3;
    const T one = 1, zero = 0, al = (T)alpha;
    for (int p = 0; p < 3; ++p) {
        const T* D1 = p == 0 ? D1O : D1E;
        // mode 1: Y1[l] (n1 x n2 n3) = D1[l] (n1 x n1) M_p (n1 x n2 n3)
        if (gemm_sb(h, rocblas_operation_none, rocblas_operation_none, n1, n2 * n3, n1, &one, D1, n1,
                    (rocblas_stride)n1 * n1, m + (size_t)p * N, n1, 0, &zero, Y1, n1, (rocblas_stride)N, R) !=
            rocblas_status_success)
            return -2;
        // mode 2: Y2[l](:,:,k) (n1 x n2) = Y1[l](:,:,k) (n1 x n2) D2[l]^T
        if (gemm_b(h, rocblas_operation_none, rocblas_operation_transpose, n1, n2, n2, &one, Y1k, n1, D2p[p], n2,
                   &zero, Y2k, n1, R * n3) != rocblas_status_success)
            return -3;
        // mode 3 and the node sum: phi (n1 n2 x n3) (+)= alpha Y2 (n1 n2 x R n3) B3[p] (R n3 x n3)
        if (gemm(h, rocblas_operation_none, rocblas_operation_none, n1 * n2, n3, R * n3, &al, Y2, n1 * n2, B3[p],
                 R * n3, p == 0 ? &zero : &one, phi, n1 * n2) != rocblas_status_success)
            return -4;
    }
    (void)Y1;
    return 0;
}

template int tg_potential<float>(void*, hipStream_t, int, int, int, int, const float*, const float*, const float*,
                                 const float* const* [3], const float* const*, float* const*, const float* const[3],
                                 float*, float*, float*, double);
template int tg_potential<double>(void*, hipStream_t, int, int, int, int, const double*, const double*,
                                  const double*, const double* const* [3], const double* const*, double* const*,
                                  const double* const[3], double*, double*, double*, double);

}  // namespace demag
