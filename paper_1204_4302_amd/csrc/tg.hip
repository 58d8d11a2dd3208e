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
// In FP32 each of the three runs the rocBLAS solution chosen for its shape
// when the method is prepared (tg_tune).  By default in FP32 modes 1 and 2 run
// instead as one hand-written kernel on the matrix cores (tg_fused.hip,
// tg_potential_fused), with half the scratch.  The field is the
// finite-difference gradient of the SP method.
#define ROCBLAS_BETA_FEATURES_API  // rocblas_gemm_ex_get_solutions: the mode-3 solution is chosen by timing
#include <rocblas/rocblas.h>

#include <algorithm>
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
namespace {

// mode 3: phi (M x N) = al Y2 (M x K) B3 (K x N) + be phi, column-major; FP32
// with rocBLAS solution `sol` (0: rocBLAS's default choice).
rocblas_status mode3(rocblas_handle h, int M, int N, int K, const float* al, const float* A, const float* B,
                     const float* be, float* C, int sol) {
    if (sol == 0) return gemm(h, rocblas_operation_none, rocblas_operation_none, M, N, K, al, A, M, B, K, be, C, M);
    return rocblas_gemm_ex(h, rocblas_operation_none, rocblas_operation_none, M, N, K, al, A, rocblas_datatype_f32_r, M,
                           B, rocblas_datatype_f32_r, K, be, C, rocblas_datatype_f32_r, M, C, rocblas_datatype_f32_r, M,
                           rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, sol, 0);
}
rocblas_status mode3(rocblas_handle h, int M, int N, int K, const double* al, const double* A, const double* B,
                     const double* be, double* C, int) {
    return gemm(h, rocblas_operation_none, rocblas_operation_none, M, N, K, al, A, M, B, K, be, C, M);
}

// mode 1: Y1[l] (n1 x n2 n3) = D1[l] (n1 x n1) Mp (n1 x n2 n3) for l < R (Mp
// shared: stride 0); FP32 with rocBLAS solution `sol` (0: the default).
rocblas_status mode1(rocblas_handle h, int n1, int nc, int R, const float* D1, const float* Mp, float* Y1, int sol) {
    const float one = 1, zero = 0;
    const rocblas_stride sD = (rocblas_stride)n1 * n1, sY = (rocblas_stride)n1 * nc;
    if (sol == 0)
        return gemm_sb(h, rocblas_operation_none, rocblas_operation_none, n1, nc, n1, &one, D1, n1, sD, Mp, n1, 0,
                       &zero, Y1, n1, sY, R);
    return rocblas_gemm_strided_batched_ex(h, rocblas_operation_none, rocblas_operation_none, n1, nc, n1, &one, D1,
                                           rocblas_datatype_f32_r, n1, sD, Mp, rocblas_datatype_f32_r, n1, 0, &zero,
                                           Y1, rocblas_datatype_f32_r, n1, sY, Y1, rocblas_datatype_f32_r, n1, sY, R,
                                           rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, sol, 0);
}
rocblas_status mode1(rocblas_handle h, int n1, int nc, int R, const double* D1, const double* Mp, double* Y1, int) {
    const double one = 1, zero = 0;
    return gemm_sb(h, rocblas_operation_none, rocblas_operation_none, n1, nc, n1, &one, D1, n1,
                   (rocblas_stride)n1 * n1, Mp, n1, 0, &zero, Y1, n1, (rocblas_stride)n1 * nc, R);
}

// mode 2: Y2[l](:,:,k) (n1 x n2) = Y1[l](:,:,k) (n1 x n2) D2[l]^T for the
// `batch` (l, k) pairs of the pointer arrays; FP32 with rocBLAS solution `sol`
// (0: the default).
rocblas_status mode2(rocblas_handle h, int n1, int n2, int batch, const float* const* Y1k, const float* const* D2,
                     float* const* Y2k, int sol) {
    const float one = 1, zero = 0;
    if (sol == 0)
        return gemm_b(h, rocblas_operation_none, rocblas_operation_transpose, n1, n2, n2, &one, Y1k, n1, D2, n2,
                      &zero, Y2k, n1, batch);
    return rocblas_gemm_batched_ex(h, rocblas_operation_none, rocblas_operation_transpose, n1, n2, n2, &one, Y1k,
                                   rocblas_datatype_f32_r, n1, D2, rocblas_datatype_f32_r, n2, &zero, Y2k,
                                   rocblas_datatype_f32_r, n1, (void*)Y2k, rocblas_datatype_f32_r, n1, batch,
                                   rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, sol, 0);
}
rocblas_status mode2(rocblas_handle h, int n1, int n2, int batch, const double* const* Y1k, const double* const* D2,
                     double* const* Y2k, int) {
    const double one = 1, zero = 0;
    return gemm_b(h, rocblas_operation_none, rocblas_operation_transpose, n1, n2, n2, &one, Y1k, n1, D2, n2, &zero,
                  Y2k, n1, batch);
}

// Of the candidate solutions `sols` (each run by run(sol); 0 is rocBLAS's
// default), the fastest that beats the default and whose first `cmp` output
// values agree with the default's to 1e-5 (relative max-norm: no solution of
// reduced precision is taken); 0 if none.  Each candidate is timed once (one
// warm-up, three runs); a candidate that cannot run the problem is skipped.
template <typename RunF>
int pick_solution(hipStream_t st, const std::vector<rocblas_int>& sols, RunF run, const float* out, size_t cmp,
                  int* best) {
    *best = 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -3;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -3;
    }
    auto time_sol = [&](int sol, float* ms) {
        if (run(sol) != rocblas_status_success) return false;
        if (hipEventRecord(e0, st) != hipSuccess) return false;
        for (int r = 0; r < 3; ++r)
            if (run(sol) != rocblas_status_success) return false;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
        return hipEventElapsedTime(ms, e0, e1) == hipSuccess;
    };
    std::vector<std::pair<float, int>> times;
    float t0 = 0;
    int rc = time_sol(0, &t0) ? 0 : -4;
    for (size_t i = 0; i < sols.size() && !rc; ++i) {
        float t = 0;
        if (sols[i] != 0 && time_sol(sols[i], &t)) times.push_back({t, sols[i]});
        (void)hipGetLastError();
    }
    std::sort(times.begin(), times.end());
    std::vector<float> ref(cmp), got(cmp);
    if (!rc && (run(0) != rocblas_status_success ||
                hipMemcpyAsync(ref.data(), out, sizeof(float) * cmp, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess))
        rc = -5;
    double scale = 0;
    for (float v : ref) scale = std::max(scale, (double)std::fabs(v));
    for (size_t i = 0; i < times.size() && i < 8 && !rc && times[i].first < t0; ++i) {
        if (run(times[i].second) != rocblas_status_success) continue;
        if (hipMemcpyAsync(got.data(), out, sizeof(float) * cmp, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = -5;
            break;
        }
        double err = 0;
        for (size_t j = 0; j < cmp; ++j) err = std::max(err, (double)std::fabs(got[j] - ref[j]));
        if (scale > 0 && err <= 1e-5 * scale) {
            *best = times[i].second;
            break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

// rocBLAS's default choice pads its tiles for some of the mode products'
// shapes (mode 3 is skinny: N = n3 against M = n1 n2 and K = R n3); every
// solution rocBLAS offers for each of the three GEMMs is timed once on the
// plan's buffers and the fastest that agrees with the default is kept
// (pick_solution).  Mode 2 runs after mode 1 and before mode 3, so that each
// reads the previous one's output.  FP64 keeps the defaults.
// rocBLAS marks its solution listing as a beta interface (deprecation attribute)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wdeprecated-declarations"
template <>
int tg_tune<float>(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const float* D1, const float* Mp,
                   float* Y1, const float* const* Y1k, const float* const* D2k, float* const* Y2k, float* Y2,
                   const float* B3, float* phi, int* sol1, int* sol2, int* sol3) {
    *sol1 = *sol2 = *sol3 = 0;
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return -1;
    const float one = 1, zero = 0;
    const int nc = n2 * n3, M = n1 * n2, K = R * n3;
    std::vector<rocblas_int> sols;
    rocblas_int count = 0;
    // mode 1
    const rocblas_stride sD = (rocblas_stride)n1 * n1, sY = (rocblas_stride)n1 * nc;
    auto list1 = [&](rocblas_int* arr) {
        return rocblas_gemm_strided_batched_ex_get_solutions(
            h, rocblas_operation_none, rocblas_operation_none, n1, nc, n1, &one, D1, rocblas_datatype_f32_r, n1, sD, Mp,
            rocblas_datatype_f32_r, n1, 0, &zero, Y1, rocblas_datatype_f32_r, n1, sY, Y1, rocblas_datatype_f32_r, n1, sY,
            R, rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, 0, arr, &count);
    };
    int rc = 0;
    if (Y1 && list1(nullptr) == rocblas_status_success && count > 0) {
        sols.assign((size_t)count, 0);
        if (list1(sols.data()) == rocblas_status_success)
            rc = pick_solution(st, sols, [&](int sol) { return mode1(h, n1, nc, R, D1, Mp, Y1, sol); }, Y1,
                               std::min<size_t>((size_t)R * n1 * nc, (size_t)1 << 22), sol1);
    }
    if (rc) return rc;
    // mode 2
    count = 0;
    const int nb = R * n3;
    auto list2 = [&](rocblas_int* arr) {
        return rocblas_gemm_batched_ex_get_solutions(
            h, rocblas_operation_none, rocblas_operation_transpose, n1, n2, n2, &one, Y1k, rocblas_datatype_f32_r, n1,
            D2k, rocblas_datatype_f32_r, n2, &zero, Y2k, rocblas_datatype_f32_r, n1, (void*)Y2k, rocblas_datatype_f32_r, n1,
            nb, rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, 0, arr, &count);
    };
    if (Y1 && list2(nullptr) == rocblas_status_success && count > 0) {
        sols.assign((size_t)count, 0);
        if (list2(sols.data()) == rocblas_status_success)
            rc = pick_solution(st, sols, [&](int sol) { return mode2(h, n1, n2, nb, Y1k, D2k, Y2k, sol); }, Y2,
                               std::min<size_t>((size_t)nb * n1 * n2, (size_t)1 << 22), sol2);
    }
    if (rc) return rc;
    // mode 3
    count = 0;
    auto list3 = [&](rocblas_int* arr) {
        return rocblas_gemm_ex_get_solutions(h, rocblas_operation_none, rocblas_operation_none, M, n3, K, &one, Y2,
                                             rocblas_datatype_f32_r, M, B3, rocblas_datatype_f32_r, K, &zero, phi,
                                             rocblas_datatype_f32_r, M, phi, rocblas_datatype_f32_r, M,
                                             rocblas_datatype_f32_r, rocblas_gemm_algo_solution_index, 0, arr, &count);
    };
    if (list3(nullptr) == rocblas_status_success && count > 0) {
        sols.assign((size_t)count, 0);
        if (list3(sols.data()) == rocblas_status_success)
            rc = pick_solution(st, sols, [&](int sol) { return mode3(h, M, n3, K, &one, Y2, B3, &zero, phi, sol); },
                               phi, std::min<size_t>((size_t)M * n3, (size_t)1 << 22), sol3);
    }
    return rc;
}
#pragma clang diagnostic pop
template <>
int tg_tune<double>(void*, hipStream_t, int, int, int, int, const double*, const double*, double*,
                    const double* const*, const double* const*, double* const*, double*, const double*, double*,
                    int* sol1, int* sol2, int* sol3) {
    *sol1 = *sol2 = *sol3 = 0;
    return 0;
}

template <typename T>
int tg_potential(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const T* m, const T* D1E,
                 const T* D1O, const T* const* D2p[3], const T* const* Y1k, T* const* Y2k, const T* const B3[3], T* Y1,
                 T* Y2, T* phi, double alpha, int sol1, int sol2, int sol3) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return -1;
    const size_t N = (size_t)n1 * n2 * n3;
    const T one = 1, zero = 0, al = (T)alpha;
    for (int p = 0; p < 3; ++p) {
        const T* D1 = p == 0 ? D1O : D1E;
        // mode 1: Y1[l] (n1 x n2 n3) = D1[l] (n1 x n1) M_p (n1 x n2 n3)
        if (mode1(h, n1, n2 * n3, R, D1, m + (size_t)p * N, Y1, sol1) != rocblas_status_success) return -2;
        // mode 2: Y2[l](:,:,k) (n1 x n2) = Y1[l](:,:,k) (n1 x n2) D2[l]^T
        if (mode2(h, n1, n2, R * n3, Y1k, D2p[p], Y2k, sol2) != rocblas_status_success) return -3;
        // mode 3 and the node sum: phi (n1 n2 x n3) (+)= alpha Y2 (n1 n2 x R n3) B3[p] (R n3 x n3)
        if (mode3(h, n1 * n2, n3, R * n3, &al, Y2, B3[p], p == 0 ? &zero : &one, phi, sol3) !=
            rocblas_status_success)
            return -4;
    }
    (void)Y1;
    return 0;
}

// The same potential with the first two mode products fused (tg_fused.hip):
// per component, Y2 = D1 M_p D2^T for every node and plane in one launch,
// then the mode-3 GEMM and the node sum as in tg_potential.
int tg_potential_fused(void* handle, hipStream_t st, int n1, int n2, int n3, int R, const float* m, const TGFused& f,
                       const float* const B3[3], float* Y2, float* phi, double alpha, int sol3) {
    rocblas_handle h = (rocblas_handle)handle;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return -1;
    const size_t N = (size_t)n1 * n2 * n3;
    const float one = 1, zero = 0, al = (float)alpha;
    for (int p = 0; p < 3; ++p) {
        if (launch_tg_mode12(st, n1, n2, n3, R, f.D1[p], f.lo1[p], f.hi1[p], m + (size_t)p * N, f.D2[p], f.lo2[p],
                             f.hi2[p], Y2) != hipSuccess)
            return -5;
        if (mode3(h, n1 * n2, n3, R * n3, &al, Y2, B3[p], p == 0 ? &zero : &one, phi, sol3) !=
            rocblas_status_success)
            return -4;
    }
    return 0;
}

template int tg_potential<float>(void*, hipStream_t, int, int, int, int, const float*, const float*, const float*,
                                 const float* const* [3], const float* const*, float* const*, const float* const[3],
                                 float*, float*, float*, double, int, int, int);
template int tg_potential<double>(void*, hipStream_t, int, int, int, int, const double*, const double*,
                                  const double*, const double* const* [3], const double* const*, double* const*,
                                  const double* const[3], double*, double*, double*, double, int, int, int);

}  // namespace demag
