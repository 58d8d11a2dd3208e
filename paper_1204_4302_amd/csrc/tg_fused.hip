// Fused first and second mode products of the tensor-grid sum (Sec. 3.2, eq.
// (sumpot)) in FP32 on the matrix cores.
//
// For node l, z-plane k and magnetization component p the sum needs
//     Y2[l](:,:,k) = D_1[l] M_p(:,:,k) D_2[l]^T            (n1 x n2)
// before the third mode product and the node sum (a GEMM with inner
// dimension R n3, left to the caller).  One workgroup computes 64 rows of
// Y2[l](:,:,k): first the 64 x n2 block of Y1 = D_1 M in registers and then
// in LDS, then Y1 D_2^T from LDS, so the intermediate Y1 (R N values per
// component) never reaches HBM.  Both products run on v_mfma_f32_16x16x4f32
// with operands read straight from the row-major Gaussian matrices and the
// magnetization: a lane's four consecutive k values (one 16-byte load) feed
// four instructions, instruction j taking k = 16 g + 4 (lane / 16) + j of the
// group g of 16, the same permutation of k on both operands, so the sum over
// a group is complete.
//
// The Gaussian matrices of the nodes with large tau are banded: their
// entries far from the diagonal are exactly zero in FP32.  For every block of
// 64 rows the range of 16-column groups holding a nonzero entry is found once
// at set-up (k_tg_band) and the products skip the groups outside it, which
// only drops products with exact zeros (the sums are unchanged for finite m).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace demag {

namespace {

typedef float tgf4 __attribute__((ext_vector_type(4)));

constexpr int kTgRows = 64;  // rows of Y2 per workgroup (four MFMA row tiles)
static_assert(kTgMode12MaxN2 <= 512, "a wave holds the bands of at most two passes of 16 column tiles");

// Columns [lo, hi] holding a nonzero entry of each row block of 64 of the
// row-major matrices [R][n][n] (lo starts above any column, hi at -1).
__global__ void __launch_bounds__(256) k_tg_band(int n, int R, const float* __restrict__ D, int* __restrict__ lo,
                                                 int* __restrict__ hi) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)R * n) return;
    const int l = (int)(t / n), row = (int)(t - (size_t)l * n);
    const float* d = D + t * n;
    int first = -1, last = -1;
    for (int c = 0; c < n; ++c)
        if (d[c] != 0.f) {
            if (first < 0) first = c;
            last = c;
        }
    if (first < 0) return;
    const int nb = (n + kTgRows - 1) / kTgRows;
    atomicMin(lo + (size_t)l * nb + row / kTgRows, first);
    atomicMax(hi + (size_t)l * nb + row / kTgRows, last);
}

// 16-column groups [g0, g1) of row block b (empty when the block is all zero)
__device__ inline void band_groups(const int* lo, const int* hi, size_t b, int& g0, int& g1) {
    const int h = hi[b];
    g0 = h < 0 ? 0 : lo[b] >> 4;
    g1 = h < 0 ? 0 : (h >> 4) + 1;
}

// Four consecutive values v[i], i = k..k+3, of a row of length n.  The
// loads are unconditional (from a clamped index) so that no branch sits
// around a load and the wait before the products covers only the loads they
// use.  MODE 2: n a multiple of 16, so no group of 16 runs past n, and a
// dead row or column (its pointer a valid one) is loaded as is: its products
// land only in rows or columns of Y1 and Y2 that are never stored or read.
// MODE 1: n a multiple of 4, one 16-byte load, zero past n or for a dead
// row; MODE 0: element loads, zero past n or for a dead row.
template <int MODE>
__device__ inline tgf4 load4(const float* __restrict__ row, int k, int n, bool live) {
    if constexpr (MODE == 2) {
        return *(const tgf4*)(row + k);
    } else if constexpr (MODE == 1) {
        const bool ok = live && k < n;
        const tgf4 v = *(const tgf4*)(row + (ok ? k : 0));
        return ok ? v : tgf4{0.f, 0.f, 0.f, 0.f};
    } else {
        tgf4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ok = live && k + e < n;
            const float x = row[ok ? k + e : 0];
            v[e] = ok ? x : 0.f;
        }
        return v;
    }
}

// 16 MFMAs per k-slot j: the 4 x 4 tiles of 16 x 16 of a wave
__device__ inline void mfma_group(tgf4 (&acc)[4][4], const tgf4 (&a)[4], const tgf4 (&b)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][j], b[ct][j], acc[rt][ct], 0, 0, 0);
}

// Operands of group g (k = 16 g + 4 (lane / 16)) from global rows / columns
template <int MODE>
__device__ inline void load_rows(const float* const (&p)[4], const bool (&live)[4], int k, int n, tgf4 (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = load4<MODE>(p[i], k, n, live[i]);
}

// the row tiles of Y1 for group g from LDS
__device__ inline void read_y1(const float* y1s, int ld, int lr, int k, tgf4 (&v)[4]) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) v[rt] = *(const tgf4*)(y1s + (16 * rt + lr) * ld + k);
}

// Y2[l](:,:,k) rows [64 rb, 64 rb + 64) for every (rb, k, l), one workgroup
// each (grid x = ceil(n1 / 64) n3 R).  D1 [R][n1][n1] and D2
// [R][n2][n2] row-major (entry (i', i) at i + i' n), M [n3][n2][n1], Y2
// [R][n3][n2][n1]; lo1/hi1 [R][ceil(n1/64)], lo2/hi2 [R][ceil(n2/64)] the
// bands of D1 and D2.  LDS: 64 rows of Y1, ld = 16 ceil(n2/16) + 4 floats.
// Each wave owns four column tiles per pass of 16 tiles.
template <int MODE>
__global__ void __launch_bounds__(256) k_tg_mode12(int n1, int n2, int n3, int R, const float* __restrict__ D1,
                                                   const int* __restrict__ lo1, const int* __restrict__ hi1,
                                                   const float* __restrict__ M, const float* __restrict__ D2,
                                                   const int* __restrict__ lo2, const int* __restrict__ hi2,
                                                   float* __restrict__ Y2) {
    extern __shared__ __align__(16) float y1s[];
    const int nb1 = (n1 + kTgRows - 1) / kTgRows, nb2 = (n2 + kTgRows - 1) / kTgRows;
    const int nct = (n2 + 15) >> 4, ld = 16 * nct + 4;
    // workgroup b runs on XCD b % 8: give each XCD a contiguous range of work,
    // (node, plane, row block) with the row blocks, then the planes of one node
    // adjacent, so that an XCD's L2 holds the node's matrices
    const unsigned T = gridDim.x, b = blockIdx.x, q = T >> 3, r = T & 7, x = b & 7, s = b >> 3;
    const unsigned lg = x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
    const int rb = (int)(lg % (unsigned)nb1);
    const unsigned rest = lg / (unsigned)nb1;
    const int kz = (int)(rest % (unsigned)n3), L = (int)(rest / (unsigned)n3);
    // the nodes in the order 0, 8, 16, ..., 1, 9, ...: the banded (cheap) nodes are the
    // last ones, so every XCD's range samples the whole range of costs
    const int q8 = R >> 3, r8 = R & 7, big = r8 * (q8 + 1);
    const int l = L < big ? L / (q8 + 1) + 8 * (L % (q8 + 1))
                          : r8 + (L - big) / (q8 > 0 ? q8 : 1) + 8 * ((L - big) % (q8 > 0 ? q8 : 1));
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, lr = lane & 15, kq = lane >> 4;
    const size_t plane = (size_t)n1 * n2;
    const float* A1 = D1 + (size_t)l * n1 * n1;
    const float* B2 = D2 + (size_t)l * n2 * n2;
    const int npass = (nct + 15) >> 4;  // at most 2 (n2 <= 512)
    // bands: of this row block of D1, and of the wave's blocks of 64 columns of D2
    int g0, g1, h0[2], h1[2];
    band_groups(lo1, hi1, (size_t)l * nb1 + rb, g0, g1);
#pragma unroll
    for (int cp = 0; cp < 2; ++cp) {
        const int cb = 4 * cp + w;
        if (cb < nb2) band_groups(lo2, hi2, (size_t)l * nb2 + cb, h0[cp], h1[cp]);
        else h0[cp] = h1[cp] = 0;
    }
    const float* arow[4];
    bool alive[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int row = kTgRows * rb + 16 * rt + lr;
        alive[rt] = row < n1;
        arow[rt] = A1 + (size_t)(alive[rt] ? row : 0) * n1;
    }
    const float* Mk = M + (size_t)kz * plane;

    // ---- Y1 = D1[l](rows, :) M(:, :, k) into LDS
    for (int cp = 0; cp < npass; ++cp) {
        if (16 * cp + 4 * w >= nct) break;  // no column tile of this wave left
        const float* bcol[4];
        bool blive[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int c = 16 * (16 * cp + 4 * w + ct) + lr;
            blive[ct] = c < n2;
            bcol[ct] = Mk + (size_t)(blive[ct] ? c : 0) * n1;
        }
        tgf4 acc[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = tgf4{0.f, 0.f, 0.f, 0.f};
        // two operand sets in turn: the loads of one group are in flight during the
        // products of the other (a group past the end is loaded again as the last)
        tgf4 a0[4] = {}, b0[4] = {}, a1[4], b1[4];
        if (g0 < g1) {
            load_rows<MODE>(arow, alive, 16 * g0 + 4 * kq, n1, a0);
            load_rows<MODE>(bcol, blive, 16 * g0 + 4 * kq, n1, b0);
        }
        int g = g0;
        for (; g + 1 < g1; g += 2) {
            load_rows<MODE>(arow, alive, 16 * (g + 1) + 4 * kq, n1, a1);
            load_rows<MODE>(bcol, blive, 16 * (g + 1) + 4 * kq, n1, b1);
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the products
            mfma_group(acc, a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            const int k2 = 16 * (g + 2 < g1 ? g + 2 : g1 - 1) + 4 * kq;
            load_rows<MODE>(arow, alive, k2, n1, a0);
            load_rows<MODE>(bcol, blive, k2, n1, b0);
            __builtin_amdgcn_sched_barrier(0);
            mfma_group(acc, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (g < g1) mfma_group(acc, a0, b0);
        // accumulator: lane holds rows 4 (lane / 16) + v of column lane % 16 of each tile
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int t = 16 * cp + 4 * w + ct;
            if (t < nct) {
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) y1s[(16 * rt + 4 * kq + v) * ld + 16 * t + lr] = acc[rt][ct][v];
            }
        }
    }
    __syncthreads();

    // ---- Y2(rows, :) = Y1 D2[l]^T: columns of Y2 are rows of D2
    const size_t obase = (size_t)l * n3 * plane + (size_t)kz * plane;
    for (int cp = 0; cp < npass; ++cp) {
        const int cb = 4 * cp + w;  // this wave's block of 64 columns
        if (cb >= nb2) break;
        const int f0 = h0[cp], f1 = h1[cp];
        const float* bcol[4];
        bool blive[4];
        int cols[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int c = 16 * (16 * cp + 4 * w + ct) + lr;
            cols[ct] = c;
            blive[ct] = c < n2;
            bcol[ct] = B2 + (size_t)(blive[ct] ? c : 0) * n2;
        }
        tgf4 acc[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = tgf4{0.f, 0.f, 0.f, 0.f};
        tgf4 a0[4] = {}, b0[4] = {}, a1[4], b1[4];
        if (f0 < f1) {
            load_rows<MODE>(bcol, blive, 16 * f0 + 4 * kq, n2, b0);
            read_y1(y1s, ld, lr, 16 * f0 + 4 * kq, a0);
        }
        int g = f0;
        for (; g + 1 < f1; g += 2) {
            load_rows<MODE>(bcol, blive, 16 * (g + 1) + 4 * kq, n2, b1);
            read_y1(y1s, ld, lr, 16 * (g + 1) + 4 * kq, a1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_group(acc, a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            const int k2 = 16 * (g + 2 < f1 ? g + 2 : f1 - 1) + 4 * kq;
            load_rows<MODE>(bcol, blive, k2, n2, b0);
            read_y1(y1s, ld, lr, k2, a0);
            __builtin_amdgcn_sched_barrier(0);
            mfma_group(acc, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (g < f1) mfma_group(acc, a0, b0);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            if (!blive[ct]) continue;
            float* out = Y2 + obase + (size_t)cols[ct] * n1;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
                const int row = kTgRows * rb + 16 * rt + 4 * kq;
                if constexpr (MODE > 0) {
                    if (row < n1) *(tgf4*)(out + row) = acc[rt][ct];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (row + v < n1) out[row + v] = acc[rt][ct][v];
                }
            }
        }
    }
}

size_t mode12_lds(int n2) { return (size_t)kTgRows * (16 * ((n2 + 15) / 16) + 4) * sizeof(float); }

}  // namespace

bool tg_mode12_fits(int n2) { return n2 >= 1 && mode12_lds(n2) <= 160 * 1024 && n2 <= kTgMode12MaxN2; }

int tg_band_blocks(int n) { return (n + kTgRows - 1) / kTgRows; }

hipError_t tg_mode12_init(int n2) {
    const int lds = (int)mode12_lds(n2);
    const void* k[3] = {(const void*)k_tg_mode12<0>, (const void*)k_tg_mode12<1>, (const void*)k_tg_mode12<2>};
    for (const void* f : k) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tg_band(hipStream_t st, int n, int R, const float* D, int* lo, int* hi) {
    const size_t nb = (size_t)R * tg_band_blocks(n);
    hipError_t e = hipMemsetAsync(lo, 0x7F, nb * sizeof(int), st);
    if (e == hipSuccess) e = hipMemsetAsync(hi, 0xFF, nb * sizeof(int), st);
    if (e != hipSuccess) return e;
    const size_t total = (size_t)R * n;
    hipLaunchKernelGGL(k_tg_band, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, R, D, lo, hi);
    return hipGetLastError();
}

hipError_t launch_tg_mode12(hipStream_t st, int n1, int n2, int n3, int R, const float* D1, const int* lo1,
                            const int* hi1, const float* M, const float* D2, const int* lo2, const int* hi2,
                            float* Y2) {
    if (n1 < 1 || n2 < 1 || n3 < 1 || R < 1 || !tg_mode12_fits(n2)) return hipErrorInvalidValue;
    const size_t grid = (size_t)tg_band_blocks(n1) * n3 * R;
    if (grid > 0x7FFFFFFFu) return hipErrorInvalidValue;
    const size_t lds = mode12_lds(n2);
    const dim3 gr((unsigned)grid), bl(256);
    if ((n1 & 15) == 0 && (n2 & 15) == 0)
        hipLaunchKernelGGL(k_tg_mode12<2>, gr, bl, lds, st, n1, n2, n3, R, D1, lo1, hi1, M, D2, lo2, hi2, Y2);
    else if ((n1 & 3) == 0 && (n2 & 3) == 0)
        hipLaunchKernelGGL(k_tg_mode12<1>, gr, bl, lds, st, n1, n2, n3, R, D1, lo1, hi1, M, D2, lo2, hi2, Y2);
    else
        hipLaunchKernelGGL(k_tg_mode12<0>, gr, bl, lds, st, n1, n2, n3, R, D1, lo1, hi1, M, D2, lo2, hi2, Y2);
    return hipGetLastError();
}

}  // namespace demag
