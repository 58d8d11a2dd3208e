// Fused first and second mode products of the tensor-grid sum (Sec. 3.2, eq.
// (sumpot)) in FP32 on the matrix cores.
//
// For node l, z-plane k and magnetization component p the sum needs
//     Y2[l](:,:,k) = D_1[l] M_p(:,:,k) D_2[l]^T            (n1 x n2)
// before the third mode product and the node sum (a GEMM with inner
// dimension R n3, left to the caller).  One workgroup computes 64 rows of
// Y2[l](:,:,k): first the 64 x n2 block of Y1 = D_1 M in registers and then
// in LDS, then Y1 D_2^T from LDS, so the intermediate Y1 (R N values per
// component) never reaches HBM.  Both products run on v_mfma_f32_16x16x4f32;
// a lane's four consecutive k values (one 16-byte load) feed four
// instructions, instruction j taking k = 16 g + 4 (lane / 16) + j of the
// group g of 16, the same permutation of k on both operands, so the sum over
// a group is complete.  The Gaussian matrices are stored at set-up in that
// operand order, one contiguous 1 KB run per tile of 16 x 16 (k_tg_axis_sw),
// so that a wave loads a tile with one fully used 1 KB access; the
// magnetization is read in place (its columns, 64 bytes per row and load).
//
// The Gaussian matrices of the nodes with large tau are banded: their
// entries far from the diagonal are exactly zero in FP32.  For every block of
// 64 rows the range of 16-column groups holding a nonzero entry is found once
// at set-up (k_tg_band) and the products skip the groups outside it, which
// only drops products with exact zeros (the sums are unchanged for finite m).
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "tg_gauss.hpp"

namespace demag {

namespace {

typedef float tgf4 __attribute__((ext_vector_type(4)));

constexpr int kTgRows = 64;  // rows of Y2 per workgroup (four MFMA row tiles)
static_assert(kTgMode12MaxN2 <= 512, "a wave holds the bands of at most two passes of 16 column tiles");

__host__ __device__ inline int tiles16(int n) { return (n + 15) / 16; }

// Offset of entry (row, col) of a matrix with G = ceil(n / 16) tiles per side
// in the tiled operand order: tile (row / 16, col / 16) at (tr G + g) 256,
// lane = row % 16 + 16 ((col % 16) / 4), element col % 4.
__host__ __device__ inline size_t sw_offset(int row, int col, int G) {
    const int tile = (row >> 4) * G + (col >> 4), lane = (row & 15) + 16 * ((col & 15) >> 2);
    return ((size_t)tile * 64 + lane) * 4 + (col & 3);
}

// Gaussian matrices of one axis (n cells of edge d, reduced units), every node,
// in the tiled operand order (G x G tiles of 256 values per node), zero
// outside n x n: E(i', i) and O(i', i) at row i' (target), column i (source).
__global__ void __launch_bounds__(256) k_tg_axis_sw(int n, double d, int R, const double* __restrict__ tau,
                                                    float* __restrict__ E, float* __restrict__ O) {
    const int G = tiles16(n);
    const size_t per = (size_t)G * G * 256;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per * R) return;
    const int l = (int)(t / per);
    const size_t e = t - (size_t)l * per;
    const int elem = (int)(e & 3), lane = (int)((e >> 2) & 63);
    const size_t tile = e >> 8;
    const int row = 16 * (int)(tile / G) + (lane & 15), col = 16 * (int)(tile % G) + 4 * (lane >> 4) + elem;
    float ev = 0.f, ov = 0.f;
    if (row < n && col < n) {
        const double a = (row + 0.5) * d, c = (col + 0.5) * d, s = tau[l];
        ev = (float)gauss_even(a, c, d, s);
        ov = (float)gauss_odd(a, c, d, s);
    }
    E[t] = ev;
    O[t] = ov;
}

// Columns [lo, hi] holding a nonzero entry of each row block of 64 of the
// tiled matrices (lo starts above any column, hi at -1).
__global__ void __launch_bounds__(256) k_tg_band(int n, int R, const float* __restrict__ D, int* __restrict__ lo,
                                                 int* __restrict__ hi) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)R * n) return;
    const int l = (int)(t / n), row = (int)(t - (size_t)l * n), G = tiles16(n);
    const float* d = D + (size_t)l * G * G * 256;
    int first = -1, last = -1;
    for (int c = 0; c < n; ++c)
        if (d[sw_offset(row, c, G)] != 0.f) {
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

// Four consecutive values v[i], i = k..k+3, of a column of the magnetization
// of length n.  The loads are unconditional (from a clamped index) so that no
// branch sits around a load and the wait before the products covers only the
// loads they use.  MODE 2: n a multiple of 16, so no group of 16 runs past n,
// and a dead column (its pointer a valid one) is loaded as is: its products
// land only in columns of Y1 that are never stored.  MODE 1: n a multiple of
// 4, one 16-byte load, zero past n or for a dead column; MODE 0: element
// loads, zero past n or for a dead column.
template <int MODE>
__device__ inline tgf4 load4(const float* __restrict__ col, int k, int n, bool live) {
    if constexpr (MODE == 2) {
        return *(const tgf4*)(col + k);
    } else if constexpr (MODE == 1) {
        const bool ok = live && k < n;
        const tgf4 v = *(const tgf4*)(col + (ok ? k : 0));
        return ok ? v : tgf4{0.f, 0.f, 0.f, 0.f};
    } else {
        tgf4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool ok = live && k + e < n;
            const float x = col[ok ? k + e : 0];
            v[e] = ok ? x : 0.f;
        }
        return v;
    }
}

template <int MODE>
__device__ inline void load_cols(const float* const (&p)[4], const bool (&live)[4], int k, int n, tgf4 (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = load4<MODE>(p[i], k, n, live[i]);
}

// the lane's values of group g of four tiles of a tiled matrix (p: the tiles'
// first group, lane offset included); zero padding makes every group valid
__device__ inline void load_tiles(const float* const (&p)[4], int g, tgf4 (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = *(const tgf4*)(p[i] + (size_t)g * 256);
}

// the row tiles of Y1 for group g from LDS
__device__ inline void read_y1(const float* y1s, int ld, int lr, int k, tgf4 (&v)[4]) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) v[rt] = *(const tgf4*)(y1s + (16 * rt + lr) * ld + k);
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

// Y2[l](:,:,k) rows [64 rb, 64 rb + 64) for every (rb, k, l), one workgroup
// each (grid x = ceil(n1 / 64) n3 R).  D1 and D2 tiled (k_tg_axis_sw), M
// [n3][n2][n1], Y2 [R][n3][n2][n1]; lo1/hi1 [R][ceil(n1/64)], lo2/hi2
// [R][ceil(n2/64)] the bands of D1 and D2.  LDS: 64 rows of Y1, ld =
// 16 ceil(n2/16) + 4 floats.  Each wave owns four column tiles per pass of 16
// tiles.  A row or column tile past the matrix reads the last tile (its
// products land only in outputs that are neither stored nor read).
template <int MODE>
__global__ void __launch_bounds__(256, 2) k_tg_mode12(int n1, int n2, int n3, int R, const float* __restrict__ D1,
                                                   const int* __restrict__ lo1, const int* __restrict__ hi1,
                                                   const float* __restrict__ M, const float* __restrict__ D2,
                                                   const int* __restrict__ lo2, const int* __restrict__ hi2,
                                                   float* __restrict__ Y2) {
    extern __shared__ __align__(16) float y1s[];
    const int nb1 = (n1 + kTgRows - 1) / kTgRows, nb2 = (n2 + kTgRows - 1) / kTgRows;
    const int G1 = tiles16(n1), G2 = tiles16(n2);
    const int nct = G2, ld = 16 * nct + 4;
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
    const float* A1 = D1 + (size_t)l * G1 * G1 * 256;
    const float* B2 = D2 + (size_t)l * G2 * G2 * 256;
    const float* Mk = M + (size_t)kz * plane;
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
    const float* atile[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int tr = min(4 * rb + rt, G1 - 1);
        atile[rt] = A1 + ((size_t)tr * G1 * 64 + lane) * 4;
    }

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
        // products of the other (a group past the end is loaded again as the last);
        // the scheduling groups spread those loads through the products, one load
        // per eight MFMAs, instead of one burst ahead of them (an idle matrix unit
        // while the burst issues)
        tgf4 a0[4] = {}, b0[4] = {}, a1[4], b1[4];
        if (g0 < g1) {
            load_tiles(atile, g0, a0);
            load_cols<MODE>(bcol, blive, 16 * g0 + 4 * kq, n1, b0);
        }
        int g = g0;
        for (; g + 1 < g1; g += 2) {
            load_cols<MODE>(bcol, blive, 16 * (g + 1) + 4 * kq, n1, b1);
            load_tiles(atile, g + 1, a1);
            mfma_group(acc, a0, b0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            const int g2 = g + 2 < g1 ? g + 2 : g1 - 1;
            load_cols<MODE>(bcol, blive, 16 * g2 + 4 * kq, n1, b0);
            load_tiles(atile, g2, a0);
            mfma_group(acc, a1, b1);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
            }
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
        const float* btile[4];
        int cols[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int t = 16 * cp + 4 * w + ct;
            cols[ct] = 16 * t + lr;
            btile[ct] = B2 + ((size_t)min(t, G2 - 1) * G2 * 64 + lane) * 4;
        }
        tgf4 acc[4][4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = tgf4{0.f, 0.f, 0.f, 0.f};
        // as in the first product; the global and LDS loads alternate, each ahead of
        // eight MFMAs
        tgf4 a0[4] = {}, b0[4] = {}, a1[4], b1[4];
        if (f0 < f1) {
            load_tiles(btile, f0, b0);
            read_y1(y1s, ld, lr, 16 * f0 + 4 * kq, a0);
        }
        int g = f0;
        for (; g + 1 < f1; g += 2) {
            load_tiles(btile, g + 1, b1);
            read_y1(y1s, ld, lr, 16 * (g + 1) + 4 * kq, a1);
            mfma_group(acc, a0, b0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            const int g2 = g + 2 < f1 ? g + 2 : f1 - 1;
            load_tiles(btile, g2, b0);
            read_y1(y1s, ld, lr, 16 * g2 + 4 * kq, a0);
            mfma_group(acc, a1, b1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        if (g < f1) mfma_group(acc, a0, b0);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            if (cols[ct] >= n2) continue;
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

size_t mode12_lds(int n2) { return (size_t)kTgRows * (16 * tiles16(n2) + 4) * sizeof(float); }

}  // namespace

bool tg_mode12_fits(int n2) { return n2 >= 1 && mode12_lds(n2) <= 160 * 1024 && n2 <= kTgMode12MaxN2; }

int tg_band_blocks(int n) { return (n + kTgRows - 1) / kTgRows; }

size_t tg_tiled_floats(int n) { return (size_t)tiles16(n) * tiles16(n) * 256; }

hipError_t tg_mode12_init(int n2) {
    const int lds = (int)mode12_lds(n2);
    const void* k[3] = {(const void*)k_tg_mode12<0>, (const void*)k_tg_mode12<1>, (const void*)k_tg_mode12<2>};
    for (const void* f : k) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_tg_axis_tiled(hipStream_t st, int n, double d, int R, const double* tau, float* E, float* O) {
    const size_t total = tg_tiled_floats(n) * R;
    hipLaunchKernelGGL(k_tg_axis_sw, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, d, R, tau, E, O);
    return hipGetLastError();
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
