// Scalar-potential (SP) method: FP64 setup of the kernel spectrum and the
// finite-difference gradient (Sec. 3.1, eqs. (scpot), (convolution), (field)).
//
// phi = Ms S * m with S_a(R) the potential at R of a cell centred at the
// origin and magnetized along axis a with unit magnetization; H = -grad phi.
// Integrating eq. (scpot) along a turns the cell into two charged faces,
//     S_a(R) = (1/4pi) [ G_a(R - (d_a/2) e_a) - G_a(R + (d_a/2) e_a) ],
// G_a the potential of the unit-density d_b x d_c rectangle (closed form: the
// corner sum of u asinh(v/sqrt(u^2+w^2)) + v asinh(u/sqrt(v^2+w^2))
// - w atan(uv/(w r))).  As for the DM tensor, three routes by distance:
//   near (Chebyshev distance <= fg_cut): that closed form;
//   mid:  Gauss-Legendre of the defining volume integral
//         S_a(R) = (1/4pi) int_cell (R_a - u_a) / |R - u|^3 du (the pole is
//         outside the cell; panels no longer than its distance to the cell);
//   far  (rho >= far_cut): S_a = -(V/4pi) sum_beta c_beta d^(beta + e_a)(1/r)
//         over even multi-indices |beta| <= 6, c_beta the moments of the
//         uniform cell (d^2/12, d^4/80, d^6/448) over beta!.
// S_a is odd in axis a and even in the others; its transform is imaginary.
// The spectrum stored is Im(S^) on the octant with +1/(Px Py Pz) folded in,
// layout [Kx][Py/2+1][3][Pz/2+1].
#include <algorithm>
#include <climits>

#include "internal.hpp"
#include "newell.hpp"

namespace demag {

namespace {

constexpr double kPi = newell::kPi;

// ---- near: charged faces ---------------------------------------------------
__device__ double face_F(double u, double v, double w) {
    const double r = sqrt(u * u + v * v + w * w);
    double t = newell::asinh_term(u, v, u * u + w * w) + newell::asinh_term(v, u, v * v + w * w);
    if (w != 0.0 && u != 0.0 && v != 0.0) t -= w * atan(u * v / (w * r));
    return t;
}

// potential at (X, Y, W) of the unit-density rectangle A x B centred at 0 in the plane W = 0
__device__ double face_G(double X, double Y, double W, double A, double B) {
    const double u1 = -0.5 * A - X, u2 = 0.5 * A - X, v1 = -0.5 * B - Y, v2 = 0.5 * B - Y;
    return face_F(u2, v2, W) - face_F(u1, v2, W) - face_F(u2, v1, W) + face_F(u1, v1, W);
}

__device__ void sp_near(const double R[3], const double dt[3], double out[3]) {
    for (int a = 0; a < 3; ++a) {
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const double top = face_G(R[b], R[c], R[a] - 0.5 * dt[a], dt[b], dt[c]);
        const double bot = face_G(R[b], R[c], R[a] + 0.5 * dt[a], dt[b], dt[c]);
        out[a] = (top - bot) / (4.0 * kPi);
    }
}

// ---- far: moment series ----------------------------------------------------
// average of s^p over [-d/2, d/2], p even
__device__ double uniform_moment(int p, double d) {
    return p == 0 ? 1.0 : pow(0.5 * d, (double)p) / (p + 1.0);
}

__device__ void sp_far(const double R[3], const double dt[3], double out[3]) {
    double a[newell::kTaylorLen];
    newell::inv_r_taylor(R[0], R[1], R[2], a);
    out[0] = out[1] = out[2] = 0.0;
    for (int bx = 0; bx <= 6; bx += 2)
        for (int by = 0; by <= 6 - bx; by += 2)
            for (int bz = 0; bz <= 6 - bx - by; bz += 2) {
                const double cb = uniform_moment(bx, dt[0]) / newell::fact(bx) * uniform_moment(by, dt[1]) /
                                  newell::fact(by) * uniform_moment(bz, dt[2]) / newell::fact(bz);
                for (int c = 0; c < 3; ++c) {
                    int g[3] = {bx, by, bz};
                    g[c] += 1;
                    out[c] += cb * newell::fact(g[0]) * newell::fact(g[1]) * newell::fact(g[2]) *
                              a[newell::tidx(g[0], g[1], g[2])];
                }
            }
    const double V = dt[0] * dt[1] * dt[2];
    for (int c = 0; c < 3; ++c) out[c] *= -V / (4.0 * kPi);
}

__device__ __forceinline__ bool sp_in_far(const double R[3], double far_cut) {
    return R[0] * R[0] + R[1] * R[1] + R[2] * R[2] >= far_cut * far_cut;
}

// distance from the point R to the cell [-d/2, d/2]^3
__device__ double point_gap(const double R[3], const double dt[3]) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double g = fabs(R[k]) - 0.5 * dt[k];
        if (g > 0) s += g * g;
    }
    return sqrt(s);
}

// Near and far bands: one thread per octant offset.
__global__ void __launch_bounds__(256) k_sp_pointwise(size_t base, int nx, int ny, int nz, double dt0, double dt1,
                                                      double dt2, double far_cut, int fg_cut,
                                                      double* __restrict__ Soct) {
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    const int ox = (int)(t % nx), oy = (int)((t / nx) % ny), oz = (int)(t / ((size_t)nx * ny));
    const double dt[3] = {dt0, dt1, dt2};
    const double R[3] = {ox * dt0, oy * dt1, oz * dt2};
    double v[3];
    if (max(ox, max(oy, oz)) <= fg_cut) {
        sp_near(R, dt, v);
    } else if (sp_in_far(R, far_cut)) {
        sp_far(R, dt, v);
    } else {
        return;  // mid band: k_sp_mid
    }
    for (int c = 0; c < 3; ++c) Soct[c * ncell + t] = v[c];
}

// Mid band: one 64-lane workgroup per offset of the bounding box
// [0,bx) x [0,by) x [0,bz); offsets outside the band return at once.
__global__ void __launch_bounds__(64) k_sp_mid(long base, int nx, int ny, int nz, int bx, int by, double dt0, double dt1,
                                               double dt2, double far_cut, int fg_cut, int q, int max_panels,
                                               const double* __restrict__ gl_x, const double* __restrict__ gl_w,
                                               double* __restrict__ Soct) {
    const long b = base + blockIdx.x;
    const int ox = (int)(b % bx), oy = (int)((b / bx) % by), oz = (int)(b / ((long)bx * by));
    if (ox >= nx || oy >= ny || oz >= nz) return;
    const double dt[3] = {dt0, dt1, dt2};
    const double R[3] = {ox * dt0, oy * dt1, oz * dt2};
    if (max(ox, max(oy, oz)) <= fg_cut || sp_in_far(R, far_cut)) return;
    const double gap = point_gap(R, dt);
    int m[3], Q[3];
    for (int k = 0; k < 3; ++k) {
        m[k] = newell::mid_panels(dt[k], gap, max_panels);
        Q[k] = m[k] * q;
    }
    double acc[3] = {0, 0, 0};
    const int total = Q[0] * Q[1] * Q[2];
    for (int n = threadIdx.x; n < total; n += 64) {
        const int idx[3] = {n % Q[0], (n / Q[0]) % Q[1], n / (Q[0] * Q[1])};
        double u[3], w = 1.0;
        for (int k = 0; k < 3; ++k) {  // panel p, node j of axis k on [-d/2, d/2]
            const int p = idx[k] / q, j = idx[k] - p * q;
            const double h = dt[k] / m[k];
            u[k] = -0.5 * dt[k] + p * h + 0.5 * h * (gl_x[j] + 1.0);
            w *= 0.5 * h * gl_w[j];
        }
        const double X = R[0] - u[0], Y = R[1] - u[1], Z = R[2] - u[2];
        const double r2 = X * X + Y * Y + Z * Z;
        const double ir = 1.0 / sqrt(r2);
        const double f = w * ir * ir * ir / (4.0 * kPi);
        acc[0] += X * f;
        acc[1] += Y * f;
        acc[2] += Z * f;
    }
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t t = ((size_t)oz * ny + oy) * nx + ox;
    for (int c = 0; c < 3; ++c) {
        double s = acc[c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (threadIdx.x == 0) Soct[c * ncell + t] = s;
    }
}

// Signed offset of padded index i (period P, n valid offsets each side), or
// a flag for the zero gap.
__device__ __forceinline__ bool unpad_sp(int i, int n, int P, int* o) {
    if (i < n) { *o = i; return true; }
    if (i > P - n) { *o = i - P; return true; }
    return false;
}

// component a of the octant mirrored into the P-periodic array (odd in axis a)
__global__ void __launch_bounds__(256) k_sp_embed(size_t base, int a, int nx, int ny, int nz, int Px, int Py, int Pz,
                                                  const double* __restrict__ Soct, double* __restrict__ A) {
    const size_t total = (size_t)Px * Py * Pz;
    const size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int x = (int)(t % Px), y = (int)((t / Px) % Py), z = (int)(t / ((size_t)Px * Py));
    int o[3];
    double v = 0.0;
    if (unpad_sp(x, nx, Px, &o[0]) && unpad_sp(y, ny, Py, &o[1]) && unpad_sp(z, nz, Pz, &o[2])) {
        const size_t ncell = (size_t)nx * ny * nz;
        v = Soct[a * ncell + ((size_t)abs(o[2]) * ny + abs(o[1])) * nx + abs(o[0])];
        if (o[a] < 0) v = -v;
    }
    A[t] = v;
}

// Im of the transform on the octant, scaled; the transform of a function odd
// in axis a vanishes on that axis's Nyquist plane: stored as an exact zero.
template <typename T>
__global__ void __launch_bounds__(256) k_sp_extract(size_t base, int a, int Py, int Pz, int Kx, double scale,
                                                    const cx<double>* __restrict__ B2, T* __restrict__ shat) {
    const int Ly = Py / 2, Lz = Pz / 2;
    const size_t total = (size_t)(Ly + 1) * Kx * (Lz + 1);
    const size_t t = base + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int kz = (int)(t % (Lz + 1)), ky = (int)((t / (Lz + 1)) % (Ly + 1)),
              kx = (int)(t / ((size_t)(Lz + 1) * (Ly + 1)));
    double v = B2[((size_t)kx * Py + ky) * Pz + kz].im * scale;  // B2 [Kx][Py][Pz]
    if ((a == 0 && kx == Kx - 1) || (a == 1 && ky == Ly) || (a == 2 && kz == Lz)) v = 0.0;
    shat[(((size_t)kx * (Ly + 1) + ky) * 3 + a) * (Lz + 1) + kz] = (T)v;  // [Kx][Ly+1][3][Lz+1]
}

// ---- field: H = -grad phi (eq. (field)) ---------------------------------------
// -d phi / d axis at index i of n from the five values around it (pm2 at
// i - 2 ... p2 at i + 2; only those inside the grid are used), r2h = 1/(2h):
// central inside, second-order one-sided on the faces, first order for n = 2,
// 0 for n = 1; chosen by selects, so that a face needs no branch.
template <typename T>
__device__ __forceinline__ T minus_d5(T pm2, T pm1, T p0, T p1, T p2, int i, int n, T r2h) {
    const T central = -(p1 - pm1) * r2h;
    const T first = -(T(-3) * p0 + T(4) * p1 - p2) * r2h;  // i = 0
    const T last = -(T(3) * p0 - T(4) * pm1 + pm2) * r2h;  // i = n - 1
    const T two = i == 0 ? -(p1 - p0) * (T(2) * r2h) : -(p0 - pm1) * (T(2) * r2h);
    const T d = i == 0 ? first : i == n - 1 ? last : central;
    return n == 1 ? T(0) : n == 2 ? two : d;
}

// Tiled gradient.  A workgroup owns a kGX x kGY cell tile of a z-chunk
// [z0, z0 + zc); thread (lx, ly) owns x = x0 + lx and the rows y0 + ly + 4 r
// (r < kGR) and walks z with phi at z - 2 ... z + 2 of its cells in registers
// (each plane is read once, three planes ahead of its use).  The plane's tile
// with a two-cell halo in x and y is staged in LDS, double-buffered, one
// barrier per plane; every stencil, the one-sided ones of the faces included,
// then reads LDS and registers only.  Addresses: a workgroup-uniform plane
// pointer plus a 32-bit in-plane offset per lane; a lane with nothing to load
// reads its plane's first cell and discards it.  Optional energy: one FP64
// partial of m.H per workgroup.
constexpr int kGX = 64, kGR = 4, kGY = 4 * kGR, kGH = 2;

template <typename T>
__global__ void __launch_bounds__(256) k_sp_gradient(int nx, int ny, int nz, int zc, T dx, T dy, T dz,
                                                     const T* __restrict__ phi, T* __restrict__ H,
                                                     const T* __restrict__ m, double* __restrict__ partials) {
    constexpr int TW = kGX + 2 * kGH, TH = kGY + 2 * kGH;
    __shared__ T tile[2][TH][TW];
    __shared__ double red[4];
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int ntx = (nx + kGX - 1) / kGX, nty = (ny + kGY - 1) / kGY;
    const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty, bz = blockIdx.x / (ntx * nty);
    const int x0 = bx * kGX, y0 = by * kGY, z0 = bz * zc, z1 = min(nz, z0 + zc);
    const int x = x0 + lx;
    const size_t sxy = (size_t)nx * ny, N = sxy * nz;
    auto plane = [&](const T* a, int zz) { return a + (size_t)min(max(zz, 0), nz - 1) * sxy; };
    auto ld = [&](const T* a, int zz, unsigned off, bool valid) {
        const T v = plane(a, zz)[off];
        return valid ? v : T(0);
    };
    bool ok[kGR];
    unsigned oc[kGR];
#pragma unroll
    for (int r = 0; r < kGR; ++r) {
        const int y = y0 + ly + 4 * r;
        ok[r] = x < nx && y < ny;
        oc[r] = ok[r] ? (unsigned)y * (unsigned)nx + (unsigned)x : 0u;
    }
    // halo: rows y0 - 2, y0 - 1, y0 + kGY, y0 + kGY + 1 (one per ly, column x);
    // columns x0 - 2, x0 - 1, x0 + kGX, x0 + kGX + 1 (ly = 0: lx / 16, row y0 + lx % 16)
    const int hry = ly < 2 ? y0 - kGH + ly : y0 + kGY + (ly - 2);
    const bool hrv = x < nx && hry >= 0 && hry < ny;
    const unsigned ohr = hrv ? (unsigned)hry * (unsigned)nx + (unsigned)x : 0u;
    const int hrt = ly < 2 ? ly : kGY + kGH + (ly - 2);  // its tile row
    const int hk = lx >> 4;
    const int hcx = hk < 2 ? x0 - kGH + hk : x0 + kGX + (hk - 2), hcy = y0 + (lx & 15);
    const bool hcv = ly == 0 && hcx >= 0 && hcx < nx && hcy < ny;
    const unsigned ohc = hcv ? (unsigned)hcy * (unsigned)nx + (unsigned)hcx : 0u;
    const int hct = hk < 2 ? hk : kGX + kGH + (hk - 2);  // its tile column
    T w[5][kGR];  // phi at z - 2 ... z + 2
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int r = 0; r < kGR; ++r) {
            const int zz = z0 - 2 + k;
            w[k][r] = ld(phi, zz, oc[r], ok[r] && zz >= 0 && zz < nz);
        }
    T hr = ld(phi, z0, ohr, hrv), hc = ld(phi, z0, ohc, hcv);
    const T rx = T(1) / (T(2) * dx), ry = T(1) / (T(2) * dy), rz = T(1) / (T(2) * dz);
    const int tx = lx + kGH;
    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
#pragma unroll
        for (int r = 0; r < kGR; ++r) tile[b][ly + 4 * r + kGH][tx] = w[2][r];
        tile[b][hrt][tx] = hr;
        if (ly == 0) tile[b][(lx & 15) + kGH][hct] = hc;
        // the values of later planes, in flight while this plane is differenced
        T wn[kGR];
#pragma unroll
        for (int r = 0; r < kGR; ++r) wn[r] = ld(phi, z + 3, oc[r], ok[r] && z + 3 < nz);
        const T hrn = ld(phi, z + 1, ohr, hrv && z + 1 < z1), hcn = ld(phi, z + 1, ohc, hcv && z + 1 < z1);
        T mv[kGR][3];
        if (m) {
#pragma unroll
            for (int r = 0; r < kGR; ++r)
#pragma unroll
                for (int a = 0; a < 3; ++a) mv[r][a] = plane(m + a * N, z)[oc[r]];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kGR; ++r) {
            const int ty = ly + 4 * r + kGH, y = y0 + ly + 4 * r;
            const T c = w[2][r];
            const T hxv = minus_d5(tile[b][ty][tx - 2], tile[b][ty][tx - 1], c, tile[b][ty][tx + 1], tile[b][ty][tx + 2],
                                   x, nx, rx);
            const T hyv = minus_d5(tile[b][ty - 2][tx], tile[b][ty - 1][tx], c, tile[b][ty + 1][tx], tile[b][ty + 2][tx],
                                   y, ny, ry);
            const T hzv = minus_d5(w[0][r], w[1][r], c, w[3][r], w[4][r], z, nz, rz);
            if (ok[r]) {
                T* hz = H + (size_t)z * sxy;
                hz[oc[r]] = hxv;
                hz[N + oc[r]] = hyv;
                hz[2 * N + oc[r]] = hzv;
                if (m) acc += (double)(mv[r][0] * hxv) + (double)(mv[r][1] * hyv) + (double)(mv[r][2] * hzv);
            }
        }
#pragma unroll
        for (int r = 0; r < kGR; ++r) {
            w[0][r] = w[1][r];
            w[1][r] = w[2][r];
            w[2][r] = w[3][r];
            w[3][r] = w[4][r];
            w[4][r] = wn[r];
        }
        hr = hrn;
        hc = hcn;
    }
    if (partials) {
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lx == 0) red[ly] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

}  // namespace

hipError_t launch_sp_kernel_octant(hipStream_t st, int nx, int ny, int nz, const double dt[3], const TensorBands& tb,
                                   const double* gl_x_dev, const double* gl_w_dev, double* Soct) {
    const size_t ncell = (size_t)nx * ny * nz;
    hipError_t e = launch_pieces(ncell, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL(k_sp_pointwise, dim3(blocks), dim3(256), 0, st, base, nx, ny, nz, dt[0], dt[1], dt[2],
                           tb.far_cut, tb.fg_cut, Soct);
    });
    if (e != hipSuccess) return e;
    // (in floating point: far_cut / dt may exceed the int range)
    auto box = [&](int n, double d) { return (int)std::min<double>(n, ceil(tb.far_cut / d) + 1.0); };
    const int bx = box(nx, dt[0]), by = box(ny, dt[1]), bz = box(nz, dt[2]);
    const long nb = (long)bx * by * bz;
    if (nb > 0 && tb.far_cut > 0) {  // one 64-lane workgroup per offset of the box
        e = launch_pieces((size_t)nb * 64, 64, [&](size_t base, unsigned blocks) {
            hipLaunchKernelGGL(k_sp_mid, dim3(blocks), dim3(64), 0, st, (long)(base / 64), nx, ny, nz, bx, by, dt[0],
                               dt[1], dt[2], tb.far_cut, tb.fg_cut, tb.gl_q, tb.max_panels, gl_x_dev, gl_w_dev, Soct);
        });
    }
    return e;
}

hipError_t launch_sp_embed(hipStream_t st, int a, int nx, int ny, int nz, int Px, int Py, int Pz, const double* Soct,
                           double* A) {
    const size_t total = (size_t)Px * Py * Pz;
    return launch_pieces(total, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL(k_sp_embed, dim3(blocks), dim3(256), 0, st, base, a, nx, ny, nz, Px, Py, Pz, Soct, A);
    });
}

template <typename T>
hipError_t launch_sp_extract(hipStream_t st, int a, int Py, int Pz, int Kx, double scale, const cx<double>* B2,
                             T* shat) {
    const size_t total = (size_t)(Py / 2 + 1) * Kx * (Pz / 2 + 1);
    return launch_pieces(total, 256, [&](size_t base, unsigned blocks) {
        hipLaunchKernelGGL((k_sp_extract<T>), dim3(blocks), dim3(256), 0, st, base, a, Py, Pz, Kx, scale, B2, shat);
    });
}

long sp_gradient_tiles(int nx, int ny, int nz, int zc) {
    return (long)((nx + kGX - 1) / kGX) * ((ny + kGY - 1) / kGY) * ((nz + zc - 1) / zc);
}

// z-chunk: the longest (up to 16 planes) that still gives about 1024
// workgroups, so that the device is filled and each chunk reuses its planes
int sp_gradient_zc(int nx, int ny, int nz) {
    int zc = 16;
    while (zc > 1 && sp_gradient_tiles(nx, ny, nz, zc) < 1024) zc >>= 1;
    return std::min(zc, std::max(nz, 1));
}

template <typename T>
hipError_t launch_sp_gradient(hipStream_t st, int nx, int ny, int nz, const double d[3], const T* phi, T* H,
                              const T* m, double* partials, int* nparts) {
    const int zc = sp_gradient_zc(nx, ny, nz);
    const long tiles = sp_gradient_tiles(nx, ny, nz, zc);
    if (tiles > INT_MAX) return hipErrorInvalidValue;
    if (nparts) *nparts = (int)tiles;
    hipLaunchKernelGGL((k_sp_gradient<T>), dim3((unsigned)tiles), dim3(256), 0, st, nx, ny, nz, zc, (T)d[0], (T)d[1],
                       (T)d[2], phi, H, m, partials);
    return hipGetLastError();
}

template hipError_t launch_sp_extract<float>(hipStream_t, int, int, int, int, double, const cx<double>*, float*);
template hipError_t launch_sp_extract<double>(hipStream_t, int, int, int, int, double, const cx<double>*, double*);
template hipError_t launch_sp_gradient<float>(hipStream_t, int, int, int, const double[3], const float*, float*,
                                              const float*, double*, int*);
template hipError_t launch_sp_gradient<double>(hipStream_t, int, int, int, const double[3], const double*, double*,
                                               const double*, double*, int*);

}  // namespace demag
