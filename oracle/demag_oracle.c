/*
 * Plain CPU oracle for the demagnetization-tensor (DM) stray-field method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.
 *
 * What it computes (Abert et al., "Numerical Methods for the Stray-Field
 * Calculation", Sec. 3.1, eq. (demag)): the field of a cell-wise constant
 * magnetization on a regular cuboid grid is the discrete matrix-vector
 * convolution
 *
 *      H_i = -Ms * sum_j N(r_i - r_j) m_j          (every cell j, j = i included)
 *
 * with N the cell-averaged demagnetization tensor of homogeneously magnetized
 * cuboid cells (Sec. 5.1: the tensor assumes homogeneously magnetized cells and
 * the field is averaged over each cell).  The paper names this tensor but does
 * not print it; the closed forms used here are those of Newell, Williams and
 * Dunlop (J. Geophys. Res. 98, 1993): N is (1/(4 pi V)) times the 27-point
 * second difference of the auxiliary functions f (diagonal) and g
 * (off-diagonal) over the cell lattice.  Those functions are evaluated in
 * binary128 (__float128) so that the cancellation of the second difference at
 * large offsets costs nothing visible in the rounded FP64 result.
 *
 * The energy is the stray-field energy of Sec. 2, in SI units:
 *      E = -(mu0/2) * Ms * V * sum_i m_i . H_i,   mu0 = 4 pi 1e-7 H/m.
 *
 * Everything here is the plain definition: no FFT, no blocking, no fusion.
 * Loops over cells are parallelised with OpenMP; each target's sum is a plain
 * FP64 accumulation in source order.
 *
 * Layouts: a vector field is SoA [3][nz][ny][nx] (x fastest).  A tensor
 * "octant" is [6][nz][ny][nx] holding N(o) for offsets o in [0,n) per axis,
 * components in the order xx, yy, zz, xy, xz, yz.
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

#define ORACLE_MU0 (4.0e-7 * 3.14159265358979323846264338327950288)

/* ---- Newell auxiliary functions (binary128) ------------------------------
 * A term whose polynomial prefactor is exactly zero contributes zero; this
 * is the limit of every such term (x*asinh(c/x) -> 0 and so on) and also
 * removes the 0/0 and asinh(inf) forms at lattice points on the axes.      */

static quad q_asinh_term(quad pre, quad num, quad den2)
{
    if (pre == 0) return 0;
    return pre * asinhq(num / sqrtq(den2));
}

static quad q_atan_term(quad pre, quad num, quad den)
{
    if (pre == 0) return 0;
    return pre * atanq(num / den);
}

/* f(x,y,z): diagonal auxiliary function (even in x, y and z). */
static quad newell_f(quad x, quad y, quad z)
{
    quad x2 = x * x, y2 = y * y, z2 = z * z;
    quad R = sqrtq(x2 + y2 + z2);
    quad s = 0;
    s += q_asinh_term(y / 2 * (z2 - x2), y, x2 + z2);
    s += q_asinh_term(z / 2 * (y2 - x2), z, x2 + y2);
    s -= q_atan_term(x * y * z, y * z, x * R);
    s += (2 * x2 - y2 - z2) * R / 6;
    return s;
}

/* g(x,y,z): off-diagonal auxiliary function (odd in x, odd in y, even in z). */
static quad newell_g(quad x, quad y, quad z)
{
    quad x2 = x * x, y2 = y * y, z2 = z * z;
    quad R = sqrtq(x2 + y2 + z2);
    quad s = 0;
    s += q_asinh_term(x * y * z, z, x2 + y2);
    s += q_asinh_term(y / 6 * (3 * z2 - y2), x, y2 + z2);
    s += q_asinh_term(x / 6 * (3 * z2 - x2), y, x2 + z2);
    s -= q_atan_term(z * z2 / 6, x * y, z * R);
    s -= q_atan_term(z * y2 / 2, x * z, y * R);
    s -= q_atan_term(z * x2 / 2, y * z, x * R);
    s -= x * y * R / 3;
    return s;
}

/* Lattice value of component c at integer lattice point (a,b,c3), with the
 * cell edges already in reduced units (dt = d / max(d)).                    */
static quad lattice_value(int comp, long a, long b, long c3, const quad dt[3])
{
    quad X = (quad)a * dt[0], Y = (quad)b * dt[1], Z = (quad)c3 * dt[2];
    switch (comp) {
    case 0: return newell_f(X, Y, Z);     /* xx */
    case 1: return newell_f(Y, X, Z);     /* yy */
    case 2: return newell_f(Z, Y, X);     /* zz */
    case 3: return newell_g(X, Y, Z);     /* xy */
    case 4: return newell_g(X, Z, Y);     /* xz */
    default: return newell_g(Y, Z, X);    /* yz */
    }
}

static void reduced_cell(double dx, double dy, double dz, quad dt[3])
{
    double h = dx;
    if (dy > h) h = dy;
    if (dz > h) h = dz;
    dt[0] = (quad)dx / (quad)h;
    dt[1] = (quad)dy / (quad)h;
    dt[2] = (quad)dz / (quad)h;
}

/* Weight of the 27-point second difference: product over axes of
 * 2 (eps = 0) or -1 (eps = +-1), i.e. 8, -4, 2, -1.                         */
static int stencil_weight(int ex, int ey, int ez)
{
    int w = 1;
    w *= (ex == 0) ? 2 : -1;
    w *= (ey == 0) ? 2 : -1;
    w *= (ez == 0) ? 2 : -1;
    return w;
}

/* Tensor component at one integer cell offset (any sign), straight from the
 * definition.  Used by the pins for offsets the octant does not cover.      */
double oracle_tensor_at(int comp, long ox, long oy, long oz,
                        double dx, double dy, double dz)
{
    quad dt[3];
    reduced_cell(dx, dy, dz, dt);
    quad acc = 0;
    for (int ez = -1; ez <= 1; ++ez)
        for (int ey = -1; ey <= 1; ++ey)
            for (int ex = -1; ex <= 1; ++ex)
                acc += stencil_weight(ex, ey, ez) *
                       lattice_value(comp, ox + ex, oy + ey, oz + ez, dt);
    quad V = dt[0] * dt[1] * dt[2];
    return (double)(acc / (4 * M_PIq * V));
}

double oracle_f(double x, double y, double z) { return (double)newell_f(x, y, z); }
double oracle_g(double x, double y, double z) { return (double)newell_g(x, y, z); }

/* Octant of the tensor, N_comp(o) for o in [0,nx) x [0,ny) x [0,nz).  The
 * lattice is tabulated once per component on [-1,nx] x [-1,ny] x [-1,nz]
 * (every point the stencils of the octant touch) and then differenced.     */
int oracle_tensor(int nx, int ny, int nz, double dx, double dy, double dz,
                  double *Noct)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(dy > 0) || !(dz > 0))
        return -1;
    quad dt[3];
    reduced_cell(dx, dy, dz, dt);
    const long lx = nx + 2, ly = ny + 2, lz = nz + 2;
    const long nlat = lx * ly * lz;
    const long ncell = (long)nx * ny * nz;
    quad *lat = (quad *)malloc(sizeof(quad) * nlat);
    if (!lat) return -2;
    const quad norm = 1 / (4 * M_PIq * dt[0] * dt[1] * dt[2]);
    for (int comp = 0; comp < 6; ++comp) {
#pragma omp parallel for schedule(dynamic, 64)
        for (long t = 0; t < nlat; ++t) {
            long a = t % lx - 1, b = (t / lx) % ly - 1, c = t / (lx * ly) - 1;
            lat[t] = lattice_value(comp, a, b, c, dt);
        }
#pragma omp parallel for schedule(static)
        for (long t = 0; t < ncell; ++t) {
            long ox = t % nx, oy = (t / nx) % ny, oz = t / ((long)nx * ny);
            quad acc = 0;
            for (int ez = -1; ez <= 1; ++ez)
                for (int ey = -1; ey <= 1; ++ey)
                    for (int ex = -1; ex <= 1; ++ex) {
                        long a = ox + ex + 1, b = oy + ey + 1, c = oz + ez + 1;
                        acc += stencil_weight(ex, ey, ez) * lat[(c * ly + b) * lx + a];
                    }
            Noct[comp * ncell + t] = (double)(acc * norm);
        }
    }
    free(lat);
    return 0;
}

/* ---- the discrete convolution -------------------------------------------
 * N at a signed offset from the octant.  f is even in every argument, so the
 * diagonal components are even in every offset; g is odd in its first two
 * arguments and even in the third, so N_xy is odd in ox and oy, N_xz odd in
 * ox and oz, N_yz odd in oy and oz.  (The pins check these parities against
 * oracle_tensor_at at negative offsets.)                                    */
typedef struct {
    const double *Noct;
    long nx, ny, nz, ncell;
} tensor_view;

static void tensor_signed(const tensor_view *tv, long ox, long oy, long oz, double Nv[6])
{
    double sx = ox < 0 ? -1.0 : 1.0, sy = oy < 0 ? -1.0 : 1.0, sz = oz < 0 ? -1.0 : 1.0;
    long ax = labs(ox), ay = labs(oy), az = labs(oz);
    long t = (az * tv->ny + ay) * tv->nx + ax;
    Nv[0] = tv->Noct[0 * tv->ncell + t];
    Nv[1] = tv->Noct[1 * tv->ncell + t];
    Nv[2] = tv->Noct[2 * tv->ncell + t];
    Nv[3] = sx * sy * tv->Noct[3 * tv->ncell + t];
    Nv[4] = sx * sz * tv->Noct[4 * tv->ncell + t];
    Nv[5] = sy * sz * tv->Noct[5 * tv->ncell + t];
}

/* H at one target cell i: -Ms * sum_j N(r_i - r_j) m_j. */
static void field_at(const tensor_view *tv, const double *m, double Ms,
                     long ix, long iy, long iz, double out[3])
{
    const long N = tv->ncell;
    double hx = 0, hy = 0, hz = 0, Nv[6];
    for (long jz = 0; jz < tv->nz; ++jz)
        for (long jy = 0; jy < tv->ny; ++jy)
            for (long jx = 0; jx < tv->nx; ++jx) {
                long j = (jz * tv->ny + jy) * tv->nx + jx;
                tensor_signed(tv, ix - jx, iy - jy, iz - jz, Nv);
                double mx = m[j], my = m[N + j], mz = m[2 * N + j];
                hx += Nv[0] * mx + Nv[3] * my + Nv[4] * mz;
                hy += Nv[3] * mx + Nv[1] * my + Nv[5] * mz;
                hz += Nv[4] * mx + Nv[5] * my + Nv[2] * mz;
            }
    out[0] = -Ms * hx;
    out[1] = -Ms * hy;
    out[2] = -Ms * hz;
}

int oracle_field(int nx, int ny, int nz, const double *Noct, const double *m,
                 double Ms, double *H)
{
    tensor_view tv = {Noct, nx, ny, nz, (long)nx * ny * nz};
    const long N = tv.ncell;
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < N; ++i) {
        double h[3];
        field_at(&tv, m, Ms, i % nx, (i / nx) % ny, i / ((long)nx * ny), h);
        H[i] = h[0];
        H[N + i] = h[1];
        H[2 * N + i] = h[2];
    }
    return 0;
}

/* Field at a list of flat target indices only; H_t is [3][ntarget]. */
int oracle_field_targets(int nx, int ny, int nz, const double *Noct,
                         const double *m, double Ms, const int64_t *targets,
                         long ntarget, double *H_t)
{
    tensor_view tv = {Noct, nx, ny, nz, (long)nx * ny * nz};
    const long N = tv.ncell;
    for (long k = 0; k < ntarget; ++k)
        if (targets[k] < 0 || targets[k] >= N) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < ntarget; ++k) {
        long i = targets[k];
        double h[3];
        field_at(&tv, m, Ms, i % nx, (i / nx) % ny, i / ((long)nx * ny), h);
        H_t[k] = h[0];
        H_t[ntarget + k] = h[1];
        H_t[2 * ntarget + k] = h[2];
    }
    return 0;
}

/* Transposed operator, written as its own loop: for each source cell j,
 * (A^T g)_j = -Ms * sum_i N(r_i - r_j)^T g_i.  The transpose is taken
 * explicitly (row and column of the 3x3 block swapped), so that the symmetry
 * of the operator is something the tests check rather than assume.         */
int oracle_field_T(int nx, int ny, int nz, const double *Noct, const double *g,
                   double Ms, double *out)
{
    tensor_view tv = {Noct, nx, ny, nz, (long)nx * ny * nz};
    const long N = tv.ncell;
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < N; ++j) {
        long jx = j % nx, jy = (j / nx) % ny, jz = j / ((long)nx * ny);
        double ax = 0, ay = 0, az = 0, Nv[6];
        for (long iz = 0; iz < nz; ++iz)
            for (long iy = 0; iy < ny; ++iy)
                for (long ix = 0; ix < nx; ++ix) {
                    long i = (iz * ny + iy) * nx + ix;
                    tensor_signed(&tv, ix - jx, iy - jy, iz - jz, Nv);
                    /* block B = N(r_i - r_j); rows a, columns b:
                     * B = [[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]] as stored;
                     * (B^T g)_a = sum_b B[b][a] g_b.                        */
                    double B[3][3] = {{Nv[0], Nv[3], Nv[4]},
                                      {Nv[3], Nv[1], Nv[5]},
                                      {Nv[4], Nv[5], Nv[2]}};
                    double gx = g[i], gy = g[N + i], gz = g[2 * N + i];
                    ax += B[0][0] * gx + B[1][0] * gy + B[2][0] * gz;
                    ay += B[0][1] * gx + B[1][1] * gy + B[2][1] * gz;
                    az += B[0][2] * gx + B[1][2] * gy + B[2][2] * gz;
                }
        out[j] = -Ms * ax;
        out[N + j] = -Ms * ay;
        out[2 * N + j] = -Ms * az;
    }
    return 0;
}

/* The transposed operator at a list of flat source indices only; out_t is
 * [3][ntarget].  Same loop as oracle_field_T for each listed j.            */
int oracle_field_T_targets(int nx, int ny, int nz, const double *Noct, const double *g,
                           double Ms, const int64_t *targets, long ntarget, double *out_t)
{
    tensor_view tv = {Noct, nx, ny, nz, (long)nx * ny * nz};
    const long N = tv.ncell;
    for (long k = 0; k < ntarget; ++k)
        if (targets[k] < 0 || targets[k] >= N) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long k = 0; k < ntarget; ++k) {
        long j = targets[k];
        long jx = j % nx, jy = (j / nx) % ny, jz = j / ((long)nx * ny);
        double ax = 0, ay = 0, az = 0, Nv[6];
        for (long iz = 0; iz < nz; ++iz)
            for (long iy = 0; iy < ny; ++iy)
                for (long ix = 0; ix < nx; ++ix) {
                    long i = (iz * ny + iy) * nx + ix;
                    tensor_signed(&tv, ix - jx, iy - jy, iz - jz, Nv);
                    double B[3][3] = {{Nv[0], Nv[3], Nv[4]},
                                      {Nv[3], Nv[1], Nv[5]},
                                      {Nv[4], Nv[5], Nv[2]}};
                    double gx = g[i], gy = g[N + i], gz = g[2 * N + i];
                    ax += B[0][0] * gx + B[1][0] * gy + B[2][0] * gz;
                    ay += B[0][1] * gx + B[1][1] * gy + B[2][1] * gz;
                    az += B[0][2] * gx + B[1][2] * gy + B[2][2] * gz;
                }
        out_t[k] = -Ms * ax;
        out_t[ntarget + k] = -Ms * ay;
        out_t[2 * ntarget + k] = -Ms * az;
    }
    return 0;
}

/* E = -(mu0/2) Ms V sum_i m_i . H_i  (Sec. 2, SI units). */
double oracle_energy(int nx, int ny, int nz, double dx, double dy, double dz,
                     const double *m, const double *H, double Ms)
{
    const long N = (long)nx * ny * nz;
    double s = 0;
    for (long t = 0; t < 3 * N; ++t) s += m[t] * H[t];
    return -0.5 * ORACLE_MU0 * Ms * (dx * dy * dz) * s;
}

/* Explicit operator matrix A (3N x 3N, row-major), H = A m:
 * A[a*N + i][b*N + j] = -Ms N_ab(r_i - r_j).  Only for small grids.        */
int oracle_matrix(int nx, int ny, int nz, const double *Noct, double Ms, double *A)
{
    tensor_view tv = {Noct, nx, ny, nz, (long)nx * ny * nz};
    const long N = tv.ncell;
    if (N > 4096) return -1;
    const int ia[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    for (long i = 0; i < N; ++i) {
        long ix = i % nx, iy = (i / nx) % ny, iz = i / ((long)nx * ny);
        for (long j = 0; j < N; ++j) {
            long jx = j % nx, jy = (j / nx) % ny, jz = j / ((long)nx * ny);
            double Nv[6];
            tensor_signed(&tv, ix - jx, iy - jy, iz - jz, Nv);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    A[(a * N + i) * (3 * N) + (b * N + j)] = -Ms * Nv[ia[a][b]];
        }
    }
    return 0;
}

double oracle_mu0(void) { return ORACLE_MU0; }

/* Threads an OpenMP loop of this library runs on (reporting only). */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
