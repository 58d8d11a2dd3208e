/*
 * Plain CPU oracle for the scalar-potential (SP) stray-field method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite and the benchmark's CPU leg do.  It
 * shares no code, header or table with the GPU path.
 *
 * What it computes (Abert et al., "Numerical Methods for the Stray-Field
 * Calculation", Sec. 3.1, eqs. (scpot), (convolution), (field)): the scalar
 * potential of a cell-wise constant magnetization is the convolution of the
 * magnetization with the vector kernel S, the field is minus its gradient,
 * taken by finite differences.  On a regular grid of cuboid cells, with the
 * potential sampled at cell centres,
 *
 *      phi_i = Ms * sum_j sum_a S_a(r_i - r_j) m_{a,j}      (every cell j)
 *
 * where S_a(R) is the potential at R of the cell centred at the origin with
 * unit magnetization along axis a.  Integrating the kernel of eq. (scpot)
 * along a turns that cell into two charged faces:
 *
 *      S_a(R) = (1/(4 pi)) [ G_a(R - (d_a/2) e_a) - G_a(R + (d_a/2) e_a) ]
 *
 * with G_a(R') the Newton potential at relative position R' of the unit-
 * density rectangle d_b x d_c (the face perpendicular to a) centred in its
 * plane.  Its closed form is the corner sum of
 *
 *      F(u, v, w) = u asinh(v / sqrt(u^2 + w^2)) + v asinh(u / sqrt(v^2 + w^2))
 *                   - w atan(u v / (w sqrt(u^2 + v^2 + w^2))),
 *
 * d^2 F / du dv = 1 / sqrt(u^2 + v^2 + w^2) (w the distance to the plane), a
 * term with a zero prefactor counting as zero.  F is evaluated in binary128,
 * so that the cancellation between the two faces at large offsets is
 * invisible in the rounded FP64 kernel.
 *
 * The field (eq. (field)): H = -grad phi by central differences inside the
 * grid and second-order one-sided differences on its faces (first order for
 * two cells along an axis, zero for one cell), since the paper leaves the
 * stencil open and the potential is only sampled inside the body.
 *
 * Layouts: a vector field is SoA [3][nz][ny][nx] (x fastest); the potential
 * [nz][ny][nx]; the kernel "octant" [3][nz][ny][nx] holds S_a(o) for offsets
 * o in [0, n) per axis (S_a is odd in axis a and even in the other two).
 */
#include <math.h>
#include <omp.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>

typedef __float128 quad;

static quad sq_asinh(quad pre, quad num, quad den2)
{
    if (pre == 0) return 0;
    return pre * asinhq(num / sqrtq(den2));
}

/* F(u, v, w) above */
static quad face_F(quad u, quad v, quad w)
{
    quad r = sqrtq(u * u + v * v + w * w);
    quad t = sq_asinh(u, v, u * u + w * w) + sq_asinh(v, u, v * v + w * w);
    if (w != 0 && u != 0 && v != 0) t -= w * atanq(u * v / (w * r));
    return t;
}

/* G: potential at (X, Y, W) of the unit-density rectangle [-A/2, A/2] x
 * [-B/2, B/2] in the plane w = 0 (all lengths in one unit) */
static quad face_G(quad X, quad Y, quad W, quad A, quad B)
{
    quad u1 = -A / 2 - X, u2 = A / 2 - X, v1 = -B / 2 - Y, v2 = B / 2 - Y;
    return face_F(u2, v2, W) - face_F(u1, v2, W) - face_F(u2, v1, W) + face_F(u1, v1, W);
}

double sp_face_potential(double X, double Y, double W, double A, double B)
{
    return (double)face_G(X, Y, W, A, B);
}

/* S_a at offset R (physical units), straight from the two faces */
static quad sp_S(int a, quad Rx, quad Ry, quad Rz, const quad d[3])
{
    const quad R[3] = {Rx, Ry, Rz};
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    quad top = face_G(R[b], R[c], R[a] - d[a] / 2, d[b], d[c]);
    quad bot = face_G(R[b], R[c], R[a] + d[a] / 2, d[b], d[c]);
    return (top - bot) / (4 * M_PIq);
}

/* S_a at a signed integer cell offset, physical units (potential per unit
 * magnetization: metres) */
double oracle_sp_kernel_at(int a, long ox, long oy, long oz, double dx, double dy, double dz)
{
    const quad d[3] = {dx, dy, dz};
    return (double)sp_S(a, ox * d[0], oy * d[1], oz * d[2], d);
}

/* The kernel octant: S_a(o) for o in [0, n) per axis, each value straight
 * from its two faces.  Lengths are scaled by h = max(d) (S is homogeneous of
 * degree one in length) to keep the binary128 arguments near one. */
int oracle_sp_kernel(int nx, int ny, int nz, double dx, double dy, double dz, double *Soct)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const double h = fmax(dx, fmax(dy, dz));
    const quad d[3] = {dx / h, dy / h, dz / h};
    const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x)
                for (int a = 0; a < 3; ++a)
                    Soct[(size_t)a * N + ((size_t)z * ny + y) * nx + x] =
                        (double)(sp_S(a, x * d[0], y * d[1], z * d[2], d) * h);
    return 0;
}

/* S_a at a signed offset from the octant: odd in axis a, even in the others */
static double s_signed(const double *Soct, int nx, int ny, int nz, int a, long ox, long oy, long oz)
{
    const long o[3] = {ox, oy, oz};
    double sign = o[a] < 0 ? -1.0 : 1.0;
    const size_t N = (size_t)nx * ny * nz;
    return sign * Soct[(size_t)a * N + ((size_t)labs(oz) * ny + labs(oy)) * nx + labs(ox)];
}

static double potential_at(int nx, int ny, int nz, const double *Soct, const double *m, double Ms,
                           long tx, long ty, long tz)
{
    const size_t N = (size_t)nx * ny * nz;
    double acc = 0.0;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                const size_t j = ((size_t)z * ny + y) * nx + x;
                for (int a = 0; a < 3; ++a)
                    acc += s_signed(Soct, nx, ny, nz, a, tx - x, ty - y, tz - z) * m[(size_t)a * N + j];
            }
    return Ms * acc;
}

/* phi at every cell, Sec. 3.1 eq. (scpot) as a plain sum */
int oracle_sp_potential(int nx, int ny, int nz, const double *Soct, const double *m, double Ms, double *phi)
{
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x)
                phi[((size_t)z * ny + y) * nx + x] = potential_at(nx, ny, nz, Soct, m, Ms, x, y, z);
    return 0;
}

/* -d phi / d axis at cell index i along an axis of n cells, spacing h, from
 * the potential along that line (stride s from the cell's own value p) */
static double minus_derivative(const double *p, long i, long n, long s, double h)
{
    if (n == 1) return 0.0;
    if (n == 2) return i == 0 ? -(p[s] - p[0]) / h : -(p[0] - p[-s]) / h;
    if (i == 0) return -(-3.0 * p[0] + 4.0 * p[s] - p[2 * s]) / (2.0 * h);
    if (i == n - 1) return -(3.0 * p[0] - 4.0 * p[-s] + p[-2 * s]) / (2.0 * h);
    return -(p[s] - p[-s]) / (2.0 * h);
}

/* H = -grad phi (eq. (field)) at every cell from a potential on the grid */
int oracle_sp_gradient(int nx, int ny, int nz, double dx, double dy, double dz, const double *phi, double *H)
{
    const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                const size_t i = ((size_t)z * ny + y) * nx + x;
                H[i] = minus_derivative(phi + i, x, nx, 1, dx);
                H[N + i] = minus_derivative(phi + i, y, ny, nx, dy);
                H[2 * N + i] = minus_derivative(phi + i, z, nz, (long)nx * ny, dz);
            }
    return 0;
}

/* the SP field at every cell: potential, then its gradient */
int oracle_sp_field(int nx, int ny, int nz, double dx, double dy, double dz, const double *Soct,
                    const double *m, double Ms, double *H)
{
    double *phi = malloc(sizeof(double) * (size_t)nx * ny * nz);
    if (!phi) return -2;
    oracle_sp_potential(nx, ny, nz, Soct, m, Ms, phi);
    oracle_sp_gradient(nx, ny, nz, dx, dy, dz, phi, H);
    free(phi);
    return 0;
}

/* The SP field at selected cells only: the potential is summed at each target
 * and at the cells its difference stencils read, then differenced as in
 * oracle_sp_gradient.  out[3][count]. */
int oracle_sp_field_targets(int nx, int ny, int nz, double dx, double dy, double dz, const double *Soct,
                            const double *m, double Ms, const int64_t *targets, long count, double *out)
{
    const size_t N = (size_t)nx * ny * nz;
    for (long t = 0; t < count; ++t)
        if (targets[t] < 0 || (size_t)targets[t] >= N) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < count; ++t) {
        const long i = (long)targets[t];
        const long x = i % nx, y = (i / nx) % ny, z = i / ((long)nx * ny);
        const long c[3] = {x, y, z}, n[3] = {nx, ny, nz};
        const double h[3] = {dx, dy, dz};
        for (int a = 0; a < 3; ++a) {
            /* the potential on the line through the target along a, at the
             * offsets its stencil reads (-2..2), stored around index 2 */
            double line[5] = {0, 0, 0, 0, 0};
            for (long e = -2; e <= 2; ++e) {
                const long q = c[a] + e;
                if (q < 0 || q >= n[a]) continue;
                long p[3] = {x, y, z};
                p[a] = q;
                line[e + 2] = potential_at(nx, ny, nz, Soct, m, Ms, p[0], p[1], p[2]);
            }
            out[(size_t)a * count + t] = minus_derivative(line + 2, c[a], n[a], 1, h[a]);
        }
    }
    return 0;
}
