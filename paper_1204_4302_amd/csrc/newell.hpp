// Cell-averaged demagnetization tensor of homogeneously magnetized cuboid
// cells, in FP64, for one integer cell offset o (device math for the setup).
//
// The paper uses the tensor of homogeneously magnetized cells whose field is
// averaged over each cell (Sec. 5.1) without printing it.  Three routes to the
// same quantity, chosen per offset by distance:
//
//  near  (Chebyshev distance <= fg_cut): the closed form of Newell, Williams
//        and Dunlop (1993), (1/(4 pi V)) x 27-point second difference of the
//        auxiliary functions f (diagonal) and g (off-diagonal).  Exact, but the
//        second difference cancels catastrophically as the offset grows.
//  mid   : the defining integral N(R) = V * int D(R+u) prod_k W_k(u_k) du over
//        u in [-d,d]^3, D_ab = (delta_ab r^2 - 3 r_a r_b)/(4 pi r^5) the point
//        dipole kernel and W_k(s) = (d_k - |s|)/d_k^2 the autocorrelation of two
//        cells.  Product Gauss-Legendre on panels no longer than the gap
//        between the two cells, so the integrand is smooth on each panel.
//  far   (rho = |o (.) d| / max d >= far_cut): the same integral expanded in
//        the even moments of W: N ~ V sum_beta c_beta d^beta D(R) over even
//        multi-indices |beta| <= 6, c_beta = prod_k M_{beta_k}/beta_k!,
//        M_2 = d^2/6, M_4 = d^4/15, M_6 = d^6/28.  Derivatives of 1/r come from
//        the Cartesian Taylor-coefficient recurrence
//        n r^2 a_alpha = -(2n-1) sum_i x_i a_{alpha-e_i} - (n-1) sum_i a_{alpha-2e_i},
//        a_alpha = d^alpha(1/r)/alpha!,  n = |alpha|.
//
// All lengths are in reduced units (cell edges divided by the largest edge):
// N is invariant under a common scaling.  Components: xx, yy, zz, xy, xz, yz.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define DEMAG_HD __host__ __device__ inline

namespace demag {
namespace newell {

constexpr double kPi = 3.14159265358979323846264338327950288;

// ---- near band: Newell f / g ------------------------------------------------
// A term whose polynomial prefactor is zero is zero (its limit); this also
// removes the 0/0 and asinh(inf) forms on the lattice axes.
DEMAG_HD double asinh_term(double pre, double num, double den2) {
    return pre == 0.0 ? 0.0 : pre * asinh(num / sqrt(den2));
}
DEMAG_HD double atan_term(double pre, double num, double den) {
    return pre == 0.0 ? 0.0 : pre * atan(num / den);
}

DEMAG_HD double f_aux(double x, double y, double z) {
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    double s = asinh_term(0.5 * y * (z2 - x2), y, x2 + z2);
    s += asinh_term(0.5 * z * (y2 - x2), z, x2 + y2);
    s -= atan_term(x * y * z, y * z, x * R);
    s += (2.0 * x2 - y2 - z2) * R / 6.0;
    return s;
}

DEMAG_HD double g_aux(double x, double y, double z) {
    double x2 = x * x, y2 = y * y, z2 = z * z;
    double R = sqrt(x2 + y2 + z2);
    double s = asinh_term(x * y * z, z, x2 + y2);
    s += asinh_term(y * (3.0 * z2 - y2) / 6.0, x, y2 + z2);
    s += asinh_term(x * (3.0 * z2 - x2) / 6.0, y, x2 + z2);
    s -= atan_term(z * z2 / 6.0, x * y, z * R);
    s -= atan_term(0.5 * z * y2, x * z, y * R);
    s -= atan_term(0.5 * z * x2, y * z, x * R);
    s -= x * y * R / 3.0;
    return s;
}

// Auxiliary function of component c at lattice point (a,b,cc) (cell units).
DEMAG_HD double aux(int comp, double X, double Y, double Z) {
    switch (comp) {
    case 0: return f_aux(X, Y, Z);
    case 1: return f_aux(Y, X, Z);
    case 2: return f_aux(Z, Y, X);
    case 3: return g_aux(X, Y, Z);
    case 4: return g_aux(X, Z, Y);
    default: return g_aux(Y, Z, X);
    }
}

DEMAG_HD void near_fg(int ox, int oy, int oz, const double dt[3], double out[6]) {
    const double norm = 1.0 / (4.0 * kPi * dt[0] * dt[1] * dt[2]);
    for (int comp = 0; comp < 6; ++comp) {
        double acc = 0.0;
        for (int ez = -1; ez <= 1; ++ez)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    double w = (ex == 0 ? 2.0 : -1.0) * (ey == 0 ? 2.0 : -1.0) * (ez == 0 ? 2.0 : -1.0);
                    acc += w * aux(comp, (ox + ex) * dt[0], (oy + ey) * dt[1], (oz + ez) * dt[2]);
                }
        out[comp] = acc * norm;
    }
}

// ---- far band: moment series of the point-dipole kernel ---------------------
constexpr int kFarMaxDeriv = 8;  // |gamma| = |beta| + 2 with |beta| <= 6

// Flat (tetrahedral) index of multi-index (i,j,k), i + j + k <= kFarMaxDeriv.
constexpr int kTaylorLen = (kFarMaxDeriv + 1) * (kFarMaxDeriv + 2) * (kFarMaxDeriv + 3) / 6;
DEMAG_HD int tidx(int i, int j, int k) {
    int n = i + j + k, jk = j + k;
    return n * (n + 1) * (n + 2) / 6 + jk * (jk + 1) / 2 + k;
}

DEMAG_HD double fact(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// Taylor coefficients a[i][j][k] = d^(i,j,k)(1/r)/(i! j! k!) for i+j+k <= 8.
DEMAG_HD void inv_r_taylor(double x, double y, double z, double a[kTaylorLen]) {
    const double r2 = x * x + y * y + z * z;
    a[tidx(0, 0, 0)] = 1.0 / sqrt(r2);
    for (int n = 1; n <= kFarMaxDeriv; ++n)
        for (int i = n; i >= 0; --i)
            for (int j = n - i; j >= 0; --j) {
                int k = n - i - j;
                double s1 = 0.0, s2 = 0.0;
                if (i >= 1) s1 += x * a[tidx(i - 1, j, k)];
                if (j >= 1) s1 += y * a[tidx(i, j - 1, k)];
                if (k >= 1) s1 += z * a[tidx(i, j, k - 1)];
                if (i >= 2) s2 += a[tidx(i - 2, j, k)];
                if (j >= 2) s2 += a[tidx(i, j - 2, k)];
                if (k >= 2) s2 += a[tidx(i, j, k - 2)];
                a[tidx(i, j, k)] = (-(2.0 * n - 1.0) * s1 - (n - 1.0) * s2) / (n * r2);
            }
}

DEMAG_HD double even_moment(int p, double d) {
    // int s^p W(s) ds, W(s) = (d - |s|)/d^2 on [-d, d], p even
    return p == 0 ? 1.0 : 2.0 * pow(d, (double)p) / ((p + 1.0) * (p + 2.0));
}

DEMAG_HD void far_series(int ox, int oy, int oz, const double dt[3], double out[6]) {
    double a[kTaylorLen];
    inv_r_taylor(ox * dt[0], oy * dt[1], oz * dt[2], a);
    const int ca[6] = {0, 1, 2, 0, 0, 1}, cb[6] = {0, 1, 2, 1, 2, 2};
    const double V = dt[0] * dt[1] * dt[2];
    for (int comp = 0; comp < 6; ++comp) out[comp] = 0.0;
    for (int bx = 0; bx <= 6; bx += 2)
        for (int by = 0; by <= 6 - bx; by += 2)
            for (int bz = 0; bz <= 6 - bx - by; bz += 2) {
                double cbeta = even_moment(bx, dt[0]) / fact(bx) * even_moment(by, dt[1]) / fact(by) *
                               even_moment(bz, dt[2]) / fact(bz);
                for (int comp = 0; comp < 6; ++comp) {
                    int g[3] = {bx, by, bz};
                    g[ca[comp]] += 1;
                    g[cb[comp]] += 1;
                    double gfac = fact(g[0]) * fact(g[1]) * fact(g[2]);
                    out[comp] += cbeta * gfac * a[tidx(g[0], g[1], g[2])];
                }
            }
    for (int comp = 0; comp < 6; ++comp) out[comp] *= -V / (4.0 * kPi);
}

// ---- mid band: Gauss-Legendre of the cell-average integral -------------------
// Panel count per half-axis so that each panel is no longer than the gap
// between the two cells (the distance from the integration box to the pole).
DEMAG_HD double cell_gap(int ox, int oy, int oz, const double dt[3]) {
    double s = 0.0;
    const int o[3] = {ox, oy, oz};
    for (int k = 0; k < 3; ++k) {
        double g = fabs((double)o[k]) * dt[k] - dt[k];
        if (g > 0) s += g * g;
    }
    return sqrt(s);
}

DEMAG_HD int mid_panels(double d, double gap, int max_panels) {
    int m = (int)ceil(d / gap - 1e-12);
    if (m < 1) m = 1;
    if (m > max_panels) m = max_panels;
    return m;
}

// Node k of axis with cell edge d, m panels per half, q GL nodes per panel
// (xg, wg on [-1,1]); returns position s and weight w (incl. W(s)).
DEMAG_HD void mid_node(int k, double d, int m, int q, const double* xg, const double* wg,
                       double* s, double* w) {
    int half = k / (m * q);  // 0: [-d,0], 1: [0,d]
    int rem = k - half * m * q;
    int panel = rem / q, node = rem - panel * q;
    double h = d / m;
    double lo = (half == 0 ? -d : 0.0) + panel * h;
    double pos = lo + 0.5 * h * (xg[node] + 1.0);
    *s = pos;
    *w = 0.5 * h * wg[node] * (d - fabs(pos)) / (d * d);
}

DEMAG_HD void dipole_add(double X, double Y, double Z, double w, double acc[6]) {
    double r2 = X * X + Y * Y + Z * Z;
    double ir = 1.0 / sqrt(r2);
    double ir5 = ir * ir * ir * ir * ir * w / (4.0 * kPi);
    acc[0] += (r2 - 3.0 * X * X) * ir5;
    acc[1] += (r2 - 3.0 * Y * Y) * ir5;
    acc[2] += (r2 - 3.0 * Z * Z) * ir5;
    acc[3] += -3.0 * X * Y * ir5;
    acc[4] += -3.0 * X * Z * ir5;
    acc[5] += -3.0 * Y * Z * ir5;
}

}  // namespace newell
}  // namespace demag
