// Local element kernels on a prism with vertical columns.
//
// Geometry: the bottom triangle has vertices (x_a, y_a), a = 0..2, and the
// column above vertex a rises by h_a over the layer (terrain-following
// layers are allowed; (x, y) is the same at both levels).  With reference
// coordinates (xi, eta) on the triangle, barycentrics lambda_a, and zeta in
// [0, 1] upwards, the Jacobian determinant of the P1 x P1 coordinate map is
//     det J = 2A * sum_a lambda_a h_a,
// 2A the (absolute) doubled area of the base triangle: linear in the
// horizontal variables and constant in zeta.  The integrals below are exact
// for that geometry.
//
// Reference-triangle integrals use the barycentric monomial rule
//     integral of l0^i l1^j l2^k over the reference triangle = i! j! k! / (i+j+k+2)!.
#pragma once

#include <hip/hip_runtime.h>

namespace exm {

__device__ __forceinline__ double twice_area(const double x[3], const double y[3])
{
    return fabs((x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]));
}

// P1 x P1 (and DG1 x DG1, which has the same local basis) mass action on one
// prism: y = M x with x given at the bottom (xb) and top (xt) node of every
// base vertex.  M = 2A * T(h) (x) V with
//     T_ab(h) = sum_c h_c integral lambda_a lambda_b lambda_c
//             = (2 h_a + H) / 60 on the diagonal, (h_a + h_b + H) / 120 off it
//     (H = h_0 + h_1 + h_2), and V = [[1/3, 1/6], [1/6, 1/3]] on [0, 1].
// Sum-factorised: g = V x per vertex, then
//     y_a = (2A / 120) ((2 h_a + H) g_a + (h_a + H) G + sum_b h_b g_b),  G = sum_b g_b.
__device__ __forceinline__ void p1_mass(double twoA, const double h[3], const double xb[3], const double xt[3],
                                        double yb[3], double yt[3])
{
    constexpr double sixth = 1.0 / 6.0;
    const double s = twoA * (1.0 / 120.0);
    const double H = h[0] + h[1] + h[2];
    double gb[3], gt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gb[a] = (2.0 * xb[a] + xt[a]) * sixth;
        gt[a] = (xb[a] + 2.0 * xt[a]) * sixth;
    }
    const double Gb = gb[0] + gb[1] + gb[2];
    const double Gt = gt[0] + gt[1] + gt[2];
    const double HGb = h[0] * gb[0] + h[1] * gb[1] + h[2] * gb[2];
    const double HGt = h[0] * gt[0] + h[1] * gt[1] + h[2] * gt[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double da = 2.0 * h[a] + H;
        const double oa = h[a] + H;
        yb[a] = s * (da * gb[a] + oa * Gb + HGb);
        yt[a] = s * (da * gt[a] + oa * Gt + HGt);
    }
}

// DG0 x DG0: integral of the prism = 2A * sum_c h_c / 6 (each lambda_c
// integrates to 1/6 on the reference triangle).
__device__ __forceinline__ double dg0_mass(double twoA, const double h[3], double x)
{
    return x * twoA * (h[0] + h[1] + h[2]) * (1.0 / 6.0);
}

// P2 x P2 mass action.  Horizontal nodes: vertices 0, 1, 2 (basis
// lambda_a (2 lambda_a - 1)) then edges 0, 1, 2 (edge a opposite vertex a,
// basis 4 lambda_{a+1} lambda_{a+2}).  Vertical nodes: bottom, top, middle of
// the interval.  M = 2A * T2(h) (x) V2 with
//     T2(h) = sum_c h_c K_c / 2520,   K_c[i][j] = 2520 * integral phi_i phi_j lambda_c,
//     V2 = [[4, -1, 2], [-1, 4, 2], [2, 2, 16]] / 30.
// K_c follows from the monomial rule; rows/columns in node order above.
#define EXM_P2_K_TABLE                                                                            \
    {{{30, -4, -4, -4, 12, 12}, {-4, 6, 1, -4, -12, -8}, {-4, 1, 6, -4, -8, -12},               \
      {-4, -4, -4, 32, 32, 32}, {12, -12, -8, 32, 96, 48}, {12, -8, -12, 32, 48, 96}},          \
     {{6, -4, 1, -12, -4, -8}, {-4, 30, -4, 12, -4, 12}, {1, -4, 6, -8, -4, -12},               \
      {-12, 12, -8, 96, 32, 48}, {-4, -4, -4, 32, 32, 32}, {-8, 12, -12, 48, 32, 96}},          \
     {{6, 1, -4, -12, -8, -4}, {1, 6, -4, -8, -12, -4}, {-4, -4, 30, 12, 12, -4},               \
      {-12, -8, 12, 96, 48, 32}, {-8, -12, 12, 48, 96, 32}, {-4, -4, -4, 32, 32, 32}}}

// x[e][beta], y[e][beta]: e = horizontal node 0..5, beta = bottom, top, middle.
__device__ __forceinline__ void p2_mass(double twoA, const double h[3], const double x[6][3], double y[6][3])
{
    // vertical factor, scaled by 2A / (2520 * 30)
    constexpr double K[3][6][6] = EXM_P2_K_TABLE;
    const double s = twoA * (1.0 / (2520.0 * 30.0));
    double g[6][3];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        g[e][0] = 4.0 * x[e][0] - x[e][1] + 2.0 * x[e][2];
        g[e][1] = -x[e][0] + 4.0 * x[e][1] + 2.0 * x[e][2];
        g[e][2] = 2.0 * (x[e][0] + x[e][1]) + 16.0 * x[e][2];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double t = h[0] * K[0][i][j] + h[1] * K[1][i][j] + h[2] * K[2][i][j];
            acc0 += t * g[j][0];
            acc1 += t * g[j][1];
            acc2 += t * g[j][2];
        }
        y[i][0] = s * acc0;
        y[i][1] = s * acc1;
        y[i][2] = s * acc2;
    }
}

// ---------------------------------------------------------------------------
// Quadrature for the nonlinear P1 x P1 forms.  The integrand of the cubic
// residual (u^3 - f) v det J has degree 5 horizontally and 4 vertically on
// these prisms, so the 7-point degree-5 triangle rule of Radon (centroid and
// two three-point orbits built on sqrt(15)) times 3-point Gauss-Legendre in
// zeta integrates it exactly.

struct CubicRule {
    // barycentric coordinates and weights (weights sum to 1/2, the reference area)
    double lam[7][3];
    double w[7];
    double z[3];
    double wz[3];
};

__device__ __forceinline__ void cubic_rule(CubicRule& r)
{
    const double s15 = 3.872983346207416885;   // sqrt(15)
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double w1 = (155.0 - s15) / 2400.0, w2 = (155.0 + s15) / 2400.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    const double L[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
                            {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2}};
    const double W[7] = {9.0 / 80.0, w1, w1, w1, w2, w2, w2};
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        r.w[i] = W[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) r.lam[i][a] = L[i][a];
    }
    const double g = 0.5 * 0.774596669241483377;   // sqrt(3/5) / 2
    r.z[0] = 0.5 - g;
    r.z[1] = 0.5;
    r.z[2] = 0.5 + g;
    r.wz[0] = 5.0 / 18.0;
    r.wz[1] = 8.0 / 18.0;
    r.wz[2] = 5.0 / 18.0;
}

// Values of a P1 x P1 field at the 21 points: v[i][j] (triangle point i,
// interval point j).
__device__ __forceinline__ void p1_at_points(const CubicRule& r, const double xb[3], const double xt[3],
                                             double v[7][3])
{
    double col[3][3];   // column value of vertex a at height z_j
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) col[a][j] = xb[a] + r.z[j] * (xt[a] - xb[a]);
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            v[i][j] = r.lam[i][0] * col[0][j] + r.lam[i][1] * col[1][j] + r.lam[i][2] * col[2][j];
}

// Test a point-value field s[i][j] (already multiplied by weights and det J)
// against the P1 x P1 basis: out_b[a] += sum s lambda_a (1 - z), out_t[a] += sum s lambda_a z.
__device__ __forceinline__ void p1_test(const CubicRule& r, const double s[7][3], double ob[3], double ot[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double tb = 0.0, tt = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 7; ++i) t += r.lam[i][a] * s[i][j];
            tb += (1.0 - r.z[j]) * t;
            tt += r.z[j] * t;
        }
        ob[a] = tb;
        ot[a] = tt;
    }
}

// det J times the quadrature weight at every point.
__device__ __forceinline__ void cubic_weights(const CubicRule& r, double twoA, const double h[3], double W[7][3])
{
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const double dj = twoA * (r.lam[i][0] * h[0] + r.lam[i][1] * h[1] + r.lam[i][2] * h[2]);
#pragma unroll
        for (int j = 0; j < 3; ++j) W[i][j] = r.w[i] * r.wz[j] * dj;
    }
}

}  // namespace exm
