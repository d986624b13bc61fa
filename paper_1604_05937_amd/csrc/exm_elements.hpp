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

// Row of node v (index 0) of the P1 x P1 mass action on one prism (the
// sum-factorised form of p1_mass restricted to one vertex):
//   y_v = (2A / 120) ((2 h_v + H) g_v + (h_v + H) G + sum_a h_a g_a),
// g = V x per vertex at the bottom and at the top.
__device__ __forceinline__ void p1_row(double s, const double h[3], const double xb[3], const double xt[3],
                                       double& yb, double& yt)
{
    constexpr double sixth = 1.0 / 6.0;
    const double H = h[0] + h[1] + h[2];
    double gb[3], gt[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gb[a] = (2.0 * xb[a] + xt[a]) * sixth;
        gt[a] = (xb[a] + 2.0 * xt[a]) * sixth;
    }
    const double Gb = gb[0] + gb[1] + gb[2], Gt = gt[0] + gt[1] + gt[2];
    const double HGb = h[0] * gb[0] + h[1] * gb[1] + h[2] * gb[2];
    const double HGt = h[0] * gt[0] + h[1] * gt[1] + h[2] * gt[2];
    const double d = 2.0 * h[0] + H, o = h[0] + H;
    yb = s * (d * gb[0] + o * Gb + HGb);
    yt = s * (d * gt[0] + o * Gt + HGt);
}

// Horizontal P1 mass with the column heights as weight, applied to one value
// per base vertex (a vertically constant field):
//     y_a = 2A sum_b T_ab(h) x_b = (2A / 120) ((2 h_a + H) x_a + (h_a + H) X + sum_b h_b x_b),
// X = sum_b x_b (the T of p1_mass).
__device__ __forceinline__ void tri_mass(double twoA, const double h[3], const double x[3], double y[3])
{
    const double s = twoA * (1.0 / 120.0);
    const double H = h[0] + h[1] + h[2];
    const double X = x[0] + x[1] + x[2];
    const double HX = h[0] * x[0] + h[1] * x[1] + h[2] * x[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) y[a] = s * ((2.0 * h[a] + H) * x[a] + (h[a] + H) * X + HX);
}

// Mass action of the tensor-product element with NH horizontal nodes (3:
// linear on the triangle, 1: constant) and NV vertical nodes (2: linear,
// bottom and top; 1: constant) on one prism: x[alpha][beta] -> y[alpha][beta].
template <int NH, int NV>
__device__ __forceinline__ void tp_mass(double twoA, const double h[3], const double x[NH][NV], double y[NH][NV])
{
    if constexpr (NH == 3 && NV == 2) {
        double xb[3], xt[3], yb[3], yt[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xb[a] = x[a][0];
            xt[a] = x[a][1];
        }
        p1_mass(twoA, h, xb, xt, yb, yt);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[a][0] = yb[a];
            y[a][1] = yt[a];
        }
    } else if constexpr (NH == 3) {
        double xv[3], yv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) xv[a] = x[a][0];
        tri_mass(twoA, h, xv, yv);
#pragma unroll
        for (int a = 0; a < 3; ++a) y[a][0] = yv[a];
    } else {
        const double c = twoA * (h[0] + h[1] + h[2]) * (1.0 / 6.0);
        if constexpr (NV == 2) {
            y[0][0] = c * (x[0][0] * (1.0 / 3.0) + x[0][1] * (1.0 / 6.0));
            y[0][1] = c * (x[0][0] * (1.0 / 6.0) + x[0][1] * (1.0 / 3.0));
        } else {
            y[0][0] = c * x[0][0];
        }
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

// Vertical factor of the P2 mass action, 30 V2 x per horizontal node:
// x[e][beta], g[e][beta], e = horizontal node 0..5, beta = bottom, top, middle.
__device__ __forceinline__ void p2_vertical(const double x[6][3], double g[6][3])
{
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        g[e][0] = 4.0 * x[e][0] - x[e][1] + 2.0 * x[e][2];
        g[e][1] = -x[e][0] + 4.0 * x[e][1] + 2.0 * x[e][2];
        g[e][2] = 2.0 * (x[e][0] + x[e][1]) + 16.0 * x[e][2];
    }
}

// Row i (horizontal node i, all three vertical nodes) of the P2 mass action
// from the vertical factors: yi[beta] = 2A / (2520 * 30) sum_j (sum_c h_c
// K_c[i][j]) g[j][beta].
__device__ __forceinline__ void p2_mass_row(double twoA, const double h[3], const double g[6][3], int i,
                                            double yi[3])
{
    constexpr double K[3][6][6] = EXM_P2_K_TABLE;
    const double s = twoA * (1.0 / (2520.0 * 30.0));
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const double t = h[0] * K[0][i][j] + h[1] * K[1][i][j] + h[2] * K[2][i][j];
        acc0 += t * g[j][0];
        acc1 += t * g[j][1];
        acc2 += t * g[j][2];
    }
    yi[0] = s * acc0;
    yi[1] = s * acc1;
    yi[2] = s * acc2;
}

// x[e][beta], y[e][beta]: e = horizontal node 0..5, beta = bottom, top, middle.
__device__ __forceinline__ void p2_mass(double twoA, const double h[3], const double x[6][3], double y[6][3])
{
    double g[6][3];
    p2_vertical(x, g);
#pragma unroll
    for (int i = 0; i < 6; ++i) p2_mass_row(twoA, h, g, i, y[i]);
}

// ---------------------------------------------------------------------------
// Integration of the nonlinear P1 x P1 forms.  The integrand of the cubic
// residual u^3 v det J has degree 5 horizontally and 4 vertically on these
// prisms (and so does the adjoint integrand 3 u^2 w v det J): the 7-point
// degree-5 triangle rule of Radon (centroid and two three-point orbits built
// on sqrt(15)) integrates it exactly over the triangle, and along each
// column the zeta integral is taken in closed form.  The terms linear in an
// input are the closed-form P1 mass action.
//
// The triangle points are visited one at a time and their contributions to
// the test functions summed as they go, so that no per-point table of the
// fields is held in registers.

namespace cubic {

constexpr double kS15 = 3.872983346207416885;   // sqrt(15)
constexpr double kA1 = (6.0 - kS15) / 21.0, kA2 = (6.0 + kS15) / 21.0;
constexpr double kB1 = 1.0 - 2.0 * kA1, kB2 = 1.0 - 2.0 * kA2;
constexpr double kW1 = (155.0 - kS15) / 2400.0, kW2 = (155.0 + kS15) / 2400.0;
// barycentric coordinates and weights of the triangle rule (weights sum to
// 1/2, the reference area)
constexpr double kLam[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {kA1, kA1, kB1}, {kA1, kB1, kA1}, {kB1, kA1, kA1},
                               {kA2, kA2, kB2}, {kA2, kB2, kA2}, {kB2, kA2, kA2}};
constexpr double kWt[7] = {9.0 / 80.0, kW1, kW1, kW1, kW2, kW2, kW2};

}  // namespace cubic

// The terms in u^3 and 3 u^2 w of the nonlinear P1 x P1 forms on one prism,
// added to the bottom and top rows fb, ft (F) and gb, gt (g_u); ub, ut and
// wb, wt are the bottom and top nodal values of u and w at the three
// vertices.  Along a vertical column det J is constant in zeta and, at a
// triangle point, u and w are linear in zeta between their bottom and top
// values there, so the zeta integrals against the test functions 1 - zeta
// and zeta are closed forms.  Written in the Bernstein basis of degree 3
// (a cubic c(zeta) with coefficients c_0 .. c_3 against C(3,k) (1 - zeta)^(3-k)
// zeta^k), the two moments are (4 c_0 + 3 c_1 + 2 c_2 + c_3) / 20 and
// (c_0 + 2 c_1 + 3 c_2 + 4 c_3) / 20.  For u^3 the coefficients are
// ub^(3-k) ut^k; for u^2 w they are ub^2 wb, (ub^2 wt + 2 ub ut wb) / 3,
// (2 ub ut wt + ut^2 wb) / 3 and ut^2 wt; grouped by p = ub^2, q = ut^2 and
// r = ub ut below.
//
// Every point of the triangle rule is the centroid or one of the three
// permutations of (a, a, b) of an orbit, so a linear field at the orbit point
// with b on vertex k is a X + (b - a) x_k (X the sum over the three vertices),
// and the sum over an orbit of lambda_j s is a (the orbit's sum of s) +
// (b - a) s at the point with b on vertex j; at the centroid both are a
// third of the sums.
template <bool F, bool GU>
__device__ __forceinline__ void cubic_points_orbits(double twoA, const double h[3], const double ub[3],
                                                    const double ut[3], const double wb[3], const double wt[3],
                                                    double fb[3], double ft[3], double gb[3], double gt[3])
{
    using namespace cubic;
    const double Hs = h[0] + h[1] + h[2];
    const double U0 = ub[0] + ub[1] + ub[2], U1 = ut[0] + ut[1] + ut[2];
    double W0 = 0.0, W1 = 0.0;
    if constexpr (GU) {
        W0 = wb[0] + wb[1] + wb[2];
        W1 = wt[0] + wt[1] + wt[2];
    }
    // the moments at one point: weight cw (rule weight / 20 times 2A), column
    // height hq, u and w at the bottom and top
    auto point = [&](double cw, double hq, double u0, double u1, double w0, double w1, double& sfb, double& sft,
                     double& sgb, double& sgt) {
        const double wj = cw * hq;
        const double p = u0 * u0, q = u1 * u1;
        if constexpr (F) {
            sfb = wj * (p * (4.0 * u0 + 3.0 * u1) + q * (2.0 * u0 + u1));
            sft = wj * (p * (u0 + 2.0 * u1) + q * (3.0 * u0 + 4.0 * u1));
        }
        if constexpr (GU) {
            const double r = u0 * u1, w3 = 3.0 * wj;
            sgb = w3 * (p * (4.0 * w0 + w1) + r * (2.0 * w0 + (4.0 / 3.0) * w1) + q * ((2.0 / 3.0) * w0 + w1));
            sgt = w3 * (p * (w0 + (2.0 / 3.0) * w1) + r * ((4.0 / 3.0) * w0 + 2.0 * w1) + q * (w0 + 4.0 * w1));
        }
    };
    // parts of the rows common to the three vertices
    double cfb, cft, cgb = 0.0, cgt = 0.0;
    {
        constexpr double t = 1.0 / 3.0;
        double sfb = 0.0, sft = 0.0, sgb = 0.0, sgt = 0.0;
        point(kWt[0] * (1.0 / 20.0) * twoA, t * Hs, t * U0, t * U1, t * W0, t * W1, sfb, sft, sgb, sgt);
        cfb = t * sfb;
        cft = t * sft;
        if constexpr (GU) {
            cgb = t * sgb;
            cgt = t * sgt;
        }
    }
    constexpr double kOa[2] = {kA1, kA2}, kOb[2] = {kB1, kB2}, kOw[2] = {kW1, kW2};
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double a = kOa[m], d = kOb[m] - kOa[m];
        const double cw = kOw[m] * (1.0 / 20.0) * twoA;
        const double aH = a * Hs, aU0 = a * U0, aU1 = a * U1, aW0 = a * W0, aW1 = a * W1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double sfb = 0.0, sft = 0.0, sgb = 0.0, sgt = 0.0;
            point(cw, aH + d * h[k], aU0 + d * ub[k], aU1 + d * ut[k], GU ? aW0 + d * wb[k] : 0.0,
                  GU ? aW1 + d * wt[k] : 0.0, sfb, sft, sgb, sgt);
            if constexpr (F) {
                fb[k] += d * sfb;
                ft[k] += d * sft;
                cfb += a * sfb;
                cft += a * sft;
            }
            if constexpr (GU) {
                gb[k] += d * sgb;
                gt[k] += d * sgt;
                cgb += a * sgb;
                cgt += a * sgt;
            }
            __builtin_amdgcn_sched_barrier(0);   // one point at a time: fewer live values
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if constexpr (F) {
            fb[k] += cfb;
            ft[k] += cft;
        }
        if constexpr (GU) {
            gb[k] += cgb;
            gt[k] += cgt;
        }
    }
}

// Both forms at once.  With w = u the moments of 3 u^2 w are three times
// those of u^3, and both are linear in the second factor x (u for F, w for
// g_u): (alpha x0 + beta x1, beta x0 + gamma x1) with alpha = 4p + 2r + 2q/3,
// beta = p + q + 4r/3, gamma = 2p/3 + 2r + 4q, so one set of alpha, beta,
// gamma per point serves both.  The points come from the table: the orbit
// sums would cost this form its fourth wave per SIMD.
__device__ __forceinline__ void cubic_points_both(double twoA, const double h[3], const double ub[3],
                                                  const double ut[3], const double wb[3], const double wt[3],
                                                  double fb[3], double ft[3], double gb[3], double gt[3])
{
    using namespace cubic;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const double wj =
            (kWt[i] * (1.0 / 20.0)) * (twoA * (kLam[i][0] * h[0] + kLam[i][1] * h[1] + kLam[i][2] * h[2]));
        const double u0 = kLam[i][0] * ub[0] + kLam[i][1] * ub[1] + kLam[i][2] * ub[2];
        const double u1 = kLam[i][0] * ut[0] + kLam[i][1] * ut[1] + kLam[i][2] * ut[2];
        const double w0 = kLam[i][0] * wb[0] + kLam[i][1] * wb[1] + kLam[i][2] * wb[2];
        const double w1 = kLam[i][0] * wt[0] + kLam[i][1] * wt[1] + kLam[i][2] * wt[2];
        const double p = u0 * u0, q = u1 * u1, r = u0 * u1;
        const double al = 4.0 * p + 2.0 * r + (2.0 / 3.0) * q;
        const double be = (p + q) + (4.0 / 3.0) * r;
        const double ga = (2.0 / 3.0) * p + 2.0 * r + 4.0 * q;
        const double w3 = 3.0 * wj;
        const double sfb = wj * (al * u0 + be * u1), sft = wj * (be * u0 + ga * u1);
        const double sgb = w3 * (al * w0 + be * w1), sgt = w3 * (be * w0 + ga * w1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fb[a] += kLam[i][a] * sfb;
            ft[a] += kLam[i][a] * sft;
            gb[a] += kLam[i][a] * sgb;
            gt[a] += kLam[i][a] * sgt;
        }
    }
}

template <bool F, bool GU>
__device__ __forceinline__ void cubic_points(double twoA, const double h[3], const double ub[3], const double ut[3],
                                             const double wb[3], const double wt[3], double fb[3], double ft[3],
                                             double gb[3], double gt[3])
{
    if constexpr (F && GU)
        cubic_points_both(twoA, h, ub, ut, wb, wt, fb, ft, gb, gt);
    else
        cubic_points_orbits<F, GU>(twoA, h, ub, ut, wb, wt, fb, ft, gb, gt);
}

// Nonlinear P1 x P1 element forms on one prism (b, t: bottom / top nodal
// values of each input at the three vertices; yb, yt: outputs likewise).
//   FORM 1: F = integral (u^3 - f) v             inputs u, f;    output F
//   FORM 2: g_u = integral 3 u^2 w v, g_f = -M w inputs u, w;    outputs g_u, g_f
//   FORM 3: F, g_u, g_f together                 inputs u, f, w; outputs F, g_u, g_f
// The terms linear in an input (-M f of F, g_f = -M w) are the closed-form
// P1 mass action; the quadrature carries only the terms in u^3 and 3 u^2 w.
template <int FORM>
__device__ __forceinline__ void cubic_element(double twoA, const double h[3], const double b[][3],
                                              const double t[][3], double yb[][3], double yt[][3])
{
    constexpr bool F = FORM == 1 || FORM == 3;
    constexpr bool GU = FORM == 2 || FORM == 3;
    constexpr int iw = FORM == 2 ? 1 : 2;      // input index of w
    constexpr int ou = FORM == 2 ? 0 : 1;      // output index of g_u
    double fb[3] = {0.0, 0.0, 0.0}, ft[3] = {0.0, 0.0, 0.0};   // F
    double gb[3] = {0.0, 0.0, 0.0}, gt[3] = {0.0, 0.0, 0.0};   // g_u
    if constexpr (F) {   // F starts from -M f
        p1_mass(twoA, h, b[1], t[1], fb, ft);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            fb[a] = -fb[a];
            ft[a] = -ft[a];
        }
    }
    cubic_points<F, GU>(twoA, h, b[0], t[0], b[iw], t[iw], fb, ft, gb, gt);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (F) {
            yb[0][a] = fb[a];
            yt[0][a] = ft[a];
        }
        if constexpr (GU) {
            yb[ou][a] = gb[a];
            yt[ou][a] = gt[a];
        }
    }
    if constexpr (GU) {   // g_f = -M w
        double mb[3], mt[3];
        p1_mass(twoA, h, b[iw], t[iw], mb, mt);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            yb[ou + 1][a] = -mb[a];
            yt[ou + 1][a] = -mt[a];
        }
    }
}

}  // namespace exm
