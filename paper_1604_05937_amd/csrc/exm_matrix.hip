// Matrices of bilinear forms in the extruded layout.
//
// The vertical-innermost numbering (Algorithm 1) puts the DoFs of one node of
// an entity column at a fixed stride: node alpha of entity e sits at
// c0 + s * w for its slots s = 0, 1, ... (c0 = S(e) + alpha, w = DoFs per level
// of the column, Algorithm 2's offset).  Call such a run a class.  Two DoFs
// couple when they share a prism, so a class couples with the classes of the
// base cells around its entity, and only at slot distance -1, 0 or +1.  The
// matrix therefore needs no column index per entry: the classes a class
// couples with (a pattern over base entities, the same at every level) and,
// per pattern entry, three values per slot (one per slot distance), stored
// slot-innermost so that a wavefront of consecutive slots reads them in one
// coalesced sweep.  This is the vertical alignment of the global matrix that
// Section 5 points to; CSR with per-entry column indices is produced on
// request.
//
// Assembly gathers: one thread per (pattern entry, slot) sums the element
// matrix entries of every prism that contributes to it (the base cells that
// hold both classes, layers s - 1 and s) and writes its values once, so no
// atomics, no colouring and a bitwise reproducible result.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "exm_elements.hpp"
#include "exm_internal.hpp"

namespace exm {
namespace {

constexpr int kKindH = 0;   // a node on a level (horizontal DoF): slots 0 .. lambda
constexpr int kKindV = 1;   // a node inside a layer (vertical DoF): slots 0 .. lambda - 1

// Do a row class of kind kr at slot s and a column class of kind kq at slot
// s + d share a prism?  A level node belongs to the layers below and above
// it, a layer node to its own layer.
__host__ __device__ inline bool pair_valid(int kr, int kq, int d, int s, int lam)
{
    const int r0 = kr == kKindV ? s : s - 1, r1 = s;
    const int t = s + d;
    const int c0 = kq == kKindV ? t : t - 1, c1 = t;
    const int lo = std::max(std::max(r0, c0), 0);
    const int hi = std::min(std::min(r1, c1), lam - 1);
    return lo <= hi;
}

// Horizontal and vertical factors of the tensor-product elements: the mass of
// a prism with vertical columns is 2A * T(h) (x) V exactly (the Jacobian
// determinant is 2A times the linear interpolant of the column heights).
//   HK 0: the three P1 barycentric functions, T_ab = (h_a + h_b + H)(1 + [a = b]) / 120
//   HK 1: the constant, T = H / 6
//   HK 2: the six P2 functions, T_ab = sum_c h_c K_c[a][b] / 2520
//   VK 0: linear on [0, 1] (bottom, top), V = [[1/3, 1/6], [1/6, 1/3]]
//   VK 1: the constant, V = 1
//   VK 2: quadratic (bottom, top, middle), V = [[4, -1, 2], [-1, 4, 2], [2, 2, 16]] / 30
struct ElementKinds {
    int hk, vk;
};

ElementKinds element_kinds(int32_t el)
{
    switch (el) {
    case EXM_ELEMENT_P1P1: return {0, 0};
    case EXM_ELEMENT_DG0DG0: return {1, 1};
    case EXM_ELEMENT_DG1DG1: return {0, 0};
    case EXM_ELEMENT_P2P2: return {2, 2};
    case EXM_ELEMENT_P1DG0: return {0, 1};
    case EXM_ELEMENT_P1DG1: return {0, 0};
    case EXM_ELEMENT_DG0P1: return {1, 0};
    case EXM_ELEMENT_DG0DG1: return {1, 0};
    case EXM_ELEMENT_DG1P1: return {0, 0};
    default: return {0, 1};   // DG1DG0
    }
}

// Horizontal node a and vertical node b of stencil position p (the order of
// the explicit lists: per closure entity its bottom, top and vertical DoFs).
void position_nodes(int32_t el, int p, int& a, int& b)
{
    switch (el) {
    case EXM_ELEMENT_P1P1:
    case EXM_ELEMENT_DG1DG1:
    case EXM_ELEMENT_P1DG1: a = p / 2; b = p % 2; return;
    case EXM_ELEMENT_P2P2: a = p / 3; b = p % 3; return;
    case EXM_ELEMENT_DG0DG0: a = 0; b = 0; return;
    case EXM_ELEMENT_DG0P1:
    case EXM_ELEMENT_DG0DG1: a = 0; b = p; return;
    case EXM_ELEMENT_DG1P1: a = p % 3; b = p / 3; return;
    default: a = p; b = 0; return;   // P1DG0, DG1DG0
    }
}

template <int HK>
__device__ __forceinline__ double mass_T(const double h[3], int ai, int aj)
{
    const double H = h[0] + h[1] + h[2];
    double T;
    if constexpr (HK == 0) {
        // h_a + h_b + H, doubled on the diagonal (selects, not an indexed array)
        const double s = (ai == 0 || aj == 0 ? h[0] : 0.0) + (ai == 1 || aj == 1 ? h[1] : 0.0) +
                         (ai == 2 || aj == 2 ? h[2] : 0.0);
        T = ai == aj ? (2.0 * s + H) * (1.0 / 60.0) : (s + H) * (1.0 / 120.0);
    } else if constexpr (HK == 1) {
        T = H * (1.0 / 6.0);
    } else {
        constexpr double K[3][6][6] = EXM_P2_K_TABLE;
        T = (h[0] * K[0][ai][aj] + h[1] * K[1][ai][aj] + h[2] * K[2][ai][aj]) * (1.0 / 2520.0);
    }
    return T;
}

template <int VK>
__device__ __forceinline__ double mass_V(int bi, int bj)
{
    double V;
    if constexpr (VK == 0) {
        V = bi == bj ? 1.0 / 3.0 : 1.0 / 6.0;
    } else if constexpr (VK == 1) {
        V = 1.0;
    } else {
        constexpr double V2[3][3] = {{4.0, -1.0, 2.0}, {-1.0, 4.0, 2.0}, {2.0, 2.0, 16.0}};
        V = V2[bi][bj] * (1.0 / 30.0);
    }
    return V;
}


// Jacobian of the cubic residual on a P1 prism, integral 3 u^2 phi_j phi_i
// det J, with the triangle rule of the residual (7-point Radon, exact for
// this degree) and the zeta integrals in closed form.  Per prism, the
// vertical moments of 3 u^2 det J at every triangle point,
//     m[t][k] = 3 w_t dj_t integral_0^1 u(t, z)^2 (1 - z)^(2 - k) z^k dz,  k = 0, 1, 2,
// serve all its entries: entry (a_i, b_i), (a_j, b_j) = sum_t lambda_ai
// lambda_aj m[t][b_i + b_j].  ub, ut: u at the bottom and top node of the
// three vertices.  With u = u0 (1 - z) + u1 z, u^2 = p (1 - z)^2 + 2 r z (1 - z)
// + q z^2 (p = u0^2, r = u0 u1, q = u1^2), and the integral of (1 - z)^a z^b
// over [0, 1] is a! b! / (a + b + 1)!, so the three moments are
// p/5 + r/10 + q/30, p/20 + r/15 + q/20 and p/30 + r/10 + q/5.
__device__ __forceinline__ void cubic_jac_moments(double twoA, const double h[3], const double ub[3],
                                                  const double ut[3], double m[7][3])
{
    using namespace cubic;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        const double dj = twoA * (kLam[t][0] * h[0] + kLam[t][1] * h[1] + kLam[t][2] * h[2]);
        const double u0 = kLam[t][0] * ub[0] + kLam[t][1] * ub[1] + kLam[t][2] * ub[2];
        const double u1 = kLam[t][0] * ut[0] + kLam[t][1] * ut[1] + kLam[t][2] * ut[2];
        const double p = u0 * u0, r = u0 * u1, q = u1 * u1;
        const double s0 = p * (1.0 / 5.0) + r * (1.0 / 10.0) + q * (1.0 / 30.0);
        const double s1 = p * (1.0 / 20.0) + r * (1.0 / 15.0) + q * (1.0 / 20.0);
        const double s2 = p * (1.0 / 30.0) + r * (1.0 / 10.0) + q * (1.0 / 5.0);
        const double c = 3.0 * kWt[t] * dj;
        m[t][0] = c * s0;
        m[t][1] = c * s1;
        m[t][2] = c * s2;
    }
}

__device__ __forceinline__ double cubic_jac_entry(const double m[7][3], int ai, int aj, int bb)
{
    using namespace cubic;
    // weights instead of an index, so that the moments stay in registers
    const double w0 = bb == 0 ? 1.0 : 0.0, w1 = bb == 1 ? 1.0 : 0.0, w2 = bb == 2 ? 1.0 : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        const double li = ai == 0 ? kLam[t][0] : (ai == 1 ? kLam[t][1] : kLam[t][2]);
        const double lj = aj == 0 ? kLam[t][0] : (aj == 1 ? kLam[t][1] : kLam[t][2]);
        acc += li * lj * (w0 * m[t][0] + w1 * m[t][1] + w2 * m[t][2]);
    }
    return acc;
}

__device__ __forceinline__ unsigned xcd_block_m(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Rows of at most this many pattern entries take the Jacobian by rows.
constexpr int kRowEntries = 8;

struct GatherArgs {
    int32_t lam, L, band;
    int64_t n_pat;                        // pattern entries
    const int64_t* __restrict__ pc_ptr;   // [n_pat + 1] contributions of every pattern entry
    const int32_t* __restrict__ pc_cell;  // base cell of every contribution (ascending within an entry)
    const int32_t* __restrict__ pc_info;  // a_i | a_j << 3 | b_i << 6 | b_j << 8 | top_i << 10 | top_j << 11
    const int32_t* __restrict__ xmap;     // coordinate lists [n_cells * 6]
    const double* __restrict__ X;         // coordinates, component-major
    int64_t xn;
    const int32_t* __restrict__ fmap;     // field lists (Jacobian: u's space, P1 x P1)
    const double* __restrict__ u;
    double* __restrict__ val;             // [n_pat][band][L]
    // by rows (k_mat_jac_rows): the contributions to the entries of each row
    // class, ordered by cell, with the entry's place in its row
    int32_t n_rows;
    const int32_t* __restrict__ pptr;     // [n_rows + 1] first pattern entry of every row
    const int64_t* __restrict__ rc_ptr;   // [n_rows + 1]
    const int32_t* __restrict__ rc_cell;
    const int32_t* __restrict__ rc_info;  // pc_info | (entry - first entry of the row) << 12
};

// One wavefront per (pattern entry p, 64 consecutive slots): the entry, its
// contribution list, the cells and their base geometry are the same for
// every lane (scalar loads); the lanes read z (and u) of their own levels,
// contiguous along the columns, and write their values in one coalesced
// sweep.  (Issuing the next cell's loads before the current cell's entries
// measured slower: the registers it takes cost more occupancy than the
// latency it hides.)
template <int HK, int VK, bool JAC>
__global__ void __launch_bounds__(256) k_mat_gather(const GatherArgs g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_m(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int nsteps = (g.L + 63) >> 6;
    const int64_t p = wid / nsteps;
    if (p >= g.n_pat) return;   // uniform over the wavefront
    const int s = (int)(wid - p * nsteps) * 64 + lane;
    const bool act = s < g.L;
    double acc[3] = {0.0, 0.0, 0.0};
    int64_t e = g.pc_ptr[p];
    const int64_t end = g.pc_ptr[p + 1];
    const double* __restrict__ Z = g.X + 2 * g.xn;
    while (e < end) {
        const int32_t c = g.pc_cell[e];
        double x[3], y[3], hlo[3], hhi[3], ul[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int xb = g.xmap[(int64_t)c * 6 + 2 * a];
            x[a] = g.X[xb];
            y[a] = g.X[g.xn + xb];
            // z at levels s - 1, s, s + 1 (those inside the column)
            double z[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lev = s - 1 + k;
                z[k] = act && lev >= 0 && lev <= g.lam ? Z[xb + lev] : 0.0;
            }
            hlo[a] = z[1] - z[0];   // layer s - 1
            hhi[a] = z[2] - z[1];   // layer s
            if constexpr (JAC) {
                const int fb = g.fmap[(int64_t)c * 6 + 2 * a];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int lev = s - 1 + k;
                    ul[a][k] = act && lev >= 0 && lev <= g.lam ? g.u[fb + lev] : 0.0;
                }
            }
        }
        const double twoA = twice_area(x, y);
        double mlo[7][3], mhi[7][3];   // Jacobian: moments of the prisms of layers s - 1 and s
        if constexpr (JAC) {
            double ub[3], ut[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ub[a] = ul[a][0];
                ut[a] = ul[a][1];
            }
            cubic_jac_moments(twoA, hlo, ub, ut, mlo);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ub[a] = ul[a][1];
                ut[a] = ul[a][2];
            }
            cubic_jac_moments(twoA, hhi, ub, ut, mhi);
        }
        // the horizontal nodes of the row and column classes are the same in
        // every contribution of this cell (checked when the plan is built):
        // 2A T(h) of both layers, or the Jacobian's entries, once
        const int info0 = g.pc_info[e];
        const int ai0 = info0 & 7, aj0 = (info0 >> 3) & 7;
        double Tlo = 0.0, Thi = 0.0;
        double Jlo[3], Jhi[3];   // Jacobian: the entry of either layer for vertical nodes summing to 0, 1, 2
        if constexpr (!JAC) {
            Tlo = twoA * mass_T<HK>(hlo, ai0, aj0);
            Thi = twoA * mass_T<HK>(hhi, ai0, aj0);
        } else {
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                Jlo[bb] = cubic_jac_entry(mlo, ai0, aj0, bb);
                Jhi[bb] = cubic_jac_entry(mhi, ai0, aj0, bb);
            }
        }
        for (; e < end && g.pc_cell[e] == c; ++e) {
            const int info = g.pc_info[e];
            const int bi = (info >> 6) & 3, bj = (info >> 8) & 3;
            const int ti = (info >> 10) & 1, tj = (info >> 11) & 1;
            const int l = s - ti;   // the prism: the row node is its top (layer s - 1) or bottom / inside (layer s)
            if (l < 0 || l >= g.lam) continue;
            double v;
            if constexpr (JAC) {
                const int bb = bi + bj;
                const double vlo = bb == 0 ? Jlo[0] : (bb == 1 ? Jlo[1] : Jlo[2]);
                const double vhi = bb == 0 ? Jhi[0] : (bb == 1 ? Jhi[1] : Jhi[2]);
                v = ti ? vlo : vhi;
            } else {
                v = (ti ? Tlo : Thi) * mass_V<VK>(bi, bj);
            }
            const int d = tj - ti;
            if (d < 0) acc[0] += v;
            else if (d == 0) acc[1] += v;
            else acc[2] += v;
        }
    }
    if (!act) return;
    if (g.band == 3) {
#pragma unroll
        for (int d = 0; d < 3; ++d) g.val[(p * 3 + d) * g.L + s] = acc[d];
    } else {
        g.val[p * g.L + s] = acc[1];
    }
}

// The cubic Jacobian by rows (P1 x P1, every row of at most NE entries): one
// wavefront per (row class r, 64 consecutive slots) takes the cells around
// the row's vertex once each.  A cell's moments of either layer become the
// nine entries of the row's vertex against the cell's three vertices (one
// per sum of vertical nodes) right away, so that the moments do not stay
// live, and every contribution of the cell picks its entry.
template <int NE>
__global__ void __launch_bounds__(256) k_mat_jac_rows(const GatherArgs g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_m(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int nsteps = (g.L + 63) >> 6;
    const int64_t r = wid / nsteps;
    if (r >= g.n_rows) return;   // uniform over the wavefront
    const int s = (int)(wid - r * nsteps) * 64 + lane;
    const bool act = s < g.L;
    double acc[NE][3];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
    int64_t e = g.rc_ptr[r];
    const int64_t end = g.rc_ptr[r + 1];
    const double* __restrict__ Z = g.X + 2 * g.xn;
    while (e < end) {
        const int32_t c = g.rc_cell[e];
        const int ai = g.rc_info[e] & 7;   // the row's vertex in this cell (the same in all its contributions)
        double x[3], y[3], hlo[3], hhi[3], ul[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int xb = g.xmap[(int64_t)c * 6 + 2 * a];
            x[a] = g.X[xb];
            y[a] = g.X[g.xn + xb];
            double z[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lev = s - 1 + k;
                z[k] = act && lev >= 0 && lev <= g.lam ? Z[xb + lev] : 0.0;
            }
            hlo[a] = z[1] - z[0];
            hhi[a] = z[2] - z[1];
            const int fb = g.fmap[(int64_t)c * 6 + 2 * a];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lev = s - 1 + k;
                ul[a][k] = act && lev >= 0 && lev <= g.lam ? g.u[fb + lev] : 0.0;
            }
        }
        const double twoA = twice_area(x, y);
        double J[2][3][3];   // layer (s - 1, s), column vertex aj, sum of vertical nodes
#pragma unroll
        for (int ly = 0; ly < 2; ++ly) {
            double m[7][3], ub[3], ut[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ub[a] = ul[a][ly];
                ut[a] = ul[a][ly + 1];
            }
            cubic_jac_moments(twoA, ly == 0 ? hlo : hhi, ub, ut, m);
#pragma unroll
            for (int aj = 0; aj < 3; ++aj)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) J[ly][aj][bb] = cubic_jac_entry(m, ai, aj, bb);
        }
        for (; e < end && g.rc_cell[e] == c; ++e) {
            const int info = g.rc_info[e];
            const int aj = (info >> 3) & 7, bi = (info >> 6) & 3, bj = (info >> 8) & 3;
            const int ti = (info >> 10) & 1, tj = (info >> 11) & 1, le = info >> 12;
            const int l = s - ti;   // the prism: the row node is its top (layer s - 1) or bottom (layer s)
            if (l < 0 || l >= g.lam) continue;
            const int ly = ti ? 0 : 1, bb = bi + bj;
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)   // aj, bb and ti are the same on every lane
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (a == aj && b == bb) v = ly == 0 ? J[0][a][b] : J[1][a][b];
            const int d = tj - ti + 1;
#pragma unroll
            for (int q = 0; q < NE; ++q)   // le is the same on every lane
                if (q == le) {
                    if (d == 0) acc[q][0] += v;
                    else if (d == 1) acc[q][1] += v;
                    else acc[q][2] += v;
                }
        }
    }
    if (!act) return;
    const int32_t p0 = g.pptr[r], ne = g.pptr[r + 1] - p0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if (q >= ne) break;
        const int64_t p = p0 + q;
#pragma unroll
        for (int d = 0; d < 3; ++d) g.val[(p * 3 + d) * g.L + s] = acc[q][d];
    }
}

// The mass form by rows (every row of at most NE entries): one wavefront per
// (row class r, 64 consecutive slots) takes the cells around the row's
// entity once each; a cell's contributions come in entry order, and 2A T(h)
// of both layers is formed once per entry.
template <int HK, int VK, int NE>
__global__ void __launch_bounds__(256) k_mat_mass_rows(const GatherArgs g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_m(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int nsteps = (g.L + 63) >> 6;
    const int64_t r = wid / nsteps;
    if (r >= g.n_rows) return;   // uniform over the wavefront
    const int s = (int)(wid - r * nsteps) * 64 + lane;
    const bool act = s < g.L;
    double acc[NE][3];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
    int64_t e = g.rc_ptr[r];
    const int64_t end = g.rc_ptr[r + 1];
    const double* __restrict__ Z = g.X + 2 * g.xn;
    while (e < end) {
        const int32_t c = g.rc_cell[e];
        double x[3], y[3], hlo[3], hhi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int xb = g.xmap[(int64_t)c * 6 + 2 * a];
            x[a] = g.X[xb];
            y[a] = g.X[g.xn + xb];
            double z[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int lev = s - 1 + k;
                z[k] = act && lev >= 0 && lev <= g.lam ? Z[xb + lev] : 0.0;
            }
            hlo[a] = z[1] - z[0];
            hhi[a] = z[2] - z[1];
        }
        const double twoA = twice_area(x, y);
        int cur = -1;   // the entry whose factors are formed
        double Tlo = 0.0, Thi = 0.0;
        for (; e < end && g.rc_cell[e] == c; ++e) {
            const int info = g.rc_info[e];
            const int le = info >> 12;
            if (le != cur) {   // the same on every lane
                const int ai = info & 7, aj = (info >> 3) & 7;
                Tlo = twoA * mass_T<HK>(hlo, ai, aj);
                Thi = twoA * mass_T<HK>(hhi, ai, aj);
                cur = le;
            }
            const int bi = (info >> 6) & 3, bj = (info >> 8) & 3;
            const int ti = (info >> 10) & 1, tj = (info >> 11) & 1;
            const int l = s - ti;
            if (l < 0 || l >= g.lam) continue;
            const double v = (ti ? Tlo : Thi) * mass_V<VK>(bi, bj);
            const int d = tj - ti + 1;
#pragma unroll
            for (int q = 0; q < NE; ++q)   // le is the same on every lane
                if (q == le) {
                    if (d == 0) acc[q][0] += v;
                    else if (d == 1) acc[q][1] += v;
                    else acc[q][2] += v;
                }
        }
    }
    if (!act) return;
    const int32_t p0 = g.pptr[r], ne = g.pptr[r + 1] - p0;
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        if (q >= ne) break;
        const int64_t p = p0 + q;
        if (g.band == 3) {
#pragma unroll
            for (int d = 0; d < 3; ++d) g.val[(p * 3 + d) * g.L + s] = acc[q][d];
        } else {
            g.val[p * g.L + s] = acc[q][1];
        }
    }
}

struct RowArgs {
    int32_t lam, L, band, write;
    int32_t n_classes;
    int64_t n_items;                      // classes x slots
    const int32_t* __restrict__ c0;       // [n_classes] DoF at slot 0
    const int32_t* __restrict__ wk;       // [n_classes] stride | kind << 16
    const int32_t* __restrict__ pptr;     // [n_classes + 1]
    const int32_t* __restrict__ pcol;     // [n_pat]
    const double* __restrict__ val;
    const double* __restrict__ x;
    double* __restrict__ y;
    const int64_t* __restrict__ rowptr;   // CSR export
    int64_t* __restrict__ cnt;
    int32_t* __restrict__ ccol;
    double* __restrict__ cval;
};

// y = A x, one wavefront per (class r, 64 consecutive slots): the pattern
// row and the coupled classes are the same for every lane (scalar loads);
// each lane reads its slot's values (coalesced across the lanes) and x at the
// neighbouring slots of the coupled class.
__global__ void __launch_bounds__(256) k_mat_spmv(const RowArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_m(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int nsteps = (a.L + 63) >> 6;
    const int32_t r = (int32_t)(wid / nsteps);
    if (r >= a.n_classes) return;   // uniform over the wavefront
    const int s = (int)(wid - (int64_t)r * nsteps) * 64 + lane;
    const int wr = a.wk[r] & 0xffff, kr = a.wk[r] >> 16;
    if (s >= a.L || (kr == kKindV && s == a.lam)) return;   // no such row
    double acc = 0.0;
    for (int32_t p = a.pptr[r]; p < a.pptr[r + 1]; ++p) {
        const int32_t q = a.pcol[p];
        const int64_t cq = a.c0[q];
        const int wq = a.wk[q] & 0xffff, kq = a.wk[q] >> 16;
        if (a.band == 3) {
#pragma unroll
            for (int d = -1; d <= 1; ++d)
                if (pair_valid(kr, kq, d, s, a.lam))
                    acc += a.val[((int64_t)p * 3 + d + 1) * a.L + s] * a.x[cq + (int64_t)(s + d) * wq];
        } else {
            acc += a.val[(int64_t)p * a.L + s] * a.x[cq + (int64_t)s * wq];
        }
    }
    const int64_t row = a.c0[r] + (int64_t)s * wr;
    if (a.write)
        a.y[row] = acc;
    else
        a.y[row] += acc;
}

// CSR export, pass 1: entries of every row.
__global__ void __launch_bounds__(256) k_csr_count(const RowArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n_items) return;
    const int32_t r = (int32_t)(idx / a.L);
    const int s = (int)(idx - (int64_t)r * a.L);
    const int wr = a.wk[r] & 0xffff, kr = a.wk[r] >> 16;
    if (kr == kKindV && s == a.lam) return;
    int64_t n = 0;
    for (int32_t p = a.pptr[r]; p < a.pptr[r + 1]; ++p) {
        const int kq = a.wk[a.pcol[p]] >> 16;
        for (int d = -1; d <= 1; ++d)
            if ((a.band == 3 || d == 0) && pair_valid(kr, kq, d, s, a.lam)) ++n;
    }
    a.cnt[a.c0[r] + (int64_t)s * wr] = n;
}

// CSR export, pass 2: column indices and values of every row, sorted by column.
__global__ void __launch_bounds__(256) k_csr_fill(const RowArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.n_items) return;
    const int32_t r = (int32_t)(idx / a.L);
    const int s = (int)(idx - (int64_t)r * a.L);
    const int wr = a.wk[r] & 0xffff, kr = a.wk[r] >> 16;
    if (kr == kKindV && s == a.lam) return;
    const int64_t row = a.c0[r] + (int64_t)s * wr;
    const int64_t b = a.rowptr[row];
    int64_t n = 0;
    for (int32_t p = a.pptr[r]; p < a.pptr[r + 1]; ++p) {
        const int32_t q = a.pcol[p];
        const int64_t cq = a.c0[q];
        const int wq = a.wk[q] & 0xffff, kq = a.wk[q] >> 16;
        for (int d = -1; d <= 1; ++d) {
            if (!((a.band == 3 || d == 0) && pair_valid(kr, kq, d, s, a.lam))) continue;
            const int32_t col = (int32_t)(cq + (int64_t)(s + d) * wq);
            const double v = a.val[((int64_t)p * a.band + (a.band == 3 ? d + 1 : 0)) * a.L + s];
            // insertion into the sorted prefix of the row
            int64_t j = n;
            while (j > 0 && a.ccol[b + j - 1] > col) {
                a.ccol[b + j] = a.ccol[b + j - 1];
                a.cval[b + j] = a.cval[b + j - 1];
                --j;
            }
            a.ccol[b + j] = col;
            a.cval[b + j] = v;
            ++n;
        }
    }
}

// ---------------------------------------------------------------------------
// In-place inclusive scan of int64 values for the CSR export without
// allocation: segments of kScanSeg values per workgroup, the segment totals
// in `scratch`, then one workgroup scans the totals and every segment adds its
// offset.

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
constexpr int64_t kScanSeg = (int64_t)kScanThreads * kScanPer;
constexpr int64_t kScanMaxSegs = 65536;

__device__ __forceinline__ int64_t wave_inclusive(int64_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive prefix over the workgroup of one value per thread; *total gets
// the workgroup's sum.
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* total)
{
    __shared__ int64_t wsum[kScanThreads / 64 + 1];   // per-wave offsets, then the total
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t inc = wave_inclusive(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        const int64_t x = lane < kScanThreads / 64 ? wsum[lane] : 0;
        const int64_t xi = wave_inclusive(x);
        if (lane < kScanThreads / 64) wsum[lane] = xi - x;
        if (lane == kScanThreads / 64 - 1) wsum[kScanThreads / 64] = xi;
    }
    __syncthreads();
    const int64_t r = wsum[w] + inc - v;
    *total = wsum[kScanThreads / 64];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_segments(int64_t* __restrict__ a, int64_t n,
                                                                int64_t* __restrict__ seg_total)
{
    const int64_t base = (int64_t)blockIdx.x * kScanSeg + (int64_t)threadIdx.x * kScanPer;
    int64_t v[kScanPer];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? a[base + k] : 0;
        run += v[k];
        v[k] = run;
    }
    int64_t total;
    const int64_t off = block_exclusive(run, &total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) a[base + k] = v[k] + off;
    if (threadIdx.x == 0) seg_total[blockIdx.x] = total;
}

// Exclusive scan of the nseg segment totals, in place, by one workgroup.
__global__ void __launch_bounds__(kScanThreads) k_scan_totals(int64_t* __restrict__ t, int64_t nseg)
{
    const int64_t per = (nseg + kScanThreads - 1) / kScanThreads;
    const int64_t b = (int64_t)threadIdx.x * per;
    int64_t run = 0;
    for (int64_t i = b; i < b + per && i < nseg; ++i) run += t[i];
    int64_t total;
    int64_t off = block_exclusive(run, &total);
    for (int64_t i = b; i < b + per && i < nseg; ++i) {
        const int64_t x = t[i];
        t[i] = off;
        off += x;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int64_t* __restrict__ a, int64_t n,
                                                           const int64_t* __restrict__ seg_off)
{
    const int64_t add = seg_off[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanSeg;
    for (int k = threadIdx.x; k < kScanSeg; k += kScanThreads)
        if (base + k < n) a[base + k] += add;
}

// The CSR export's first pass writing its counts straight into the row
// pointers: rowptr[row + 1] = entries of the row, rowptr[0] = 0.
__global__ void __launch_bounds__(256) k_csr_count_rowptr(const RowArgs a, int64_t* __restrict__ rowptr)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx == 0) rowptr[0] = 0;
    if (idx >= a.n_items) return;
    const int32_t r = (int32_t)(idx / a.L);
    const int s = (int)(idx - (int64_t)r * a.L);
    const int wr = a.wk[r] & 0xffff, kr = a.wk[r] >> 16;
    if (kr == kKindV && s == a.lam) return;
    int64_t n = 0;
    for (int32_t p = a.pptr[r]; p < a.pptr[r + 1]; ++p) {
        const int kq = a.wk[a.pcol[p]] >> 16;
        for (int d = -1; d <= 1; ++d)
            if ((a.band == 3 || d == 0) && pair_valid(kr, kq, d, s, a.lam)) ++n;
    }
    rowptr[a.c0[r] + (int64_t)s * wr + 1] = n;
}

}  // namespace

// Workspace of exm_matrix_csr_noalloc: the segment totals of the scan of the
// row pointers (at most kScanMaxSegs segments of kScanSeg rows, 512 KiB).
// Every GPU the library runs on holds its own copy for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// gives on that device.
static __device__ __align__(256) int64_t scratch[kScanMaxSegs];

}  // namespace exm

using namespace exm;

struct exm_matrix {
    const exm_space* space = nullptr;
    int32_t element = 0, lam = 0, L = 0, band = 3;
    int32_t n_classes = 0;
    int64_t n_pat = 0, n_contrib = 0, nnz = 0;
    DevBuf<int32_t> c0, wk, pptr, pcol;
    DevBuf<int64_t> pc_ptr;
    DevBuf<int32_t> pc_cell, pc_info;
    DevBuf<int64_t> rc_ptr;   // by rows, when no row has more than kRowEntries entries
    DevBuf<int32_t> rc_cell, rc_info;
    DevBuf<double> val;
};

extern "C" {

int32_t exm_matrix_create(const exm_space* space, exm_matrix** out)
{
    clear_error();
    EXM_CHECK(space != nullptr && out != nullptr, EXM_EINVAL, "space or out is NULL");
    EXM_CHECK(space->element != EXM_ELEMENT_NONE, EXM_EINVAL, "the space has no element");
    const exm_mesh* mesh = space->mesh;
    EXM_CHECK(!mesh->variable, EXM_EUNSUPPORTED, "matrices take meshes with one layer count per column");
    EXM_CHECK(!space->mixed, EXM_EUNSUPPORTED, "matrices take spaces with one DoF count per entity type");
    auto A = std::make_unique<exm_matrix>();
    A->space = space;
    A->element = space->element;
    A->lam = mesh->n_layers;
    A->L = A->lam + 1;
    const int32_t* delta = space->delta;
    bool any_h = false;
    int64_t cbase[3], nclass = 0;
    int32_t w[3];
    for (int d = 0; d < 3; ++d) {
        w[d] = delta[2 * d] + delta[2 * d + 1];
        any_h = any_h || delta[2 * d] > 0;
        cbase[d] = nclass;
        nclass += (int64_t)mesh->n[d] * w[d];
    }
    A->band = any_h ? 3 : 1;   // only layer nodes: couplings stay within one slot
    EXM_CHECK(nclass < INT32_MAX, EXM_EOVERFLOW, "%lld classes exceed the int32 range", (long long)nclass);
    A->n_classes = (int32_t)nclass;
    // classes: node alpha of entity e (dimension d), in Algorithm 1's order
    std::vector<int32_t> c0(nclass), wk(nclass);
    for (int d = 0; d < 3; ++d)
        for (int32_t e = 0; e < mesh->n[d]; ++e)
            for (int al = 0; al < w[d]; ++al) {
                const int64_t id = cbase[d] + (int64_t)e * w[d] + al;
                c0[id] = (int32_t)(space->base[d] + (int64_t)e * space->col_size[d] + al);
                wk[id] = w[d] | ((al < delta[2 * d] ? kKindH : kKindV) << 16);
            }
    // stencil positions: class offset within the entity, top flag, nodes
    struct Pos {
        int ent, al, top, a, b;
    };
    std::vector<Pos> pos;
    for (int ent = 0; ent < 7; ++ent) {
        const int d = ent < 3 ? 0 : (ent < 6 ? 1 : 2);
        const int nh = delta[2 * d], nv = delta[2 * d + 1];
        for (int part = 0; part < 3; ++part)
            for (int j = 0; j < (part < 2 ? nh : nv); ++j)
                pos.push_back({ent, part == 2 ? nh + j : j, part == 1 ? 1 : 0, 0, 0});
    }
    const int k = (int)pos.size();
    EXM_CHECK(k == space->k, EXM_EINVAL, "stencil layout mismatch (%d vs %d)", k, space->k);
    for (int p = 0; p < k; ++p) position_nodes(A->element, p, pos[p].a, pos[p].b);
    const int32_t nc = mesh->n[2];
    const int32_t* cv = mesh->h_cell_vertex.data();
    const int32_t* ce = mesh->h_cell_edge.empty() ? nullptr : mesh->h_cell_edge.data();
    auto cls_of = [&](int32_t cell, int p) -> int32_t {
        const int ent = pos[p].ent;
        const int d = ent < 3 ? 0 : (ent < 6 ? 1 : 2);
        const int32_t i = d == 0 ? cv[cell * 3 + ent] : (d == 1 ? ce[cell * 3 + (ent - 3)] : cell);
        return (int32_t)(cbase[d] + (int64_t)i * w[d] + pos[p].al);
    };
    // pattern: the classes of the cells around each class
    std::vector<std::vector<int32_t>> rows(nclass);
    std::vector<int32_t> cc(k);
    for (int32_t cell = 0; cell < nc; ++cell) {
        for (int p = 0; p < k; ++p) cc[p] = cls_of(cell, p);
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) rows[cc[p]].push_back(cc[q]);
    }
    std::vector<int32_t> pptr(nclass + 1, 0), pcol;
    for (int64_t r = 0; r < nclass; ++r) {
        auto& v = rows[r];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        EXM_CHECK((int64_t)pcol.size() + (int64_t)v.size() < INT32_MAX, EXM_EOVERFLOW, "pattern exceeds int32");
        pptr[r + 1] = pptr[r] + (int32_t)v.size();
        pcol.insert(pcol.end(), v.begin(), v.end());
        std::vector<int32_t>().swap(v);
    }
    A->n_pat = (int64_t)pcol.size();
    // contributions (cell, i, j) of every pattern entry, by counting sort
    const int64_t ncon = (int64_t)nc * k * k;
    std::vector<int32_t> pidx(ncon);
    std::vector<int64_t> pc_ptr(A->n_pat + 1, 0);
    for (int32_t cell = 0; cell < nc; ++cell) {
        for (int p = 0; p < k; ++p) cc[p] = cls_of(cell, p);
        for (int i = 0; i < k; ++i) {
            const int32_t* rb = pcol.data() + pptr[cc[i]];
            const int32_t* re = pcol.data() + pptr[cc[i] + 1];
            for (int j = 0; j < k; ++j) {
                const int32_t pe = (int32_t)(std::lower_bound(rb, re, cc[j]) - pcol.data());
                pidx[((int64_t)cell * k + i) * k + j] = pe;
                ++pc_ptr[pe + 1];
            }
        }
    }
    std::partial_sum(pc_ptr.begin(), pc_ptr.end(), pc_ptr.begin());
    std::vector<int32_t> pc_cell(ncon), pc_info(ncon);
    {
        std::vector<int64_t> fill(pc_ptr.begin(), pc_ptr.end() - 1);
        for (int32_t cell = 0; cell < nc; ++cell)
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) {
                    const int64_t at = fill[pidx[((int64_t)cell * k + i) * k + j]]++;
                    pc_cell[at] = cell;
                    pc_info[at] = pos[i].a | pos[j].a << 3 | pos[i].b << 6 | pos[j].b << 8 | pos[i].top << 10 |
                                  pos[j].top << 11;
                }
    }
    A->n_contrib = ncon;
    // the assembly forms a cell's horizontal factor once per pattern entry:
    // every contribution of one cell to one entry must pair the same
    // horizontal nodes (a class is one node of one entity)
    for (int64_t p = 0; p < A->n_pat; ++p)
        for (int64_t c = pc_ptr[p] + 1; c < pc_ptr[p + 1]; ++c)
            if (pc_cell[c] == pc_cell[c - 1])
                EXM_CHECK((pc_info[c] & 63) == (pc_info[c - 1] & 63), EXM_EINVAL,
                          "internal: pattern entry %lld pairs different horizontal nodes within cell %d",
                          (long long)p, pc_cell[c]);
    // by rows, when no row has more than kRowEntries entries: the
    // contributions of a row's entries merged in cell order (within a cell,
    // in entry order)
    std::vector<int64_t> rc_ptr;
    std::vector<int32_t> rc_cell, rc_info;
    int32_t max_row = 0;
    for (int64_t r = 0; r < nclass; ++r) max_row = std::max(max_row, pptr[r + 1] - pptr[r]);
    if (max_row <= kRowEntries) {
        rc_ptr.assign(nclass + 1, 0);
        rc_cell.resize(ncon);
        rc_info.resize(ncon);
        std::vector<std::pair<int32_t, int32_t>> row;
        for (int64_t r = 0; r < nclass; ++r) {
            row.clear();
            for (int32_t p = pptr[r]; p < pptr[r + 1]; ++p)
                for (int64_t c = pc_ptr[p]; c < pc_ptr[p + 1]; ++c)
                    row.emplace_back(pc_cell[c], pc_info[c] | (p - pptr[r]) << 12);
            std::stable_sort(row.begin(), row.end(),
                             [](const std::pair<int32_t, int32_t>& a, const std::pair<int32_t, int32_t>& b) {
                                 return a.first < b.first;
                             });
            const int64_t at = rc_ptr[r];
            for (size_t i = 0; i < row.size(); ++i) {
                rc_cell[at + i] = row[i].first;
                rc_info[at + i] = row[i].second;
                // the row's vertex has one place in a cell
                EXM_CHECK(i == 0 || row[i].first != row[i - 1].first || (row[i].second & 7) == (row[i - 1].second & 7),
                          EXM_EINVAL, "internal: row %lld meets cell %d at two places", (long long)r, row[i].first);
            }
            rc_ptr[r + 1] = at + (int64_t)row.size();
        }
    }
    // structural entries (the CSR count)
    int64_t cnt[2][2][3] = {};
    for (int kr = 0; kr < 2; ++kr)
        for (int kq = 0; kq < 2; ++kq)
            for (int d = -1; d <= 1; ++d)
                for (int s = 0; s <= A->lam; ++s)
                    if ((kr == kKindH || s < A->lam) && (A->band == 3 || d == 0) && pair_valid(kr, kq, d, s, A->lam))
                        ++cnt[kr][kq][d + 1];
    int64_t nnz = 0;
    for (int64_t r = 0; r < nclass; ++r)
        for (int32_t p = pptr[r]; p < pptr[r + 1]; ++p)
            for (int d = 0; d < 3; ++d) nnz += cnt[wk[r] >> 16][wk[pcol[p]] >> 16][d];
    A->nnz = nnz;
    int32_t st;
    if ((st = A->c0.upload(c0.data(), c0.size())) != EXM_OK) return st;
    if ((st = A->wk.upload(wk.data(), wk.size())) != EXM_OK) return st;
    if ((st = A->pptr.upload(pptr.data(), pptr.size())) != EXM_OK) return st;
    if ((st = A->pcol.upload(pcol.data(), pcol.size())) != EXM_OK) return st;
    if ((st = A->pc_ptr.upload(pc_ptr.data(), pc_ptr.size())) != EXM_OK) return st;
    if ((st = A->pc_cell.upload(pc_cell.data(), pc_cell.size())) != EXM_OK) return st;
    if ((st = A->pc_info.upload(pc_info.data(), pc_info.size())) != EXM_OK) return st;
    if (!rc_ptr.empty()) {
        if ((st = A->rc_ptr.upload(rc_ptr.data(), rc_ptr.size())) != EXM_OK) return st;
        if ((st = A->rc_cell.upload(rc_cell.data(), rc_cell.size())) != EXM_OK) return st;
        if ((st = A->rc_info.upload(rc_info.data(), rc_info.size())) != EXM_OK) return st;
    }
    if ((st = A->val.alloc((size_t)A->n_pat * A->band * A->L)) != EXM_OK) return st;
    EXM_TRY_HIP(hipMemset(A->val.p, 0, sizeof(double) * A->val.n));
    *out = A.release();
    return EXM_OK;
}

int32_t exm_matrix_info(const exm_matrix* A, int64_t* n_rows, int64_t* nnz, int64_t* n_pattern, int64_t* n_stored)
{
    clear_error();
    EXM_CHECK(A != nullptr, EXM_EINVAL, "matrix is NULL");
    if (n_rows) *n_rows = A->space->n_dofs;
    if (nnz) *nnz = A->nnz;
    if (n_pattern) *n_pattern = A->n_pat;
    if (n_stored) *n_stored = A->n_pat * A->band * A->L;
    return EXM_OK;
}

int32_t exm_matrix_assemble(int32_t kernel, exm_matrix* A, int32_t nargs, const exm_arg* args, void* stream)
{
    clear_error();
    EXM_CHECK(A != nullptr && args != nullptr, EXM_EINVAL, "matrix or args is NULL");
    EXM_CHECK(kernel == EXM_K_MASS || kernel == EXM_K_CUBIC_JAC, EXM_EINVAL,
              "kernel %d has no matrix (EXM_K_MASS or EXM_K_CUBIC_JAC)", kernel);
    const bool jac = kernel == EXM_K_CUBIC_JAC;
    EXM_CHECK(nargs == (jac ? 2 : 1), EXM_EINVAL, "kernel %d takes %d args, got %d", kernel, jac ? 2 : 1, nargs);
    const exm_mesh* m = A->space->mesh;
    const exm_arg& X = args[0];
    EXM_CHECK(X.space != nullptr && X.data != nullptr, EXM_EINVAL, "args[0] (coordinates) has a NULL space or data");
    EXM_CHECK(X.space->mesh == m, EXM_EINVAL, "coordinate space is on another mesh");
    EXM_CHECK(X.space->element == EXM_ELEMENT_P1P1 && X.dim == 3 && X.access == EXM_READ, EXM_EINVAL,
              "coordinates must be an EXM_READ P1xP1 field of dim 3");
    if (jac) {
        EXM_CHECK(A->element == EXM_ELEMENT_P1P1, EXM_EUNSUPPORTED, "the cubic Jacobian is implemented for P1xP1");
        EXM_CHECK(args[1].data != nullptr && args[1].space == A->space && args[1].dim == 1 &&
                      args[1].access == EXM_READ,
                  EXM_EINVAL, "args[1] (u) must be an EXM_READ scalar field on the matrix's space");
    }
    if (A->n_pat == 0) return EXM_OK;
    int32_t vs = ensure_vertical(X.space, X.data, (hipStream_t)stream);
    if (vs != EXM_OK) return vs;
    GatherArgs g;
    std::memset(&g, 0, sizeof(g));
    g.lam = A->lam;
    g.L = A->L;
    g.band = A->band;
    g.n_pat = A->n_pat;
    g.pc_ptr = A->pc_ptr.p;
    g.pc_cell = A->pc_cell.p;
    g.pc_info = A->pc_info.p;
    g.xmap = X.space->d_map.p;
    g.X = (const double*)X.data;
    g.xn = X.space->n_dofs;
    g.fmap = A->space->d_map.p;
    g.u = jac ? (const double*)args[1].data : nullptr;
    g.val = A->val.p;
    const int bs = 256;   // four wavefronts, each one (pattern entry, 64 slots)
    const int64_t waves = A->n_pat * ((A->L + 63) / 64);
    EXM_CHECK(waves < INT32_MAX, EXM_EOVERFLOW, "grid too large");
    const int64_t nb = (waves + 3) / 4;
    hipStream_t hs = (hipStream_t)stream;
    const ElementKinds ek = element_kinds(A->element);
    if (jac && A->rc_ptr.p) {   // the Jacobian by rows
        g.n_rows = A->n_classes;
        g.pptr = A->pptr.p;
        g.rc_ptr = A->rc_ptr.p;
        g.rc_cell = A->rc_cell.p;
        g.rc_info = A->rc_info.p;
        const int64_t rwaves = (int64_t)A->n_classes * ((A->L + 63) / 64);
        EXM_CHECK(rwaves < INT32_MAX, EXM_EOVERFLOW, "grid too large");
        hipLaunchKernelGGL((k_mat_jac_rows<kRowEntries>), dim3((unsigned)((rwaves + 3) / 4)), dim3(bs), 0, hs, g);
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    if (!jac && A->rc_ptr.p) {   // the mass by rows
        g.n_rows = A->n_classes;
        g.pptr = A->pptr.p;
        g.rc_ptr = A->rc_ptr.p;
        g.rc_cell = A->rc_cell.p;
        g.rc_info = A->rc_info.p;
        const int64_t rwaves = (int64_t)A->n_classes * ((A->L + 63) / 64);
        EXM_CHECK(rwaves < INT32_MAX, EXM_EOVERFLOW, "grid too large");
        const dim3 grid((unsigned)((rwaves + 3) / 4));
#define EXM_ROWS(HK, VK) hipLaunchKernelGGL((k_mat_mass_rows<HK, VK, kRowEntries>), grid, dim3(bs), 0, hs, g)
        if (ek.hk == 0 && ek.vk == 0) EXM_ROWS(0, 0);
        else if (ek.hk == 0) EXM_ROWS(0, 1);
        else if (ek.hk == 1 && ek.vk == 0) EXM_ROWS(1, 0);
        else if (ek.hk == 1) EXM_ROWS(1, 1);
        else EXM_ROWS(2, 2);
#undef EXM_ROWS
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
#define EXM_GATHER(HK, VK, J) hipLaunchKernelGGL((k_mat_gather<HK, VK, J>), dim3((unsigned)nb), dim3(bs), 0, hs, g)
    if (jac) EXM_GATHER(0, 0, true);
    else if (ek.hk == 0 && ek.vk == 0) EXM_GATHER(0, 0, false);
    else if (ek.hk == 0) EXM_GATHER(0, 1, false);
    else if (ek.hk == 1 && ek.vk == 0) EXM_GATHER(1, 0, false);
    else if (ek.hk == 1) EXM_GATHER(1, 1, false);
    else EXM_GATHER(2, 2, false);
#undef EXM_GATHER
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

static RowArgs row_args(const exm_matrix* A)
{
    RowArgs a;
    std::memset(&a, 0, sizeof(a));
    a.lam = A->lam;
    a.L = A->L;
    a.band = A->band;
    a.n_classes = A->n_classes;
    a.n_items = (int64_t)A->n_classes * A->L;
    a.c0 = A->c0.p;
    a.wk = A->wk.p;
    a.pptr = A->pptr.p;
    a.pcol = A->pcol.p;
    a.val = A->val.p;
    return a;
}

int32_t exm_matrix_spmv(const exm_matrix* A, const double* x, double* y, int32_t access, void* stream)
{
    clear_error();
    EXM_CHECK(A != nullptr && x != nullptr && y != nullptr, EXM_EINVAL, "matrix, x or y is NULL");
    EXM_CHECK(x != y, EXM_EINVAL, "y aliases x");
    EXM_CHECK(access == EXM_WRITE || access == EXM_INC, EXM_EINVAL, "access must be EXM_WRITE or EXM_INC");
    RowArgs a = row_args(A);
    if (a.n_items == 0) return EXM_OK;
    a.write = access == EXM_WRITE;
    a.x = x;
    a.y = y;
    const int bs = 256;   // four wavefronts, each one (class, 64 slots)
    const int64_t waves = (int64_t)A->n_classes * ((A->L + 63) / 64);
    EXM_CHECK(waves < INT32_MAX, EXM_EOVERFLOW, "grid too large");
    const int64_t nb = (waves + 3) / 4;
    hipLaunchKernelGGL(k_mat_spmv, dim3((unsigned)nb), dim3(bs), 0, (hipStream_t)stream, a);
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t exm_matrix_csr(const exm_matrix* A, int64_t* rowptr, int32_t* col, double* val, void* stream)
{
    clear_error();
    EXM_CHECK(A != nullptr && rowptr != nullptr, EXM_EINVAL, "matrix or rowptr is NULL");
    EXM_CHECK(A->nnz == 0 || (col != nullptr && val != nullptr), EXM_EINVAL, "col or val is NULL");
    const int64_t n = A->space->n_dofs;
    hipStream_t hs = (hipStream_t)stream;
    RowArgs a = row_args(A);
    DevBuf<int64_t> cnt;
    int32_t st;
    if ((st = cnt.alloc((size_t)n + 1)) != EXM_OK) return st;
    EXM_TRY_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int64_t) * (size_t)(n + 1), hs));
    a.cnt = cnt.p;
    const int bs = 256;
    const int64_t nb = (a.n_items + bs - 1) / bs;
    if (a.n_items) hipLaunchKernelGGL(k_csr_count, dim3((unsigned)nb), dim3(bs), 0, hs, a);
    EXM_TRY_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    EXM_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt.p, rowptr, (int)(n + 1), hs));
    DevBuf<unsigned char> tmp;
    if ((st = tmp.alloc(tmp_bytes)) != EXM_OK) return st;
    EXM_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, cnt.p, rowptr, (int)(n + 1), hs));
    a.rowptr = rowptr;
    a.ccol = col;
    a.cval = val;
    if (a.n_items) hipLaunchKernelGGL(k_csr_fill, dim3((unsigned)nb), dim3(bs), 0, hs, a);
    EXM_TRY_HIP(hipGetLastError());
    // cnt and tmp are freed on return: wait for the kernels that use them
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    return EXM_OK;
}

// Device address of `scratch` on the current device, looked up once per device.
static int32_t scratch_address(int64_t** out)
{
    static std::mutex mu;
    static std::vector<int64_t*> addr;
    int dev = 0;
    EXM_TRY_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        EXM_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        addr[dev] = (int64_t*)p;
    }
    *out = addr[dev];
    return EXM_OK;
}

int32_t exm_matrix_csr_noalloc(const exm_matrix* A, int64_t* rowptr, int32_t* col, double* val, void* stream)
{
    clear_error();
    EXM_CHECK(A != nullptr && rowptr != nullptr, EXM_EINVAL, "matrix or rowptr is NULL");
    EXM_CHECK(A->nnz == 0 || (col != nullptr && val != nullptr), EXM_EINVAL, "col or val is NULL");
    const int64_t n = A->space->n_dofs;
    const int64_t nseg = (n + kScanSeg - 1) / kScanSeg;
    EXM_CHECK(nseg <= kScanMaxSegs, EXM_ERANGE, "%lld rows exceed the %lld this call can scan without allocating",
              (long long)n, (long long)(kScanMaxSegs * kScanSeg));
    int64_t* seg = nullptr;
    int32_t st = scratch_address(&seg);
    if (st != EXM_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    RowArgs a = row_args(A);
    const int bs = 256;
    const int64_t nb = std::max<int64_t>(1, (a.n_items + bs - 1) / bs);
    hipLaunchKernelGGL(k_csr_count_rowptr, dim3((unsigned)nb), dim3(bs), 0, hs, a, rowptr);
    EXM_TRY_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_scan_segments, dim3((unsigned)nseg), dim3(kScanThreads), 0, hs, rowptr + 1, n, seg);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, hs, seg, nseg);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nseg), dim3(kScanThreads), 0, hs, rowptr + 1, n, seg);
        EXM_TRY_HIP(hipGetLastError());
    }
    a.rowptr = rowptr;
    a.ccol = col;
    a.cval = val;
    if (a.n_items) hipLaunchKernelGGL(k_csr_fill, dim3((unsigned)nb), dim3(bs), 0, hs, a);
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

void exm_matrix_destroy(exm_matrix* A) { delete A; }

}  // extern "C"
