// GATHER schedule of the mass action on the spaces whose DoFs sit on vertex
// columns (P1 x P1, CG1 x DG0, CG1 x DG1): the column loop turned around to
// iterate the vertex columns of the output (owner computes).  Variants: two
// levels per lane for long P1 columns, one lane per layer for the spaces
// discontinuous across levels, and columns of different heights.
//
// P1 x P1:
// A wavefront owns one base vertex v and 62 consecutive levels of its column
// (lanes hold levels l0 - 1 .. l0 + 62; the two end lanes are halo).  It walks
// the fan of base cells around v in cyclic order, so that every neighbouring
// vertex column is loaded once for the two cells that share it, and sums the
// row of v of every prism around its levels: lane l evaluates prism (c, l)
// for node v at the bottom and at the top, keeps the bottom row and passes
// the top row one lane up (it is level l + 1's share).  Every output DoF is
// written once by its owner: no atomics, no colours, no LDS and no barriers;
// the neighbouring columns come from L2, since the fans of consecutive
// vertices (in the RCM order) overlap.
#include <algorithm>
#include <cstring>

#include "exm_elements.hpp"
#include "exm_internal.hpp"
#include "exm_tiled.hpp"

namespace exm {
namespace {

constexpr int kOwned = 62;   // levels written per wavefront step (64 lanes, one halo lane each side)

__device__ __forceinline__ unsigned xcd_block_g(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

struct GatherP1Args {
    int32_t n_vertices, lam, n_steps, write;
    int64_t fbase, xbase;          // column start of vertex w: base + w * (lam + 1)
    const int32_t* __restrict__ fan_off;   // [n_vertices + 1]
    const int32_t* __restrict__ fan;       // neighbour ids; bit 31: the entry starts a fan (no cell with the previous)
    const double* __restrict__ X;          // coordinates, component-major
    int64_t xn;
    const double* __restrict__ f;
    double* __restrict__ y;
    // columns of different heights
    const int32_t* __restrict__ fstart;    // column start of every vertex in the field space
    const int32_t* __restrict__ xstart;    // ... in the coordinate space
    const int32_t* __restrict__ vlo;       // level range lo .. hi of every vertex column
    const int32_t* __restrict__ vhi;
    const int32_t* __restrict__ cell_lo;   // layers cell_lo .. cell_lo + cell_lam - 1 of every cell
    const int32_t* __restrict__ cell_lam;
    const int32_t* __restrict__ fan_cell;  // the cell of every fan entry (-1 at the start of a fan)
};

__global__ void __launch_bounds__(256) k_gather_p1(const GatherP1Args g)
{
    const int lane = threadIdx.x & 63;
    // the wavefront's work item, made visibly uniform so that its indices live in scalar registers
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_g(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t v = wid / g.n_steps;
    if (v >= g.n_vertices) return;   // uniform over the wavefront
    const int l0 = (int)(wid - v * g.n_steps) * kOwned;
    const int lev = l0 - 1 + lane;
    const bool in = lev >= 0 && lev <= g.lam;   // a level of the column
    const bool prism = lev >= 0 && lev < g.lam; // the prism above this level exists
    const int64_t lamp = (int64_t)g.lam + 1;
    const double* __restrict__ Z = g.X + 2 * g.xn;
    // own column: f and z at this level and the next (the next lane's)
    const int64_t fv = g.fbase + v * lamp, xv = g.xbase + v * lamp;
    const double f0 = in ? g.f[fv + lev] : 0.0;
    const double z0 = in ? Z[xv + lev] : 0.0;
    const double f0n = __shfl_down(f0, 1, 64), z0n = __shfl_down(z0, 1, 64);
    const double px0 = g.X[xv], py0 = g.X[g.xn + xv];
    double acc_b = 0.0, acc_t = 0.0;
    double fp = 0.0, fpn = 0.0, zp = 0.0, zpn = 0.0, pxp = 0.0, pyp = 0.0;   // previous neighbour
    const int32_t e0 = g.fan_off[v], e1 = g.fan_off[v + 1];
    // blocks of kBlk fan entries: every load of a block is issued before the
    // first of its cells is evaluated, so the wavefront waits once per block
    constexpr int kBlk = 4;
    for (int32_t e = e0; e < e1; e += kBlk) {
        int32_t ent[kBlk];
        double f1[kBlk], z1[kBlk], px1[kBlk], py1[kBlk];
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            const bool has = e + k < e1;   // uniform over the wavefront
            ent[k] = has ? g.fan[e + k] : 0;
            const int64_t w = ent[k] & 0x7fffffff;
            const int64_t fw = g.fbase + w * lamp, xw = g.xbase + w * lamp;
            f1[k] = has && in ? g.f[fw + lev] : 0.0;
            z1[k] = has && in ? Z[xw + lev] : 0.0;
            px1[k] = has ? g.X[xw] : 0.0;
            py1[k] = has ? g.X[g.xn + xw] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            if (e + k >= e1) break;
            const double f1n = __shfl_down(f1[k], 1, 64), z1n = __shfl_down(z1[k], 1, 64);
            if (ent[k] >= 0 && prism) {   // cell (v, previous, w)
                const double twoA = fabs((pxp - px0) * (py1[k] - py0) - (px1[k] - px0) * (pyp - py0));
                const double h[3] = {z0n - z0, zpn - zp, z1n - z1[k]};
                const double xb[3] = {f0, fp, f1[k]};
                const double xt[3] = {f0n, fpn, f1n};
                double yb, yt;
                p1_row(twoA * (1.0 / 120.0), h, xb, xt, yb, yt);
                acc_b += yb;
                acc_t += yt;
            }
            fp = f1[k];
            fpn = f1n;
            zp = z1[k];
            zpn = z1n;
            pxp = px1[k];
            pyp = py1[k];
        }
    }
    // level lev takes the bottom rows of the prisms above it and the top rows
    // of the prisms below it (computed by the lane below)
    const double below = __shfl_up(acc_t, 1, 64);
    if (lane >= 1 && lane <= kOwned && in) {
        const double val = acc_b + below;
        if (g.write)
            g.y[fv + lev] = val;
        else
            g.y[fv + lev] += val;
    }
}

// Two levels per lane: lanes hold levels b = l0 - 1 + 2 i and b + 1, so a
// wavefront covers 126 owned levels (the first level of lane 0 and the second
// of lane 63 are halo) and a 101-level column needs one wavefront instead of
// two.  A lane evaluates prisms (c, b) and (c, b + 1) for node v; level b
// takes the bottom row of prism b and the top row of prism b - 1 (the lane
// below), level b + 1 the bottom row of prism b + 1 and the top row of
// prism b.
constexpr int kOwned2 = 126;

__global__ void __launch_bounds__(256) k_gather_p1x2(const GatherP1Args g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_g(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t v = wid / g.n_steps;
    if (v >= g.n_vertices) return;   // uniform over the wavefront
    const int l0 = (int)(wid - v * g.n_steps) * kOwned2;
    const int b = l0 - 1 + 2 * lane;
    const bool in0 = b >= 0 && b <= g.lam, in1 = b + 1 >= 0 && b + 1 <= g.lam;
    const bool pr0 = b >= 0 && b < g.lam, pr1 = b + 1 >= 0 && b + 1 < g.lam;   // prisms above b and b + 1
    const int64_t lamp = (int64_t)g.lam + 1;
    const double* __restrict__ Z = g.X + 2 * g.xn;
    const int64_t fv = g.fbase + v * lamp, xv = g.xbase + v * lamp;
    // own column at levels b, b + 1 and (from the next lane) b + 2
    const double f0a = in0 ? g.f[fv + b] : 0.0, f0b = in1 ? g.f[fv + b + 1] : 0.0;
    const double z0a = in0 ? Z[xv + b] : 0.0, z0b = in1 ? Z[xv + b + 1] : 0.0;
    const double f0c = __shfl_down(f0a, 1, 64), z0c = __shfl_down(z0a, 1, 64);
    const double px0 = g.X[xv], py0 = g.X[g.xn + xv];
    double yb0 = 0.0, yt0 = 0.0, yb1 = 0.0, yt1 = 0.0;
    double fpa = 0.0, fpb = 0.0, fpc = 0.0, zpa = 0.0, zpb = 0.0, zpc = 0.0, pxp = 0.0, pyp = 0.0;
    const int32_t e0 = g.fan_off[v], e1 = g.fan_off[v + 1];
    constexpr int kBlk = 4;
    for (int32_t e = e0; e < e1; e += kBlk) {
        int32_t ent[kBlk];
        double fa[kBlk], fb[kBlk], za[kBlk], zb[kBlk], px1[kBlk], py1[kBlk];
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            const bool has = e + k < e1;   // uniform over the wavefront
            ent[k] = has ? g.fan[e + k] : 0;
            const int64_t w = ent[k] & 0x7fffffff;
            const int64_t fw = g.fbase + w * lamp, xw = g.xbase + w * lamp;
            fa[k] = has && in0 ? g.f[fw + b] : 0.0;
            fb[k] = has && in1 ? g.f[fw + b + 1] : 0.0;
            za[k] = has && in0 ? Z[xw + b] : 0.0;
            zb[k] = has && in1 ? Z[xw + b + 1] : 0.0;
            px1[k] = has ? g.X[xw] : 0.0;
            py1[k] = has ? g.X[g.xn + xw] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            if (e + k >= e1) break;
            const double fc = __shfl_down(fa[k], 1, 64), zc = __shfl_down(za[k], 1, 64);
            if (ent[k] >= 0) {   // cell (v, previous, w)
                const double twoA = fabs((pxp - px0) * (py1[k] - py0) - (px1[k] - px0) * (pyp - py0));
                const double s = twoA * (1.0 / 120.0);
                if (pr0) {
                    const double h[3] = {z0b - z0a, zpb - zpa, zb[k] - za[k]};
                    const double xb[3] = {f0a, fpa, fa[k]};
                    const double xt[3] = {f0b, fpb, fb[k]};
                    double r0, r1;
                    p1_row(s, h, xb, xt, r0, r1);
                    yb0 += r0;
                    yt0 += r1;
                }
                if (pr1) {
                    const double h[3] = {z0c - z0b, zpc - zpb, zc - zb[k]};
                    const double xb[3] = {f0b, fpb, fb[k]};
                    const double xt[3] = {f0c, fpc, fc};
                    double r0, r1;
                    p1_row(s, h, xb, xt, r0, r1);
                    yb1 += r0;
                    yt1 += r1;
                }
            }
            fpa = fa[k];
            fpb = fb[k];
            fpc = fc;
            zpa = za[k];
            zpb = zb[k];
            zpc = zc;
            pxp = px1[k];
            pyp = py1[k];
        }
    }
    const double below = __shfl_up(yt1, 1, 64);   // top row of prism b - 1
    const auto put = [&](int lev, double val) {
        if (g.write)
            g.y[fv + lev] = val;
        else
            g.y[fv + lev] += val;
    };
    if (lane >= 1 && in0) put(b, yb0 + below);
    if (lane <= 62 && in1) put(b + 1, yb1 + yt0);
}

// The same owner-computes walk for the spaces whose vertex columns are
// discontinuous across levels: CG1 x DG0 (NV = 1, one DoF per layer) and
// CG1 x DG1 (NV = 2, bottom and top node per layer).  There is no vertical
// coupling, so a lane owns one layer (no halo lanes): it reads z at both
// levels of its layer and the field at its layer for v and the fan, and
// writes the row of v of every prism of that layer around v:
//   y_(v, b) = (2A / 120) ((2 h_v + H) g_v + (h_v + H) G + sum_a h_a g_a),
// g = V x per vertex (V the vertical mass of the layer's nodes).
template <int NV>
__global__ void __launch_bounds__(256) k_gather_p1dg(const GatherP1Args g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_g(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t v = wid / g.n_steps;
    if (v >= g.n_vertices) return;   // uniform over the wavefront
    const int l = (int)(wid - v * g.n_steps) * 64 + lane;
    const bool act = l < g.lam;
    const int64_t col = (int64_t)NV * g.lam;          // DoFs of a vertex column
    const int64_t lamp = (int64_t)g.lam + 1;          // levels of a coordinate column
    const double* __restrict__ Z = g.X + 2 * g.xn;
    const int64_t fv = g.fbase + v * col, xv = g.xbase + v * lamp;
    double x0[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) x0[b] = act ? g.f[fv + NV * l + b] : 0.0;
    const double z0 = act ? Z[xv + l] : 0.0, z0n = act ? Z[xv + l + 1] : 0.0;
    const double px0 = g.X[xv], py0 = g.X[g.xn + xv];
    double acc[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) acc[b] = 0.0;
    double xp[NV], zp = 0.0, zpn = 0.0, pxp = 0.0, pyp = 0.0;   // previous neighbour
#pragma unroll
    for (int b = 0; b < NV; ++b) xp[b] = 0.0;
    const int32_t e0 = g.fan_off[v], e1 = g.fan_off[v + 1];
    constexpr int kBlk = 4;
    for (int32_t e = e0; e < e1; e += kBlk) {
        int32_t ent[kBlk];
        double x1[kBlk][NV], z1[kBlk], z1n[kBlk], px1[kBlk], py1[kBlk];
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            const bool has = e + k < e1;   // uniform over the wavefront
            ent[k] = has ? g.fan[e + k] : 0;
            const int64_t w = ent[k] & 0x7fffffff;
            const int64_t fw = g.fbase + w * col, xw = g.xbase + w * lamp;
#pragma unroll
            for (int b = 0; b < NV; ++b) x1[k][b] = has && act ? g.f[fw + NV * l + b] : 0.0;
            z1[k] = has && act ? Z[xw + l] : 0.0;
            z1n[k] = has && act ? Z[xw + l + 1] : 0.0;
            px1[k] = has ? g.X[xw] : 0.0;
            py1[k] = has ? g.X[g.xn + xw] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kBlk; ++k) {
            if (e + k >= e1) break;
            if (ent[k] >= 0 && act) {   // cell (v, previous, w)
                const double twoA = fabs((pxp - px0) * (py1[k] - py0) - (px1[k] - px0) * (pyp - py0));
                const double h[3] = {z0n - z0, zpn - zp, z1n[k] - z1[k]};
                const double H = h[0] + h[1] + h[2];
                const double s = twoA * (1.0 / 120.0);
#pragma unroll
                for (int b = 0; b < NV; ++b) {
                    // vertical mass of the layer's nodes, then the horizontal row of v
                    double gv, gp, gw;
                    if constexpr (NV == 1) {
                        gv = x0[0];
                        gp = xp[0];
                        gw = x1[k][0];
                    } else {
                        const double cs = b == 0 ? 1.0 / 3.0 : 1.0 / 6.0, ct = b == 0 ? 1.0 / 6.0 : 1.0 / 3.0;
                        gv = cs * x0[0] + ct * x0[1];
                        gp = cs * xp[0] + ct * xp[1];
                        gw = cs * x1[k][0] + ct * x1[k][1];
                    }
                    const double G = gv + gp + gw;
                    const double HG = h[0] * gv + h[1] * gp + h[2] * gw;
                    acc[b] += s * ((2.0 * h[0] + H) * gv + (h[0] + H) * G + HG);
                }
            }
#pragma unroll
            for (int b = 0; b < NV; ++b) xp[b] = x1[k][b];
            zp = z1[k];
            zpn = z1n[k];
            pxp = px1[k];
            pyp = py1[k];
        }
    }
    if (!act) return;
#pragma unroll
    for (int b = 0; b < NV; ++b) {
        if (g.write)
            g.y[fv + NV * l + b] = acc[b];
        else
            g.y[fv + NV * l + b] += acc[b];
    }
}

// GATHER on a mesh whose columns differ in height (P1 x P1).  The wavefront
// walks its vertex column from the column's own bottom level; a neighbour's
// values come from its own column at the same absolute level, and the
// prisms of a cell of the fan count only within the cell's layer range (the
// columns of its three vertices span that range, so the levels it needs are
// present).
__global__ void __launch_bounds__(256) k_gather_p1_var(const GatherP1Args g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_g(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t v = wid / g.n_steps;
    if (v >= g.n_vertices) return;   // uniform over the wavefront
    const int lo_v = g.vlo[v], nlev = g.vhi[v] - lo_v + 1;
    const int q0 = (int)(wid - v * g.n_steps) * kOwned;
    if (q0 >= nlev) return;          // beyond this column (uniform)
    const int q = q0 - 1 + lane;     // level of the column, from its bottom
    const int lev = lo_v + q;        // absolute level
    const bool in = q >= 0 && q < nlev;
    const double* __restrict__ Z = g.X + 2 * g.xn;
    const int64_t fv = g.fstart[v], xv = g.xstart[v];
    const double f0 = in ? g.f[fv + q] : 0.0;
    const double z0 = in ? Z[xv + q] : 0.0;
    const double f0n = __shfl_down(f0, 1, 64), z0n = __shfl_down(z0, 1, 64);
    const double px0 = g.X[xv], py0 = g.X[g.xn + xv];
    double acc_b = 0.0, acc_t = 0.0;
    double fp = 0.0, fpn = 0.0, zp = 0.0, zpn = 0.0, pxp = 0.0, pyp = 0.0;
    const int32_t e0 = g.fan_off[v], e1 = g.fan_off[v + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t ent = g.fan[e];
        const int32_t w = ent & 0x7fffffff;
        const int32_t c = g.fan_cell[e];
        const int lo_w = g.vlo[w], hi_w = g.vhi[w];
        const int64_t fw = g.fstart[w], xw = g.xstart[w];
        const bool inw = in && lev >= lo_w && lev <= hi_w;
        const double f1 = inw ? g.f[fw + (lev - lo_w)] : 0.0;
        const double z1 = inw ? Z[xw + (lev - lo_w)] : 0.0;
        const double f1n = __shfl_down(f1, 1, 64), z1n = __shfl_down(z1, 1, 64);
        const double px1 = g.X[xw], py1 = g.X[g.xn + xw];
        if (c >= 0) {
            const int cb = g.cell_lo[c], ct = cb + g.cell_lam[c];
            if (in && lev >= cb && lev < ct) {   // prism (c, lev) of cell (v, previous, w)
                const double twoA = fabs((pxp - px0) * (py1 - py0) - (px1 - px0) * (pyp - py0));
                const double h[3] = {z0n - z0, zpn - zp, z1n - z1};
                const double xb[3] = {f0, fp, f1};
                const double xt[3] = {f0n, fpn, f1n};
                double yb, yt;
                p1_row(twoA * (1.0 / 120.0), h, xb, xt, yb, yt);
                acc_b += yb;
                acc_t += yt;
            }
        }
        fp = f1;
        fpn = f1n;
        zp = z1;
        zpn = z1n;
        pxp = px1;
        pyp = py1;
    }
    const double below = __shfl_up(acc_t, 1, 64);
    if (lane >= 1 && lane <= kOwned && in) {
        const double val = acc_b + below;
        if (g.write)
            g.y[fv + q] = val;
        else
            g.y[fv + q] += val;
    }
}

// GATHER on a mesh whose columns differ in height, CG1 x DG0 (NV = 1) and
// CG1 x DG1 (NV = 2): one lane per layer of the vertex column.
template <int NV>
__global__ void __launch_bounds__(256) k_gather_p1dg_var(const GatherP1Args g)
{
    const int lane = threadIdx.x & 63;
    const int64_t wid = __builtin_amdgcn_readfirstlane(
        (int32_t)(xcd_block_g(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int64_t v = wid / g.n_steps;
    if (v >= g.n_vertices) return;   // uniform over the wavefront
    const int lo_v = g.vlo[v], nl = g.vhi[v] - lo_v;
    const int q0 = (int)(wid - v * g.n_steps) * 64;
    if (q0 >= nl) return;            // beyond this column (uniform)
    const int q = q0 + lane;         // layer of the column, from its bottom
    const int lev = lo_v + q;
    const bool act = q < nl;
    const double* __restrict__ Z = g.X + 2 * g.xn;
    const int64_t fv = g.fstart[v], xv = g.xstart[v];
    double x0[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) x0[b] = act ? g.f[fv + NV * q + b] : 0.0;
    const double z0 = act ? Z[xv + q] : 0.0, z0n = act ? Z[xv + q + 1] : 0.0;
    const double px0 = g.X[xv], py0 = g.X[g.xn + xv];
    double acc[NV], xp[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) acc[b] = xp[b] = 0.0;
    double zp = 0.0, zpn = 0.0, pxp = 0.0, pyp = 0.0;
    const int32_t e0 = g.fan_off[v], e1 = g.fan_off[v + 1];
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t w = g.fan[e] & 0x7fffffff;
        const int32_t c = g.fan_cell[e];
        const int lo_w = g.vlo[w], hi_w = g.vhi[w];
        const int64_t fw = g.fstart[w], xw = g.xstart[w];
        const bool inw = act && lev >= lo_w && lev < hi_w;
        double x1[NV];
#pragma unroll
        for (int b = 0; b < NV; ++b) x1[b] = inw ? g.f[fw + NV * (lev - lo_w) + b] : 0.0;
        const double z1 = inw ? Z[xw + (lev - lo_w)] : 0.0, z1n = inw ? Z[xw + (lev - lo_w) + 1] : 0.0;
        const double px1 = g.X[xw], py1 = g.X[g.xn + xw];
        if (c >= 0) {
            const int cb = g.cell_lo[c], ct = cb + g.cell_lam[c];
            if (act && lev >= cb && lev < ct) {
                const double twoA = fabs((pxp - px0) * (py1 - py0) - (px1 - px0) * (pyp - py0));
                const double h[3] = {z0n - z0, zpn - zp, z1n - z1};
                const double H = h[0] + h[1] + h[2];
                const double s = twoA * (1.0 / 120.0);
#pragma unroll
                for (int b = 0; b < NV; ++b) {
                    double gv, gp, gw;
                    if constexpr (NV == 1) {
                        gv = x0[0];
                        gp = xp[0];
                        gw = x1[0];
                    } else {
                        const double cs = b == 0 ? 1.0 / 3.0 : 1.0 / 6.0, ct2 = b == 0 ? 1.0 / 6.0 : 1.0 / 3.0;
                        gv = cs * x0[0] + ct2 * x0[1];
                        gp = cs * xp[0] + ct2 * xp[1];
                        gw = cs * x1[0] + ct2 * x1[1];
                    }
                    const double G = gv + gp + gw;
                    const double HG = h[0] * gv + h[1] * gp + h[2] * gw;
                    acc[b] += s * ((2.0 * h[0] + H) * gv + (h[0] + H) * G + HG);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NV; ++b) xp[b] = x1[b];
        zp = z1;
        zpn = z1n;
        pxp = px1;
        pyp = py1;
    }
    if (!act) return;
#pragma unroll
    for (int b = 0; b < NV; ++b) {
        if (g.write)
            g.y[fv + NV * q + b] = acc[b];
        else
            g.y[fv + NV * q + b] += acc[b];
    }
}

}  // namespace

// Fans of base cells around every vertex, in cyclic order: for vertex v the
// list n_0, n_1, ..., n_k of neighbouring vertices such that (v, n_i, n_i+1)
// is a cell; a fan starts at a spoke with one cell (the boundary) where there
// is one, and an interior fan repeats its first neighbour at the end.  A
// vertex whose cells do not form one fan gets several, each entry that
// starts a fan flagged with bit 31.
int32_t build_vertex_fans(const exm_mesh* m, const VertexFans** out)
{
    std::lock_guard<std::mutex> lock(m->mu);
    if (m->fans) {
        *out = m->fans.get();
        return EXM_OK;
    }
    const int32_t nv = m->n[0], nc = m->n[2];
    const int32_t* cv = m->h_cell_vertex.data();
    std::vector<int64_t> vstart(nv + 1, 0);
    for (int64_t i = 0; i < (int64_t)nc * 3; ++i) vstart[cv[i] + 1]++;
    for (int32_t v = 0; v < nv; ++v) vstart[v + 1] += vstart[v];
    std::vector<int32_t> vcells(vstart[nv]);
    {
        std::vector<int64_t> fill(vstart.begin(), vstart.end() - 1);
        for (int32_t c = 0; c < nc; ++c)
            for (int a = 0; a < 3; ++a) vcells[fill[cv[c * 3 + a]]++] = c;
    }
    std::vector<int32_t> off(nv + 1, 0), fan, fcell;
    fan.reserve((size_t)nc * 4);
    fcell.reserve((size_t)nc * 4);
    std::vector<int32_t> na, nb;   // the two other vertices of every cell of the star
    std::vector<char> used;
    for (int32_t v = 0; v < nv; ++v) {
        const int64_t b = vstart[v], n = vstart[v + 1] - b;
        na.assign(n, 0);
        nb.assign(n, 0);
        used.assign(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            const int32_t c = vcells[b + i];
            int k = 0;
            int32_t o[2] = {0, 0};
            for (int a = 0; a < 3; ++a)
                if (cv[c * 3 + a] != v && k < 2) o[k++] = cv[c * 3 + a];
            na[i] = o[0];
            nb[i] = o[1];
        }
        auto spokes = [&](int32_t w) {   // cells of the star that contain w
            int cnt = 0;
            for (int64_t i = 0; i < n; ++i) cnt += (na[i] == w) + (nb[i] == w);
            return cnt;
        };
        int64_t left = n;
        while (left > 0) {
            // start at a boundary spoke if an unused cell has one
            int64_t s = -1;
            int32_t entry = 0;
            for (int64_t i = 0; i < n && s < 0; ++i) {
                if (used[i]) continue;
                if (spokes(na[i]) == 1) { s = i; entry = na[i]; }
                else if (spokes(nb[i]) == 1) { s = i; entry = nb[i]; }
            }
            if (s < 0) {
                for (int64_t i = 0; i < n && s < 0; ++i)
                    if (!used[i]) { s = i; entry = na[i]; }
            }
            fan.push_back(entry | (int32_t)0x80000000);
            fcell.push_back(-1);
            int64_t cur = s;
            int32_t from = entry;
            while (cur >= 0) {
                used[cur] = 1;
                --left;
                const int32_t exit = na[cur] == from ? nb[cur] : na[cur];
                fan.push_back(exit);
                fcell.push_back(vcells[b + cur]);
                int64_t next = -1;
                for (int64_t i = 0; i < n && next < 0; ++i)
                    if (!used[i] && (na[i] == exit || nb[i] == exit)) next = i;
                cur = next;
                from = exit;
            }
        }
        off[v + 1] = (int32_t)fan.size();
    }
    auto F = std::make_unique<VertexFans>();
    int32_t st;
    if ((st = F->off.upload(off.data(), off.size())) != EXM_OK) return st;
    if ((st = F->fan.upload(fan.data(), fan.size())) != EXM_OK) return st;
    if ((st = F->cell.upload(fcell.data(), fcell.size())) != EXM_OK) return st;
    F->n_entries = (int64_t)fan.size();
    m->fans = std::move(F);
    *out = m->fans.get();
    return EXM_OK;
}

bool gather_supported(int32_t kernel, int32_t element)
{
    return kernel == EXM_K_MASS &&
           (element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_P1DG0 || element == EXM_ELEMENT_P1DG1);
}

int32_t launch_gather(const LoopLaunch& P, const VertexFans* fans, int32_t wpb, hipStream_t s)
{
    GatherP1Args g;
    std::memset(&g, 0, sizeof(g));
    g.n_vertices = P.fspace->mesh->n[0];
    g.lam = P.n_layers;
    const bool levels = P.element == EXM_ELEMENT_P1P1;   // DoFs on the levels, else inside the layers
    const bool two = levels && P.n_layers + 1 > kOwned;   // columns longer than one 62-level step
    g.n_steps = levels ? (two ? (P.n_layers + 1 + kOwned2 - 1) / kOwned2 : (P.n_layers + 1 + kOwned - 1) / kOwned)
                       : (P.n_layers + 63) / 64;
    g.write = P.write;
    g.fbase = P.fspace->base[0];
    g.xbase = P.xspace->base[0];
    g.fan_off = fans->off.p;
    g.fan = fans->fan.p;
    g.X = P.X;
    g.xn = P.xspace->n_dofs;
    g.f = P.in[0];
    g.y = P.out[0];
    if (g.n_vertices == 0) return EXM_OK;
    const exm_mesh* m = P.fspace->mesh;
    if (m->variable) {   // columns of different heights: starts and ranges from the mesh and the spaces
        g.fstart = P.fspace->d_starts[0].p;
        g.xstart = P.xspace->d_starts[0].p;
        g.vlo = m->d_vert_lo.p;
        g.vhi = m->d_vert_hi.p;
        g.cell_lo = m->d_cell_lo.p;
        g.cell_lam = m->d_cell_lam.p;
        g.fan_cell = fans->cell.p;
        g.n_steps = levels ? (P.n_layers + 1 + kOwned - 1) / kOwned : (P.n_layers + 63) / 64;
        const int64_t waves = (int64_t)g.n_vertices * g.n_steps;
        const int64_t blocks = (waves + wpb - 1) / wpb;
        if (blocks * wpb > INT32_MAX) return fail(EXM_ERANGE, "grid too large");
        if (levels)
            hipLaunchKernelGGL(k_gather_p1_var, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
        else if (P.element == EXM_ELEMENT_P1DG0)
            hipLaunchKernelGGL(k_gather_p1dg_var<1>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
        else
            hipLaunchKernelGGL(k_gather_p1dg_var<2>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    const int64_t waves = (int64_t)g.n_vertices * g.n_steps;
    const int64_t blocks = (waves + wpb - 1) / wpb;
    if (blocks * wpb > INT32_MAX) return fail(EXM_ERANGE, "grid too large");
    if (levels && two)
        hipLaunchKernelGGL(k_gather_p1x2, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
    else if (levels)
        hipLaunchKernelGGL(k_gather_p1, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
    else if (P.element == EXM_ELEMENT_P1DG0)
        hipLaunchKernelGGL(k_gather_p1dg<1>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
    else
        hipLaunchKernelGGL(k_gather_p1dg<2>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s, g);
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

}  // namespace exm
