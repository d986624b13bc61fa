// The extruded parallel loop (Algorithm 3 of arXiv 1604.05937) for gfx950.
//
// Work decomposition ("vertical lanes").  The vertical-innermost numbering
// makes the DoFs of one entity column contiguous, so a 64-lane wavefront
// takes cols_per_wave base cells side by side and gives each 64 / cols_per_wave
// consecutive lanes, one layer per lane.  A lane reads its cell's explicit
// lists once, then the wavefront walks the column in steps of `seg` layers:
// the DoF of stencil position p at layer l is L(c)[p] + l * offset[p], and the
// `seg` lanes of one cell read `seg` consecutive DoFs of every column, so each
// gather and scatter is a coalesced run instead of one cache line per lane.
//
// DoFs on horizontal levels are shared by the layers below and above (CG in
// the vertical).  A lane adds its top-level contribution to the next lane's
// bottom-level one through a cross-lane shuffle (the first lane of a step
// takes it from a carry left by the previous step), so every level of every
// column receives exactly one update per base cell.
//
// Horizontal sharing (CG in the horizontal) is resolved either by hardware
// FP64 atomic adds or by launching one colour of base cells at a time.
#include <algorithm>

#include "exm_elements.hpp"
#include "exm_internal.hpp"

namespace exm {

struct ColArgs {
    int32_t n_layers;
    int32_t off;           // vertical offset of the field space (same for every position)
    int32_t cpw, seg;
    const int32_t* __restrict__ fmap;
    const int32_t* __restrict__ xmap;
    const double* __restrict__ X;
    const double* __restrict__ in0;
    const double* __restrict__ in1;
    const double* __restrict__ in2;
    double* __restrict__ out0;
    double* __restrict__ out1;
    double* __restrict__ out2;
    const int32_t* __restrict__ cells;
    int64_t cell_begin, cell_count;
};

// Workgroups are dispatched to the eight XCDs round-robin; renumber them so
// that every XCD (and its L2) works through one contiguous range of cells.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

struct LaneInfo {
    int lane, sub, lsub;
    bool valid;
    int32_t cell;
};

template <bool LIST>
__device__ __forceinline__ bool lane_info(const ColArgs& a, LaneInfo& L)
{
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    L.lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave * a.cpw >= a.cell_count) return false;   // uniform over the wavefront
    L.sub = L.lane / a.seg;
    L.lsub = L.lane - L.sub * a.seg;
    const int64_t slot = wave * a.cpw + L.sub;
    L.valid = L.sub < a.cpw && slot < a.cell_count;
    L.cell = 0;
    if (L.valid) L.cell = LIST ? a.cells[a.cell_begin + slot] : (int32_t)(a.cell_begin + slot);
    return true;
}

// Value of a vertically shared level for the lane's layer l: the lane's own
// bottom contribution plus the top contribution of layer l - 1.
__device__ __forceinline__ double level_value(double bot, double top, double& carry, const LaneInfo& L, int seg)
{
    const double below = __shfl(top, (L.lane + 63) & 63, 64);
    const double last = __shfl(top, min(L.sub * seg + seg - 1, 63), 64);
    const double v = bot + (L.lsub == 0 ? carry : below);
    carry = last;
    return v;
}

template <int RACE>
__device__ __forceinline__ void inc(double* p, double v)
{
    if constexpr (RACE == EXM_RACE_ATOMIC)
        unsafeAtomicAdd(p, v);
    else
        *p += v;
}

// Coordinates of the prism's base triangle and its column heights at layer l.
// xb[a], xt[a]: bottom and top DoFs of base vertex a in the coordinate space
// (offset 1 per layer).
__device__ __forceinline__ void prism_geometry(const double* __restrict__ X, const int xb[3], const int xt[3], int l,
                                               double& twoA, double h[3])
{
    double x[3], y[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double* pb = X + 3 * (int64_t)(xb[a] + l);
        x[a] = pb[0];
        y[a] = pb[1];
        h[a] = X[3 * (int64_t)(xt[a] + l) + 2] - pb[2];
    }
    twoA = twice_area(x, y);
}

__device__ __forceinline__ void load_coord_map(const ColArgs& a, const LaneInfo& L, int xb[3], int xt[3])
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        xb[v] = L.valid ? a.xmap[(int64_t)L.cell * 6 + 2 * v] : 0;
        xt[v] = L.valid ? a.xmap[(int64_t)L.cell * 6 + 2 * v + 1] : 0;
    }
}

// ---------------------------------------------------------------------------
// P1 x P1 mass action / residual of the integral of f v: y (+)= M x.

template <int RACE, bool LIST>
__global__ void __launch_bounds__(256) k_mass_p1(const ColArgs a)
{
    LaneInfo L;
    if (!lane_info<LIST>(a, L)) return;
    int fb[3], ft[3], xb[3], xt[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        fb[v] = L.valid ? a.fmap[(int64_t)L.cell * 6 + 2 * v] : 0;
        ft[v] = L.valid ? a.fmap[(int64_t)L.cell * 6 + 2 * v + 1] : 0;
    }
    load_coord_map(a, L, xb, xt);
    double carry[3] = {0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = L.valid && l < a.n_layers;
        const int lo = l * a.off;
        double yb[3] = {0.0, 0.0, 0.0}, yt[3] = {0.0, 0.0, 0.0};
        if (act) {
            double xbv[3], xtv[3], h[3], twoA;
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                xbv[v] = a.in0[fb[v] + lo];
                xtv[v] = a.in0[ft[v] + lo];
            }
            prism_geometry(a.X, xb, xt, l, twoA, h);
            p1_mass(twoA, h, xbv, xtv, yb, yt);
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const double lv = level_value(yb[v], yt[v], carry[v], L, a.seg);
            if (act) {
                inc<RACE>(a.out0 + fb[v] + lo, lv);
                if (l == a.n_layers - 1) inc<RACE>(a.out0 + ft[v] + lo, yt[v]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// DG0 x DG0 mass action: one DoF per prism, no sharing.

template <bool LIST>
__global__ void __launch_bounds__(256) k_mass_dg0(const ColArgs a, int write)
{
    LaneInfo L;
    if (!lane_info<LIST>(a, L)) return;
    const int f0 = L.valid ? a.fmap[L.cell] : 0;
    int xb[3], xt[3];
    load_coord_map(a, L, xb, xt);
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        if (!(L.valid && l < a.n_layers)) continue;
        double h[3], twoA;
        prism_geometry(a.X, xb, xt, l, twoA, h);
        const int d = f0 + l * a.off;
        const double y = dg0_mass(twoA, h, a.in0[d]);
        if (write)
            a.out0[d] = y;
        else
            a.out0[d] += y;
    }
}

// ---------------------------------------------------------------------------
// DG1 x DG1 mass action: six DoFs per prism, no sharing.  Position p of the
// list is horizontal node p / 2 (at vertex p / 2), vertical node p % 2.

template <bool LIST>
__global__ void __launch_bounds__(256) k_mass_dg1(const ColArgs a, int write)
{
    LaneInfo L;
    if (!lane_info<LIST>(a, L)) return;
    int fm[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) fm[p] = L.valid ? a.fmap[(int64_t)L.cell * 6 + p] : 0;
    int xb[3], xt[3];
    load_coord_map(a, L, xb, xt);
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        if (!(L.valid && l < a.n_layers)) continue;
        const int lo = l * a.off;
        double xbv[3], xtv[3], yb[3], yt[3], h[3], twoA;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            xbv[v] = a.in0[fm[2 * v] + lo];
            xtv[v] = a.in0[fm[2 * v + 1] + lo];
        }
        prism_geometry(a.X, xb, xt, l, twoA, h);
        p1_mass(twoA, h, xbv, xtv, yb, yt);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            if (write) {
                a.out0[fm[2 * v] + lo] = yb[v];
                a.out0[fm[2 * v + 1] + lo] = yt[v];
            } else {
                a.out0[fm[2 * v] + lo] += yb[v];
                a.out0[fm[2 * v + 1] + lo] += yt[v];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P2 x P2 mass action.  Position 3e + beta of the list: horizontal node e
// (vertices 0..2, edges 0..2), vertical node beta (bottom, top, middle).

template <int RACE, bool LIST>
__global__ void __launch_bounds__(256) k_mass_p2(const ColArgs a)
{
    LaneInfo L;
    if (!lane_info<LIST>(a, L)) return;
    int fm[18];
#pragma unroll
    for (int p = 0; p < 18; ++p) fm[p] = L.valid ? a.fmap[(int64_t)L.cell * 18 + p] : 0;
    int xb[3], xt[3];
    load_coord_map(a, L, xb, xt);
    double carry[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = L.valid && l < a.n_layers;
        const int lo = l * a.off;
        double y[6][3];
#pragma unroll
        for (int e = 0; e < 6; ++e) y[e][0] = y[e][1] = y[e][2] = 0.0;
        if (act) {
            double x[6][3], h[3], twoA;
#pragma unroll
            for (int e = 0; e < 6; ++e)
#pragma unroll
                for (int b = 0; b < 3; ++b) x[e][b] = a.in0[fm[3 * e + b] + lo];
            prism_geometry(a.X, xb, xt, l, twoA, h);
            p2_mass(twoA, h, x, y);
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const double lv = level_value(y[e][0], y[e][1], carry[e], L, a.seg);
            if (act) {
                inc<RACE>(a.out0 + fm[3 * e] + lo, lv);
                inc<RACE>(a.out0 + fm[3 * e + 2] + lo, y[e][2]);
                if (l == a.n_layers - 1) inc<RACE>(a.out0 + fm[3 * e + 1] + lo, y[e][1]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Cubic residual F = integral (u^3 - f) v and its vector-Jacobian product
// with cotangent w:  g_u = integral 3 u^2 w v,  g_f = -integral w v = -M w.
// MODE 0: F (in0 = u, in1 = f; out0 = F)
// MODE 1: g_u, g_f (in0 = u, in1 = w; out0 = g_u, out1 = g_f)
// MODE 2: F, g_u, g_f (in0 = u, in1 = f, in2 = w; out0 = F, out1 = g_u, out2 = g_f)
// The adjoint reads w where the forward scatters F and scatters g_u, g_f where
// the forward gathers u, f.

template <int MODE, int RACE, bool LIST>
__global__ void __launch_bounds__(256) k_cubic_p1(const ColArgs a)
{
    constexpr int NOUT = MODE == 0 ? 1 : (MODE == 1 ? 2 : 3);
    LaneInfo L;
    if (!lane_info<LIST>(a, L)) return;
    int fb[3], ft[3], xb[3], xt[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        fb[v] = L.valid ? a.fmap[(int64_t)L.cell * 6 + 2 * v] : 0;
        ft[v] = L.valid ? a.fmap[(int64_t)L.cell * 6 + 2 * v + 1] : 0;
    }
    load_coord_map(a, L, xb, xt);
    CubicRule R;
    cubic_rule(R);
    double carry[NOUT][3];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) carry[o][0] = carry[o][1] = carry[o][2] = 0.0;
    double* outs[3] = {a.out0, a.out1, a.out2};
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = L.valid && l < a.n_layers;
        const int lo = l * a.off;
        double yb[NOUT][3], yt[NOUT][3];
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int v = 0; v < 3; ++v) yb[o][v] = yt[o][v] = 0.0;
        if (act) {
            double h[3], twoA;
            prism_geometry(a.X, xb, xt, l, twoA, h);
            double W[7][3];
            cubic_weights(R, twoA, h, W);
            double ub[3], ut[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                ub[v] = a.in0[fb[v] + lo];
                ut[v] = a.in0[ft[v] + lo];
            }
            double uq[7][3];
            p1_at_points(R, ub, ut, uq);
            if constexpr (MODE == 0 || MODE == 2) {
                double fbv[3], ftv[3], fq[7][3], s[7][3];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    fbv[v] = a.in1[fb[v] + lo];
                    ftv[v] = a.in1[ft[v] + lo];
                }
                p1_at_points(R, fbv, ftv, fq);
#pragma unroll
                for (int i = 0; i < 7; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) s[i][j] = W[i][j] * (uq[i][j] * uq[i][j] * uq[i][j] - fq[i][j]);
                p1_test(R, s, yb[0], yt[0]);
            }
            if constexpr (MODE == 1 || MODE == 2) {
                const double* w = MODE == 1 ? a.in1 : a.in2;
                double wb[3], wt[3], wq[7][3], s[7][3];
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    wb[v] = w[fb[v] + lo];
                    wt[v] = w[ft[v] + lo];
                }
                p1_at_points(R, wb, wt, wq);
#pragma unroll
                for (int i = 0; i < 7; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) s[i][j] = W[i][j] * 3.0 * uq[i][j] * uq[i][j] * wq[i][j];
                constexpr int og = MODE == 1 ? 0 : 1;
                p1_test(R, s, yb[og], yt[og]);
                double mb[3], mt[3];
                p1_mass(twoA, h, wb, wt, mb, mt);
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    yb[og + 1][v] = -mb[v];
                    yt[og + 1][v] = -mt[v];
                }
            }
        }
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const double lv = level_value(yb[o][v], yt[o][v], carry[o][v], L, a.seg);
                if (act) {
                    inc<RACE>(outs[o] + fb[v] + lo, lv);
                    if (l == a.n_layers - 1) inc<RACE>(outs[o] + ft[v] + lo, yt[o][v]);
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Dispatch.

template <bool LIST>
static int32_t dispatch(const LoopLaunch& P, const ColArgs& a, dim3 grid, dim3 block, hipStream_t s)
{
    const bool atomic = P.race == EXM_RACE_ATOMIC;
#define EXM_LAUNCH(K) hipLaunchKernelGGL(K, grid, block, 0, s, a)
    switch (P.element) {
    case EXM_ELEMENT_P1P1:
        switch (P.kernel) {
        case EXM_K_MASS:
            if (atomic) EXM_LAUNCH((k_mass_p1<EXM_RACE_ATOMIC, LIST>));
            else EXM_LAUNCH((k_mass_p1<EXM_RACE_COLOUR, LIST>));
            break;
        case EXM_K_CUBIC:
            if (atomic) EXM_LAUNCH((k_cubic_p1<0, EXM_RACE_ATOMIC, LIST>));
            else EXM_LAUNCH((k_cubic_p1<0, EXM_RACE_COLOUR, LIST>));
            break;
        case EXM_K_CUBIC_VJP:
            if (atomic) EXM_LAUNCH((k_cubic_p1<1, EXM_RACE_ATOMIC, LIST>));
            else EXM_LAUNCH((k_cubic_p1<1, EXM_RACE_COLOUR, LIST>));
            break;
        case EXM_K_CUBIC_FUSED:
            if (atomic) EXM_LAUNCH((k_cubic_p1<2, EXM_RACE_ATOMIC, LIST>));
            else EXM_LAUNCH((k_cubic_p1<2, EXM_RACE_COLOUR, LIST>));
            break;
        default: return fail(EXM_EUNSUPPORTED, "kernel %d not available on P1xP1", P.kernel);
        }
        break;
    case EXM_ELEMENT_P2P2:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on P2xP2", P.kernel);
        if (atomic) EXM_LAUNCH((k_mass_p2<EXM_RACE_ATOMIC, LIST>));
        else EXM_LAUNCH((k_mass_p2<EXM_RACE_COLOUR, LIST>));
        break;
    case EXM_ELEMENT_DG0DG0:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on DG0xDG0", P.kernel);
        hipLaunchKernelGGL((k_mass_dg0<LIST>), grid, block, 0, s, a, P.write);
        break;
    case EXM_ELEMENT_DG1DG1:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on DG1xDG1", P.kernel);
        hipLaunchKernelGGL((k_mass_dg1<LIST>), grid, block, 0, s, a, P.write);
        break;
    default: return fail(EXM_EUNSUPPORTED, "element %d has no kernels", P.element);
    }
#undef EXM_LAUNCH
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t launch_column_loop(const LoopLaunch& P, hipStream_t stream)
{
    if (P.cell_count <= 0) return EXM_OK;
    ColArgs a;
    a.n_layers = P.n_layers;
    a.off = P.field_offset;
    a.cpw = P.shape.cpw;
    a.seg = P.shape.seg;
    a.fmap = P.fmap;
    a.xmap = P.xmap;
    a.X = P.X;
    a.in0 = P.in[0];
    a.in1 = P.in[1];
    a.in2 = P.in[2];
    a.out0 = P.out[0];
    a.out1 = P.out[1];
    a.out2 = P.out[2];
    a.cells = P.cells;
    a.cell_begin = P.cell_begin;
    a.cell_count = P.cell_count;
    const int64_t waves = (P.cell_count + a.cpw - 1) / a.cpw;
    const int64_t blocks = (waves + P.shape.wpb - 1) / P.shape.wpb;
    if (blocks > INT32_MAX) return fail(EXM_ERANGE, "grid too large");
    dim3 grid((unsigned)blocks), block((unsigned)(64 * P.shape.wpb));
    return P.cells ? dispatch<true>(P, a, grid, block, stream) : dispatch<false>(P, a, grid, block, stream);
}

}  // namespace exm
