// The extruded parallel loop (Algorithm 3 of arXiv 1604.05937) for gfx950.
//
// Lanes and layers.  The vertical-innermost numbering makes the DoFs of one
// entity column contiguous, so a 64-lane wavefront takes cpw base cells side
// by side and gives each seg = 64 / cpw consecutive lanes, one layer per lane.
// A lane reads its cell's explicit lists once; the DoF of stencil position p
// at layer l is L(c)[p] + l * offset[p], so the seg lanes of one cell read seg
// consecutive DoFs of every column: each gather and scatter is a coalesced run
// rather than one cache line per lane.  A value on the top level of layer l is
// the bottom-level value of layer l + 1, so it is taken from the next lane
// with a cross-lane shuffle instead of a second load.
//
// Vertically shared levels.  The top-level contribution of a lane is added to
// the next lane's bottom-level one through a shuffle, so every level of every
// column receives one update per base cell and step.
//
// Two schedules (see exm.h):
//  * DIRECT: wavefronts walk whole columns of their own cells in steps of seg
//    layers and update the output directly -- hardware FP64 atomic adds, or
//    plain read-add-write when one launch holds one colour of base cells.
//  * TILED: a workgroup owns a compact tile of base cells; its wavefronts walk
//    the tile's cells step by step and sum the updates of every (vertex or
//    edge, level) of the tile in LDS, then the workgroup adds each sum to HBM
//    once -- atomically only for entities another tile also touches, or with
//    plain read-add-write when one launch holds one colour of tiles.  Columns
//    of DG spaces belong to one cell, so those run DIRECT.
//
// Vector fields (the coordinates) are stored component-major: component i of
// DoF n at X[i * n_dofs + n], so each component of a column is one contiguous
// run as well.
#include <algorithm>

#include "exm_elements.hpp"
#include "exm_internal.hpp"
#include "exm_tiled.hpp"

namespace exm {

// Workgroups are dispatched to the eight XCDs round-robin; renumber them so
// that every XCD (and its L2) works through one contiguous range of work.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

struct Lane {
    int lane, sub, lsub;
};

__device__ __forceinline__ Lane lane_of(int seg)
{
    Lane L;
    L.lane = threadIdx.x & 63;
    L.sub = L.lane / seg;
    L.lsub = L.lane - L.sub * seg;
    return L;
}

// The value the next lane holds (level l + 1 of the same column when this lane
// is not the last of its column segment); the segment's last lane loads it.
__device__ __forceinline__ double from_above(double mine, const double* next_addr, bool load_it)
{
    double v = __shfl_down(mine, 1, 64);
    if (load_it) v = *next_addr;
    return v;
}

// Top-level contribution of layer l - 1, held by the previous lane.
__device__ __forceinline__ double from_below(double top)
{
    return __shfl_up(top, 1, 64);
}

template <int RACE>
__device__ __forceinline__ void inc(double* p, double v)
{
    if constexpr (RACE == EXM_RACE_ATOMIC)
        unsafeAtomicAdd(p, v);
    else
        *p += v;
}

// (x, y) of the three base vertices, read once per cell: columns are vertical,
// so the coordinate field holds the same (x, y) at every level of a column.
// xb[a]: DoF of base vertex a at level 0 in the coordinate space; xn: its DoF
// count (component stride).
struct BaseXY {
    double x[3], y[3];
};

__device__ __forceinline__ BaseXY base_xy(const double* __restrict__ X, int64_t xn, const int xb[3], bool valid)
{
    BaseXY g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.x[a] = valid ? X[xb[a]] : 0.0;
        g.y[a] = valid ? X[xn + xb[a]] : 0.0;
    }
    return g;
}

// Geometry of the prism above the lane's layer l: twice the area of the base
// triangle and the three column heights (top z shuffled from the next lane).
__device__ __forceinline__ void geometry(const double* __restrict__ X, int64_t xn, const int xb[3], const BaseXY& g,
                                         int l, bool act, bool last, double& twoA, double h[3])
{
    double zb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) zb[a] = act ? X[2 * xn + (int64_t)xb[a] + l] : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double zt = from_above(zb[a], X + 2 * xn + (int64_t)xb[a] + l + 1, act && last);
        h[a] = zt - zb[a];
    }
    twoA = twice_area(g.x, g.y);
}

// ---------------------------------------------------------------------------
// P1 x P1 element kernels on one lane.  FORM 0: mass (in0 -> y0); 1: cubic
// residual (u, f -> F); 2: cubic VJP (u, w -> g_u, g_f); 3: fused (u, f, w ->
// F, g_u, g_f).  b[k][a], t[k][a]: input k at the bottom / top node of vertex a.

template <int FORM>
struct P1Form {
    static constexpr int NIN = FORM == 0 ? 1 : (FORM == 3 ? 3 : 2);
    static constexpr int NOUT = FORM == 0 ? 1 : (FORM == 1 ? 1 : (FORM == 2 ? 2 : 3));
};

template <int FORM>
__device__ __forceinline__ void p1_element(double twoA, const double h[3], const double b[][3], const double t[][3],
                                           double yb[][3], double yt[][3])
{
    if constexpr (FORM == 0)
        p1_mass(twoA, h, b[0], t[0], yb[0], yt[0]);
    else
        cubic_element<FORM>(twoA, h, b, t, yb, yt);
}

// Gather the inputs of a P1 lane and evaluate its element: level values of
// every output at the lane's own level (bottom contribution of layer l plus
// top contribution of layer l - 1 from the previous lane; `first` lanes get
// only their bottom) and the top-level contribution yt.
template <int FORM>
__device__ __forceinline__ void p1_lane(const ColArgs& a, const int fb[3], const int xb[3], const BaseXY& g, int l,
                                        bool act, bool last, bool first, double lev[][3], double yt[][3])
{
    constexpr int NIN = P1Form<FORM>::NIN;
    constexpr int NOUT = P1Form<FORM>::NOUT;
    const double* in[3] = {a.in0, a.in1, a.in2};
    double b[NIN][3], t[NIN][3];
    const int lo = l * a.off;
#pragma unroll
    for (int k = 0; k < NIN; ++k)
#pragma unroll
        for (int v = 0; v < 3; ++v) b[k][v] = act ? in[k][fb[v] + lo] : 0.0;
#pragma unroll
    for (int k = 0; k < NIN; ++k)
#pragma unroll
        for (int v = 0; v < 3; ++v) t[k][v] = from_above(b[k][v], in[k] + fb[v] + lo + a.off, act && last);
    double twoA, h[3];
    geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
    double yb[NOUT][3];
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int v = 0; v < 3; ++v) yb[o][v] = yt[o][v] = 0.0;
    if (act) p1_element<FORM>(twoA, h, b, t, yb, yt);
#pragma unroll
    for (int o = 0; o < NOUT; ++o)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const double below = from_below(yt[o][v]);
            lev[o][v] = yb[o][v] + (first ? 0.0 : below);
        }
}

// ---------------------------------------------------------------------------
// DIRECT schedule.

// Layers of the lane's cell column: the mesh's layer count, or the cell's own
// range on a mesh with a layer range per column (0 for a lane without a cell).
__device__ __forceinline__ int column_layers(const ColArgs& a, int32_t cell, bool valid)
{
    if (!valid) return 0;
    return a.cell_lam ? a.cell_lam[cell] : a.n_layers;
}

// Largest value over the wavefront, so that every lane runs the same steps
// (the steps exchange values across lanes).
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ bool direct_cell(const ColArgs& a, const Lane& L, int32_t& cell, bool& valid)
{
    const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t wave = (int64_t)blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wave * a.cpw >= a.cell_count) return false;   // uniform over the wavefront
    const int64_t slot = wave * a.cpw + L.sub;
    valid = L.sub < a.cpw && slot < a.cell_count;
    cell = valid ? (a.cells ? a.cells[a.cell_begin + slot] : (int32_t)(a.cell_begin + slot)) : 0;
    return true;
}

template <int FORM, int RACE>
__global__ void __launch_bounds__(256) k_direct_p1(const ColArgs a)
{
    constexpr int NOUT = P1Form<FORM>::NOUT;
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lamc = column_layers(a, cell, valid);   // this lane's column
    const int lamw = wave_max(lamc);                  // loop bound of the whole wavefront
    int fb[3], xb[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        fb[v] = valid ? a.fmap[(int64_t)cell * 6 + 2 * v] : 0;
        xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    }
    double* out[3] = {a.out0, a.out1, a.out2};
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    double carry[NOUT][3];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) carry[o][0] = carry[o][1] = carry[o][2] = 0.0;
    for (int l0 = 0; l0 < lamw; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < lamc;
        const bool last = L.lsub == a.seg - 1 || l == lamc - 1;
        double lev[NOUT][3], yt[NOUT][3];
        p1_lane<FORM>(a, fb, xb, g, l, act, last, L.lsub == 0, lev, yt);
        const int lo = l * a.off;
#pragma unroll
        for (int o = 0; o < NOUT; ++o)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                // the segment's first lane takes the previous step's top contribution
                const double val = lev[o][v] + (L.lsub == 0 ? carry[o][v] : 0.0);
                carry[o][v] = __shfl(yt[o][v], min(L.sub * a.seg + a.seg - 1, 63), 64);
                if (act) {
                    inc<RACE>(out[o] + fb[v] + lo, val);
                    if (l == lamc - 1) inc<RACE>(out[o] + fb[v] + lo + a.off, yt[o][v]);
                }
            }
    }
}

// DG0 x DG0 mass action: one DoF per prism (L(c)[0] + l), no sharing.
__global__ void __launch_bounds__(256) k_direct_dg0(const ColArgs a)
{
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lamc = column_layers(a, cell, valid);   // this lane's column
    const int lamw = wave_max(lamc);                  // loop bound of the whole wavefront
    const int f0 = valid ? a.fmap[cell] : 0;
    int xb[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    for (int l0 = 0; l0 < lamw; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < lamc;
        const bool last = L.lsub == a.seg - 1 || l == lamc - 1;
        double twoA, h[3];
        geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
        if (act) {
            const int64_t d = f0 + (int64_t)l * a.off;
            const double y = dg0_mass(twoA, h, a.in0[d]);
            if (a.write)
                a.out0[d] = y;
            else
                a.out0[d] += y;
        }
    }
}

// Mass action of the other tensor-product spaces (the paper's nine spaces
// are {CG1, DG0, DG1} horizontally x vertically).  NH horizontal nodes x NV
// vertical nodes; list position of node (alpha, beta): BMAJOR ? NH beta +
// alpha : NV alpha + beta (the order Algorithm 1's entity layout gives).
//   HSH   - horizontal nodes sit on base vertices, shared with other cells:
//           INC updates go through RACE (atomic, or one colour per launch);
//   VCONT - the vertical nodes are the bottom and top levels, shared with
//           the layers below and above: the top contribution of layer l - 1
//           reaches layer l's lane through a shuffle, so every level gets one
//           update per cell.
template <int NH, int NV, bool BMAJOR, bool HSH, bool VCONT, int RACE>
__global__ void __launch_bounds__(256) k_direct_tp(const ColArgs a)
{
    constexpr int K = NH * NV;
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lamc = column_layers(a, cell, valid);   // this lane's column
    const int lamw = wave_max(lamc);                  // loop bound of the whole wavefront
    int fb[NH][NV], xb[3];
#pragma unroll
    for (int al = 0; al < NH; ++al)
#pragma unroll
        for (int be = 0; be < NV; ++be) {
            const int p = BMAJOR ? NH * be + al : NV * al + be;
            fb[al][be] = valid ? a.fmap[(int64_t)cell * K + p] : 0;
        }
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    auto update = [&](double* p, double v) {
        if (a.write)
            *p = v;
        else if constexpr (HSH)
            inc<RACE>(p, v);
        else
            *p += v;
    };
    double carry[NH];
#pragma unroll
    for (int al = 0; al < NH; ++al) carry[al] = 0.0;
    for (int l0 = 0; l0 < lamw; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < lamc;
        const bool last = L.lsub == a.seg - 1 || l == lamc - 1;
        double twoA, h[3];
        geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
        const int64_t lo = (int64_t)l * a.off;
        double x[NH][NV], y[NH][NV];
#pragma unroll
        for (int al = 0; al < NH; ++al)
#pragma unroll
            for (int be = 0; be < NV; ++be) x[al][be] = act ? a.in0[fb[al][be] + lo] : 0.0;
        tp_mass<NH, NV>(twoA, h, x, y);
        if constexpr (VCONT) {
#pragma unroll
            for (int al = 0; al < NH; ++al) {
                const double below = from_below(y[al][1]);
                const double val = y[al][0] + (L.lsub == 0 ? carry[al] : below);
                carry[al] = __shfl(y[al][1], min(L.sub * a.seg + a.seg - 1, 63), 64);
                if (act) {
                    update(a.out0 + fb[al][0] + lo, val);
                    if (l == lamc - 1) update(a.out0 + fb[al][1] + lo, y[al][1]);
                }
            }
        } else {
            if (act)
#pragma unroll
                for (int al = 0; al < NH; ++al)
#pragma unroll
                    for (int be = 0; be < NV; ++be) update(a.out0 + fb[al][be] + lo, y[al][be]);
        }
    }
}

// DG1 x DG1 mass action: six consecutive DoFs per prism, L(c)[p] + 6 l; position
// p is horizontal node p / 2 (at vertex p / 2) and vertical node p % 2.
__global__ void __launch_bounds__(256) k_direct_dg1(const ColArgs a)
{
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lamc = column_layers(a, cell, valid);   // this lane's column
    const int lamw = wave_max(lamc);                  // loop bound of the whole wavefront
    const int f0 = valid ? a.fmap[(int64_t)cell * 6] : 0;
    int xb[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    for (int l0 = 0; l0 < lamw; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < lamc;
        const bool last = L.lsub == a.seg - 1 || l == lamc - 1;
        double twoA, h[3];
        geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
        if (act) {
            const int64_t d = f0 + (int64_t)l * a.off;
            double xb_[3], xt_[3], yb[3], yt[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                xb_[q] = a.in0[d + 2 * q];
                xt_[q] = a.in0[d + 2 * q + 1];
            }
            p1_mass(twoA, h, xb_, xt_, yb, yt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (a.write) {
                    a.out0[d + 2 * q] = yb[q];
                    a.out0[d + 2 * q + 1] = yt[q];
                } else {
                    a.out0[d + 2 * q] += yb[q];
                    a.out0[d + 2 * q + 1] += yt[q];
                }
            }
        }
    }
}

// P2 x P2 on one lane.  Entity e (vertices 0..2, edges 0..2) has its level
// nodes at L(c)[3e] + 2 l (bottom) and + 2 (top), its middle node at
// L(c)[3e + 2] + 2 l.  lev[e]: bottom value plus the top value of layer l - 1;
// yt[e]: top contribution; ym[e]: middle-node value.
__device__ __forceinline__ void p2_lane(const ColArgs& a, const int fb[6], const int fm[6], const int xb[3],
                                        const BaseXY& g, int l, bool act, bool last, bool first, double lev[6],
                                        double yt[6], double ym[6])
{
    double x[6][3], y[6][3];
    const int lo = l * a.off;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        x[e][0] = act ? a.in0[fb[e] + lo] : 0.0;
        x[e][2] = act ? a.in0[fm[e] + lo] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) x[e][1] = from_above(x[e][0], a.in0 + fb[e] + lo + a.off, act && last);
    double twoA, h[3];
    geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
#pragma unroll
    for (int e = 0; e < 6; ++e) y[e][0] = y[e][1] = y[e][2] = 0.0;
    if (act) p2_mass(twoA, h, x, y);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double below = from_below(y[e][1]);
        lev[e] = y[e][0] + (first ? 0.0 : below);
        yt[e] = y[e][1];
        ym[e] = y[e][2];
    }
}

template <int RACE>
__global__ void __launch_bounds__(256) k_direct_p2(const ColArgs a)
{
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lamc = column_layers(a, cell, valid);   // this lane's column
    const int lamw = wave_max(lamc);                  // loop bound of the whole wavefront
    int fb[6], fm[6], xb[3];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        fb[e] = valid ? a.fmap[(int64_t)cell * 18 + 3 * e] : 0;
        fm[e] = valid ? a.fmap[(int64_t)cell * 18 + 3 * e + 2] : 0;
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    double carry[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < lamw; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < lamc;
        const bool last = L.lsub == a.seg - 1 || l == lamc - 1;
        double lev[6], yt[6], ym[6];
        p2_lane(a, fb, fm, xb, g, l, act, last, L.lsub == 0, lev, yt, ym);
        const int lo = l * a.off;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const double val = lev[e] + (L.lsub == 0 ? carry[e] : 0.0);
            carry[e] = __shfl(yt[e], min(L.sub * a.seg + a.seg - 1, 63), 64);
            if (act) {
                inc<RACE>(a.out0 + fb[e] + lo, val);
                inc<RACE>(a.out0 + fm[e] + lo, ym[e]);
                if (l == lamc - 1) inc<RACE>(a.out0 + fb[e] + lo + a.off, yt[e]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// TILED schedule: per-tile sums in LDS.

__device__ __forceinline__ int32_t entity_id(int32_t tagged) { return tagged & 0x7fffffff; }
__device__ __forceinline__ bool entity_shared(int32_t tagged) { return tagged < 0; }

template <bool ATOMIC>
__device__ __forceinline__ void global_add(double* p, double v, bool shared)
{
    if (ATOMIC && shared)
        unsafeAtomicAdd(p, v);
    else
        *p += v;
}

struct TileRange {
    int32_t cb, nc, vb, nv, eb, ne;
};

__device__ __forceinline__ TileRange tile_range(const ColArgs& a, const TileArgs& t)
{
    TileRange r;
    const int32_t b = (int32_t)xcd_block(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + b] : t.tile_begin + b;
    r.cb = t.cell_off[tile];
    r.nc = t.cell_off[tile + 1] - r.cb;
    r.vb = t.vert_off[tile];
    r.nv = t.vert_off[tile + 1] - r.vb;
    if (t.edge_off) {
        r.eb = t.edge_off[tile];
        r.ne = t.edge_off[tile + 1] - r.eb;
    } else {
        r.eb = r.ne = 0;
    }
    return r;
}

// LDS layout: acc[o][slot * P + j] for output o, entity slot, position j in
// 0 .. P - 1 (P = seg + 1 levels for P1, 2 seg + 1 nodes for P2), then
// carry[o][slot].
template <int FORM, bool ATOMIC>
__global__ void __launch_bounds__(512) k_tiled_p1(const ColArgs a, const TileArgs t)
{
    constexpr int NOUT = P1Form<FORM>::NOUT;
    extern __shared__ double lds[];
    const Lane L = lane_of(a.seg);
    const TileRange R = tile_range(a, t);
    const int P = a.seg + 1;
    const int SP = t.vstride * P;
    double* acc = lds;
    double* carry = acc + NOUT * SP;
    double* out[3] = {a.out0, a.out1, a.out2};
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    for (int i = threadIdx.x; i < NOUT * R.nv; i += blockDim.x) carry[(i / R.nv) * t.vstride + i % R.nv] = 0.0;
    __syncthreads();
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int nl = min(a.seg, a.n_layers - l0);
        const int nlev = nl + 1;
        const bool last_step = l0 + nl == a.n_layers;
        for (int i = threadIdx.x; i < R.nv * nlev; i += blockDim.x) {
            const int v = i / nlev;
            const int j = i - v * nlev;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) acc[o * SP + v * P + j] = j == 0 ? carry[o * t.vstride + v] : 0.0;
        }
        __syncthreads();
        for (int g = wave; g * a.cpw < R.nc; g += nwaves) {   // uniform over the wavefront
            const int slot = g * a.cpw + L.sub;
            const bool valid = L.sub < a.cpw && slot < R.nc;
            const int32_t cell = valid ? t.cells[R.cb + slot] : 0;
            int fb[3], xb[3], lv[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                fb[v] = valid ? a.fmap[(int64_t)cell * 6 + 2 * v] : 0;
                xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
                lv[v] = valid ? t.lcv[(int64_t)(R.cb + slot) * 3 + v] : 0;
            }
            const int l = l0 + L.lsub;
            const bool act = valid && L.lsub < nl;
            const bool last = L.lsub == nl - 1;
            const BaseXY gxy = base_xy(a.X, a.xn, xb, valid);
            double lev[NOUT][3], yt[NOUT][3];
            p1_lane<FORM>(a, fb, xb, gxy, l, act, last, L.lsub == 0, lev, yt);
            if (act) {
#pragma unroll
                for (int o = 0; o < NOUT; ++o)
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        atomicAdd(acc + o * SP + lv[v] * P + L.lsub, lev[o][v]);
                        if (last) atomicAdd(acc + o * SP + lv[v] * P + nl, yt[o][v]);
                    }
            }
        }
        __syncthreads();
        const int nflush = last_step ? nlev : nl;
        for (int i = threadIdx.x; i < R.nv * nlev; i += blockDim.x) {
            const int v = i / nlev;
            const int j = i - v * nlev;
            const int32_t tag = t.verts[R.vb + v];
            if (j < nflush) {
                const int64_t d = (int64_t)t.fstart0[entity_id(tag)] + (int64_t)(l0 + j) * a.off;
#pragma unroll
                for (int o = 0; o < NOUT; ++o) global_add<ATOMIC>(out[o] + d, acc[o * SP + v * P + j], entity_shared(tag));
            } else {
#pragma unroll
                for (int o = 0; o < NOUT; ++o) carry[o * t.vstride + v] = acc[o * SP + v * P + j];
            }
        }
        __syncthreads();
    }
}

template <bool ATOMIC>
__global__ void __launch_bounds__(512) k_tiled_p2(const ColArgs a, const TileArgs t)
{
    extern __shared__ double lds[];
    const Lane L = lane_of(a.seg);
    const TileRange R = tile_range(a, t);
    const int P = 2 * a.seg + 1;
    const int ES = t.vstride + t.estride;
    double* acc = lds;
    double* carry = acc + ES * P;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int nent = R.nv + R.ne;
    for (int i = threadIdx.x; i < ES; i += blockDim.x) carry[i] = 0.0;
    __syncthreads();
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int nl = min(a.seg, a.n_layers - l0);
        const int npos = 2 * nl + 1;
        const bool last_step = l0 + nl == a.n_layers;
        for (int i = threadIdx.x; i < nent * npos; i += blockDim.x) {
            const int e = i / npos;
            const int jj = i - e * npos;
            const int slot = e < R.nv ? e : t.vstride + (e - R.nv);
            acc[slot * P + jj] = jj == 0 ? carry[slot] : 0.0;
        }
        __syncthreads();
        for (int g = wave; g * a.cpw < R.nc; g += nwaves) {
            const int slot = g * a.cpw + L.sub;
            const bool valid = L.sub < a.cpw && slot < R.nc;
            const int32_t cell = valid ? t.cells[R.cb + slot] : 0;
            int fb[6], fm[6], xb[3], es[6];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                fb[e] = valid ? a.fmap[(int64_t)cell * 18 + 3 * e] : 0;
                fm[e] = valid ? a.fmap[(int64_t)cell * 18 + 3 * e + 2] : 0;
            }
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
                es[v] = valid ? t.lcv[(int64_t)(R.cb + slot) * 3 + v] : 0;
                es[3 + v] = valid ? t.vstride + t.lce[(int64_t)(R.cb + slot) * 3 + v] : 0;
            }
            const int l = l0 + L.lsub;
            const bool act = valid && L.lsub < nl;
            const bool last = L.lsub == nl - 1;
            const BaseXY gxy = base_xy(a.X, a.xn, xb, valid);
            double lev[6], yt[6], ym[6];
            p2_lane(a, fb, fm, xb, gxy, l, act, last, L.lsub == 0, lev, yt, ym);
            if (act) {
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    atomicAdd(acc + es[e] * P + 2 * L.lsub, lev[e]);
                    atomicAdd(acc + es[e] * P + 2 * L.lsub + 1, ym[e]);
                    if (last) atomicAdd(acc + es[e] * P + 2 * nl, yt[e]);
                }
            }
        }
        __syncthreads();
        const int nflush = last_step ? npos : npos - 1;
        for (int i = threadIdx.x; i < nent * npos; i += blockDim.x) {
            const int e = i / npos;
            const int jj = i - e * npos;
            const int slot = e < R.nv ? e : t.vstride + (e - R.nv);
            const int32_t tag = e < R.nv ? t.verts[R.vb + e] : t.edges[R.eb + e - R.nv];
            if (jj < nflush) {
                const int32_t start = e < R.nv ? t.fstart0[entity_id(tag)] : t.fstart1[entity_id(tag)];
                global_add<ATOMIC>(a.out0 + (int64_t)start + (int64_t)l0 * a.off + jj, acc[slot * P + jj],
                                   entity_shared(tag));
            } else {
                carry[slot] = acc[slot * P + jj];
            }
        }
        __syncthreads();
    }
}

// Mixed-degree DG mass action (a space with a DoF count per entity whose
// cells carry DG0 x DG0 or DG1 x DG1): the length of a cell's list is its DoF
// count per layer nd (1 or 6), and its DoFs are the contiguous column
// L(c)[0] + nd l + p, position p = 2a + b for DG1 (vertex a, bottom / top b).
__global__ void __launch_bounds__(256) k_direct_dgmix(const ColArgs a)
{
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int32_t lo = valid ? a.list_off[cell] : 0;
    const int nd = valid ? a.list_off[cell + 1] - lo : 0;
    const int f0 = valid ? a.fmap[lo] : 0;
    int xb[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    for (int l0 = 0; l0 < a.n_layers; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l < a.n_layers;
        const bool last = L.lsub == a.seg - 1 || l == a.n_layers - 1;
        double twoA, h[3];
        geometry(a.X, a.xn, xb, g, l, act, last, twoA, h);
        if (!act) continue;
        const int64_t d = f0 + (int64_t)l * nd;
        if (nd == 1) {
            const double y = dg0_mass(twoA, h, a.in0[d]);
            if (a.write)
                a.out0[d] = y;
            else
                a.out0[d] += y;
        } else {
            double xb6[3], xt6[3], yb[3], yt[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                xb6[q] = a.in0[d + 2 * q];
                xt6[q] = a.in0[d + 2 * q + 1];
            }
            p1_mass(twoA, h, xb6, xt6, yb, yt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (a.write) {
                    a.out0[d + 2 * q] = yb[q];
                    a.out0[d + 2 * q + 1] = yt[q];
                } else {
                    a.out0[d + 2 * q] += yb[q];
                    a.out0[d + 2 * q + 1] += yt[q];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Horizontal facets: Algorithm 3 with d2 = 0, lambda + 1 facets per column
// (levels l = 0 .. lambda).  Lane = facet.  Facet l lies between the prism of
// layer l - 1 (below) and that of layer l (above); it integrates [x][v] dS with
// [x] = x_below - x_above, zero outside the domain on the bottom and top
// facets.  The facet is the flat triangle through the column vertices at
// level l, so dS = |n| dxi deta (n the cross product of two edges) and the
// facet mass of the horizontal basis is |n| (1 + [a = b]) / 24 for the P1
// functions, |n| / 2 for the constant.  NH horizontal x NV vertical nodes,
// list position NV a + b; only vertically discontinuous spaces (the jump of a
// continuous field vanishes).
//   NV = 2: the top nodes of the prism below and the bottom nodes of the
//           prism above are distinct DoFs, each touched by one facet;
//   NV = 1: the one DoF of prism l - 1 takes shares from facets l - 1 and l:
//           lane l adds the share of facet l - 1 (shuffled up from the lane
//           below, or carried from the previous step) and updates it once.
template <int NH, int NV, bool HSH, int RACE>
__global__ void __launch_bounds__(256) k_direct_facet(const ColArgs a)
{
    constexpr int K = NH * NV;
    const Lane L = lane_of(a.seg);
    int32_t cell;
    bool valid;
    if (!direct_cell(a, L, cell, valid)) return;
    const int lam = a.n_layers;
    int fb[NH][NV], xb[3];
#pragma unroll
    for (int al = 0; al < NH; ++al)
#pragma unroll
        for (int be = 0; be < NV; ++be) fb[al][be] = valid ? a.fmap[(int64_t)cell * K + NV * al + be] : 0;
#pragma unroll
    for (int v = 0; v < 3; ++v) xb[v] = valid ? a.xmap[(int64_t)cell * 6 + 2 * v] : 0;
    const BaseXY g = base_xy(a.X, a.xn, xb, valid);
    auto update = [&](double* p, double v) {
        if (a.write)
            *p = v;
        else if constexpr (HSH)
            inc<RACE>(p, v);
        else
            *p += v;
    };
    double carry[NH], xcarry[NH];   // shares of facet l - 1 and (NV = 1) the field value below, per step
#pragma unroll
    for (int al = 0; al < NH; ++al) carry[al] = xcarry[al] = 0.0;
    for (int l0 = 0; l0 <= lam; l0 += a.seg) {
        const int l = l0 + L.lsub;
        const bool act = valid && l <= lam;
        const bool below = act && l >= 1, above = act && l < lam;
        double z[3];
#pragma unroll
        for (int v = 0; v < 3; ++v) z[v] = act ? a.X[2 * a.xn + (int64_t)xb[v] + l] : 0.0;
        const double ex0 = g.x[1] - g.x[0], ey0 = g.y[1] - g.y[0], ez0 = z[1] - z[0];
        const double ex1 = g.x[2] - g.x[0], ey1 = g.y[2] - g.y[0], ez1 = z[2] - z[0];
        const double nx = ey0 * ez1 - ez0 * ey1, ny = ez0 * ex1 - ex0 * ez1, nz = ex0 * ey1 - ey0 * ex1;
        const double n = sqrt(nx * nx + ny * ny + nz * nz);
        const int64_t lb = (int64_t)(l - 1) * a.off, la = (int64_t)l * a.off;
        double j[NH];
#pragma unroll
        for (int al = 0; al < NH; ++al) {
            const double hi = above ? a.in0[fb[al][0] + la] : 0.0;        // bottom node of the prism above
            double lo;                                                    // top node of the prism below
            if constexpr (NV == 1) {
                // one DoF per prism: the value below is the lane below's value above
                const double up = from_below(hi);
                lo = below ? (L.lsub == 0 ? xcarry[al] : up) : 0.0;
                xcarry[al] = __shfl(hi, min(L.sub * a.seg + a.seg - 1, 63), 64);
            } else {
                lo = below ? a.in0[fb[al][NV - 1] + lb] : 0.0;
            }
            j[al] = lo - hi;
        }
        double r[NH];
        if constexpr (NH == 3) {
            const double J = j[0] + j[1] + j[2];
#pragma unroll
            for (int al = 0; al < 3; ++al) r[al] = n * (j[al] + J) * (1.0 / 24.0);
        } else {
            r[0] = n * j[0] * 0.5;
        }
        if constexpr (NV == 2) {
#pragma unroll
            for (int al = 0; al < NH; ++al) {
                if (below) update(a.out0 + fb[al][1] + lb, r[al]);
                if (above) update(a.out0 + fb[al][0] + la, -r[al]);
            }
        } else {
#pragma unroll
            for (int al = 0; al < NH; ++al) {
                const double prev = from_below(-r[al]);
                const double share = L.lsub == 0 ? carry[al] : prev;
                carry[al] = __shfl(-r[al], min(L.sub * a.seg + a.seg - 1, 63), 64);
                if (below) update(a.out0 + fb[al][0] + lb, r[al] + share);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Dispatch.

ColArgs col_args(const LoopLaunch& P)
{
    ColArgs a;
    a.n_layers = P.n_layers;
    a.cell_lam = P.cell_lam;
    a.list_off = P.list_off;
    a.off = P.field_offset;
    a.cpw = P.shape.cpw;
    a.seg = P.shape.seg;
    a.xn = P.xspace->n_dofs;
    a.fn = P.fspace->n_dofs;
    a.fmap = P.fmap;
    a.xmap = P.xmap;
    a.X = P.X;
    a.in0 = P.in[0];
    a.in1 = P.in[1];
    a.in2 = P.in[2];
    a.out0 = P.out[0];
    a.out1 = P.out[1];
    a.out2 = P.out[2];
    a.write = P.write;
    a.cells = P.cells;
    a.cell_begin = P.cell_begin;
    a.cell_count = P.cell_count;
    return a;
}

int32_t launch_column_loop(const LoopLaunch& P, hipStream_t stream)
{
    if (P.cell_count <= 0) return EXM_OK;
    const ColArgs a = col_args(P);
    const int64_t waves = (P.cell_count + a.cpw - 1) / a.cpw;
    const int64_t blocks = (waves + P.shape.wpb - 1) / P.shape.wpb;
    if (blocks > INT32_MAX) return fail(EXM_ERANGE, "grid too large");
    dim3 grid((unsigned)blocks), block((unsigned)(64 * P.shape.wpb));
    const bool atomic = P.race == EXM_RACE_ATOMIC;
#define EXM_LAUNCH(K) hipLaunchKernelGGL(K, grid, block, 0, stream, a)
#define EXM_LAUNCH_RACE(F)                                                           \
    do {                                                                             \
        if (atomic) EXM_LAUNCH((k_direct_p1<F, EXM_RACE_ATOMIC>));                   \
        else EXM_LAUNCH((k_direct_p1<F, EXM_RACE_COLOUR>));                          \
    } while (0)
    if (P.kernel == EXM_K_FACET_JUMP) {
        switch (P.element) {
        case EXM_ELEMENT_DG0DG0: EXM_LAUNCH((k_direct_facet<1, 1, false, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_DG1DG1: EXM_LAUNCH((k_direct_facet<3, 2, false, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_DG0DG1: EXM_LAUNCH((k_direct_facet<1, 2, false, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_DG1DG0: EXM_LAUNCH((k_direct_facet<3, 1, false, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_P1DG0:
            if (atomic) EXM_LAUNCH((k_direct_facet<3, 1, true, EXM_RACE_ATOMIC>));
            else EXM_LAUNCH((k_direct_facet<3, 1, true, EXM_RACE_COLOUR>));
            break;
        case EXM_ELEMENT_P1DG1:
            if (atomic) EXM_LAUNCH((k_direct_facet<3, 2, true, EXM_RACE_ATOMIC>));
            else EXM_LAUNCH((k_direct_facet<3, 2, true, EXM_RACE_COLOUR>));
            break;
        default: return fail(EXM_EUNSUPPORTED, "no facet kernel on element %d", P.element);
        }
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    switch (P.element) {
    case EXM_ELEMENT_P1P1:
        switch (P.kernel) {
        case EXM_K_MASS: EXM_LAUNCH_RACE(0); break;
        case EXM_K_CUBIC: EXM_LAUNCH_RACE(1); break;
        case EXM_K_CUBIC_VJP: EXM_LAUNCH_RACE(2); break;
        case EXM_K_CUBIC_FUSED: EXM_LAUNCH_RACE(3); break;
        default: return fail(EXM_EUNSUPPORTED, "kernel %d not available on P1xP1", P.kernel);
        }
        break;
    case EXM_ELEMENT_P2P2:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on P2xP2", P.kernel);
        if (atomic) EXM_LAUNCH((k_direct_p2<EXM_RACE_ATOMIC>));
        else EXM_LAUNCH((k_direct_p2<EXM_RACE_COLOUR>));
        break;
    case EXM_ELEMENT_DG0DG0:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on DG0xDG0", P.kernel);
        EXM_LAUNCH(k_direct_dg0);
        break;
    case EXM_ELEMENT_DG1DG1:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on DG1xDG1", P.kernel);
        EXM_LAUNCH(k_direct_dg1);
        break;
    case EXM_ELEMENT_DGMIX:
        if (P.kernel != EXM_K_MASS) return fail(EXM_EUNSUPPORTED, "kernel %d not available on EXM_ELEMENT_DGMIX", P.kernel);
        EXM_LAUNCH(k_direct_dgmix);
        break;
    case EXM_ELEMENT_P1DG0:
    case EXM_ELEMENT_P1DG1:
    case EXM_ELEMENT_DG0P1:
    case EXM_ELEMENT_DG0DG1:
    case EXM_ELEMENT_DG1P1:
    case EXM_ELEMENT_DG1DG0:
        if (P.kernel != EXM_K_MASS)
            return fail(EXM_EUNSUPPORTED, "kernel %d not available on element %d", P.kernel, P.element);
        switch (P.element) {
        case EXM_ELEMENT_P1DG0:   // vertex columns, one DoF per layer
            if (atomic) EXM_LAUNCH((k_direct_tp<3, 1, false, true, false, EXM_RACE_ATOMIC>));
            else EXM_LAUNCH((k_direct_tp<3, 1, false, true, false, EXM_RACE_COLOUR>));
            break;
        case EXM_ELEMENT_P1DG1:   // vertex columns, two DoFs per layer
            if (atomic) EXM_LAUNCH((k_direct_tp<3, 2, false, true, false, EXM_RACE_ATOMIC>));
            else EXM_LAUNCH((k_direct_tp<3, 2, false, true, false, EXM_RACE_COLOUR>));
            break;
        case EXM_ELEMENT_DG0P1: EXM_LAUNCH((k_direct_tp<1, 2, false, false, true, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_DG0DG1: EXM_LAUNCH((k_direct_tp<1, 2, false, false, false, EXM_RACE_ATOMIC>)); break;
        case EXM_ELEMENT_DG1P1: EXM_LAUNCH((k_direct_tp<3, 2, true, false, true, EXM_RACE_ATOMIC>)); break;
        default: EXM_LAUNCH((k_direct_tp<3, 1, false, false, false, EXM_RACE_ATOMIC>)); break;
        }
        break;
    default: return fail(EXM_EUNSUPPORTED, "element %d has no kernels", P.element);
    }
#undef EXM_LAUNCH_RACE
#undef EXM_LAUNCH
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t tiled_max_threads(int32_t kernel, int32_t element)
{
    (void)kernel;
    (void)element;
    return 512;
}

size_t tiled_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t estride, int32_t seg)
{
    switch (element) {
    case EXM_ELEMENT_P1P1: {
        int nout = 1;
        if (kernel == EXM_K_CUBIC_VJP) nout = 2;
        if (kernel == EXM_K_CUBIC_FUSED) nout = 3;
        return sizeof(double) * (size_t)nout * vstride * (seg + 2);
    }
    case EXM_ELEMENT_P2P2: {
        const size_t es = (size_t)vstride + estride;
        return sizeof(double) * es * (2 * (size_t)seg + 2);
    }
    default: return 0;
    }
}

int32_t launch_tiled(const LoopLaunch& P, const TileArgs& t, int32_t threads, size_t lds, hipStream_t s)
{
    if (t.tile_count <= 0) return EXM_OK;
    const ColArgs a = col_args(P);
    dim3 grid((unsigned)t.tile_count), block((unsigned)threads);
    const bool atomic = P.race == EXM_RACE_ATOMIC;
#define EXM_TL(K) hipLaunchKernelGGL(K, grid, block, lds, s, a, t)
#define EXM_TL_RACE(F)                                 \
    do {                                               \
        if (atomic) EXM_TL((k_tiled_p1<F, true>));     \
        else EXM_TL((k_tiled_p1<F, false>));           \
    } while (0)
    switch (P.element) {
    case EXM_ELEMENT_P1P1:
        switch (P.kernel) {
        case EXM_K_MASS: EXM_TL_RACE(0); break;
        case EXM_K_CUBIC: EXM_TL_RACE(1); break;
        case EXM_K_CUBIC_VJP: EXM_TL_RACE(2); break;
        case EXM_K_CUBIC_FUSED: EXM_TL_RACE(3); break;
        default: return fail(EXM_EUNSUPPORTED, "kernel %d not available on P1xP1", P.kernel);
        }
        break;
    case EXM_ELEMENT_P2P2:
        if (atomic) EXM_TL((k_tiled_p2<true>));
        else EXM_TL((k_tiled_p2<false>));
        break;
    default: return fail(EXM_EUNSUPPORTED, "element %d has no tiled kernels", P.element);
    }
#undef EXM_TL_RACE
#undef EXM_TL
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

}  // namespace exm
