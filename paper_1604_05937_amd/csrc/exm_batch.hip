// Batched assembly: many extruded meshes, several fields per mesh, forward
// residual b = M f plus its adjoint g = M^T w = M w, in two launches (one
// per kind of item, on parallel branches) captured in a HIP graph.  All
// fields of a mesh live on one space and share its explicit lists (end of
// Section 3.3 of the paper), so the geometry read for a column serves
// several fields.
//
// Tiles.  Each kind normally runs on the PIPELINED tile walk (exm_pipe.hip):
// one workgroup per (item, tile) of every item of the kind runs all fields
// and adjoints of its item through one set-up of the tile.  P1 x P1 items use
// owner tiles, each overwriting the outputs of the vertices it owns; a
// DG0 x DG0 output belongs to one cell.  Tile size and chunk length are timed
// at creation.
//
// Work units.  Where no tiling fits a kind (or on request), its items are cut
// into units of consecutive base entities, and a fixed grid of workgroups
// pulls units from a device counter until the list is exhausted, so meshes
// of very different sizes and layer counts balance across the GPU.  DG0
// units are base cells, their columns walked as in the DIRECT schedule
// (cols_per_wave cells side by side, one layer per lane).  P1 units are base
// vertices, each owned by one wavefront (the GATHER form of the loop) that
// walks the fan of cells around its vertex column, 62 levels per step, four
// fields at a time.  Vertex and cell units run in two persistent kernels
// with a work list each (the P1 path's registers would otherwise lower the
// occupancy of the DG0 path); the graph first resets the two work counters
// with a one-thread kernel.
//
// Either way every output DoF is written once, so no output needs zeroing and
// no atomics are needed.
#include <algorithm>
#include <cstring>
#include <iterator>
#include <utility>
#include <vector>

#include "exm_elements.hpp"
#include "exm_tiled.hpp"

namespace exm {

struct BatchItemDev {
    int32_t element;
    int32_t n_layers;
    int32_t off;
    int32_t cpw, seg;
    int32_t n_fields;
    int32_t adjoint;
    int32_t pad;
    int64_t xn;
    int64_t fbase, xbase;     // P1: column start of vertex w is base + w (lambda + 1)
    const int32_t* fan_off;   // P1: fans of cells around every vertex (see exm_gather.hip)
    const int32_t* fan;
    const int32_t* fmap;
    const int32_t* xmap;
    const double* X;
    const double* const* f;
    double* const* b;
    const double* const* w;
    double* const* g;
};

struct Unit {
    int32_t item;
    int32_t cell_begin;
    int32_t cell_count;
    int32_t pad;
};

__global__ void k_batch_reset(int32_t* counter)
{
    counter[0] = 0;
    counter[1] = 0;
}

__device__ __forceinline__ double next_lane(double v) { return __shfl_down(v, 1, 64); }

constexpr int kVOwned = 62;   // P1: levels a wavefront writes per step (one halo lane at each end)
constexpr int kVGroup = 4;    // P1: fields (forward and adjoint counted apart) per walk of the fan
constexpr int kVBlk = 2;      // P1: fan entries whose loads are issued together

// P1 x P1: the column of base vertex v, every field and its adjoint.  Lane
// `lane` of a step holds level lev = l0 - 1 + lane; it evaluates the row of v
// of prism (c, lev) for every cell c of the fan (bottom and top), keeps the
// bottom row and passes the top row one lane up, where it belongs to level
// lev + 1.  The fan lists the neighbouring vertices in cyclic order, so each
// neighbouring column is loaded once for the two cells that share it.
__device__ void batch_p1_vertex(const BatchItemDev& I, int32_t v, int lane)
{
    const int64_t lamp = (int64_t)I.n_layers + 1;
    const double* __restrict__ Z = I.X + 2 * I.xn;
    const int64_t fv = I.fbase + (int64_t)v * lamp, xv = I.xbase + (int64_t)v * lamp;
    const double px0 = I.X[xv], py0 = I.X[I.xn + xv];
    const int32_t e0 = I.fan_off[v], e1 = I.fan_off[v + 1];
    const int nfp = I.adjoint ? 2 * I.n_fields : I.n_fields;   // forward fields, then adjoint ones
    for (int l0 = 0; l0 <= I.n_layers; l0 += kVOwned) {
        const int lev = l0 - 1 + lane;
        const bool in = lev >= 0 && lev <= I.n_layers;   // a level of the column
        const bool prism = lev >= 0 && lev < I.n_layers;  // the prism above it exists
        const double z0 = in ? Z[xv + lev] : 0.0;
        const double z0n = next_lane(z0);
        for (int k0 = 0; k0 < nfp; k0 += kVGroup) {
            const double* src[kVGroup];
            double f0[kVGroup], f0n[kVGroup], fp[kVGroup], fpn[kVGroup], ab[kVGroup], at[kVGroup];
#pragma unroll
            for (int j = 0; j < kVGroup; ++j) {
                const int k = k0 + j;   // uniform
                src[j] = k < I.n_fields ? I.f[k] : (k < nfp ? I.w[k - I.n_fields] : nullptr);
                f0[j] = k < nfp && in ? src[j][fv + lev] : 0.0;
                f0n[j] = next_lane(f0[j]);
                fp[j] = fpn[j] = ab[j] = at[j] = 0.0;
            }
            double zp = 0.0, zpn = 0.0, pxp = 0.0, pyp = 0.0;   // the previous neighbour
            for (int32_t eb = e0; eb < e1; eb += kVBlk) {
                // the loads of kVBlk fan entries are in flight before the first is used
                int32_t ent[kVBlk];
                double z1[kVBlk], px1[kVBlk], py1[kVBlk], f1[kVBlk][kVGroup];
#pragma unroll
                for (int q = 0; q < kVBlk; ++q) {
                    const bool has = eb + q < e1;   // uniform
                    ent[q] = has ? I.fan[eb + q] : 0;
                    const int64_t w = ent[q] & 0x7fffffff;
                    const int64_t fw = I.fbase + w * lamp, xw = I.xbase + w * lamp;
                    z1[q] = has && in ? Z[xw + lev] : 0.0;
                    px1[q] = has ? I.X[xw] : 0.0;
                    py1[q] = has ? I.X[I.xn + xw] : 0.0;
#pragma unroll
                    for (int j = 0; j < kVGroup; ++j) f1[q][j] = has && k0 + j < nfp && in ? src[j][fw + lev] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kVBlk; ++q) {
                    if (eb + q >= e1) break;   // uniform
                    const double z1n = next_lane(z1[q]);
                    const bool cell = ent[q] >= 0 && prism;   // cell (v, previous, w)
                    const double s =
                        fabs((pxp - px0) * (py1[q] - py0) - (px1[q] - px0) * (pyp - py0)) * (1.0 / 120.0);
                    const double h[3] = {z0n - z0, zpn - zp, z1n - z1[q]};
#pragma unroll
                    for (int j = 0; j < kVGroup; ++j) {
                        const double f1n = next_lane(f1[q][j]);
                        if (cell && k0 + j < nfp) {
                            const double xb[3] = {f0[j], fp[j], f1[q][j]};
                            const double xt[3] = {f0n[j], fpn[j], f1n};
                            double yb, yt;
                            p1_row(s, h, xb, xt, yb, yt);
                            ab[j] += yb;
                            at[j] += yt;
                        }
                        fp[j] = f1[q][j];
                        fpn[j] = f1n;
                    }
                    zp = z1[q];
                    zpn = z1n;
                    pxp = px1[q];
                    pyp = py1[q];
                }
            }
#pragma unroll
            for (int j = 0; j < kVGroup; ++j) {
                const int k = k0 + j;
                const double below = __shfl_up(at[j], 1, 64);
                if (k < nfp && lane >= 1 && lane <= kVOwned && in) {
                    double* dst = k < I.n_fields ? I.b[k] : I.g[k - I.n_fields];
                    dst[fv + lev] = ab[j] + below;
                }
            }
        }
    }
}

__device__ __forceinline__ void batch_dg0_step(const BatchItemDev& I, int f0, const int xb[3], const double gx[3],
                                               const double gy[3], int l, bool act, bool last)
{
    double zb[3], h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) zb[a] = act ? I.X[2 * I.xn + (int64_t)xb[a] + l] : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double zt = next_lane(zb[a]);
        if (act && last) zt = I.X[2 * I.xn + (int64_t)xb[a] + l + 1];
        h[a] = zt - zb[a];
    }
    if (!act) return;
    const double vol = twice_area(gx, gy) * (h[0] + h[1] + h[2]) * (1.0 / 6.0);
    const int64_t d = f0 + (int64_t)l * I.off;
    for (int k = 0; k < I.n_fields; ++k) I.b[k][d] = I.f[k][d] * vol;
    if (I.adjoint)
        for (int k = 0; k < I.n_fields; ++k) I.g[k][d] = I.w[k][d] * vol;
}

// The persistent kernel over the units of one kind: P1 (base vertices) or
// DG0 (base cells).
template <bool P1>
__global__ void __launch_bounds__(256) k_batch(const BatchItemDev* __restrict__ items, const Unit* __restrict__ units,
                                               int32_t n_units, int32_t* counter)
{
    __shared__ int32_t s_unit;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t u = s_unit;
        __syncthreads();
        if (u >= n_units) break;   // every wave of the workgroup leaves together
        const Unit U = units[u];
        const BatchItemDev& I = items[U.item];
        if constexpr (P1) {   // a range of base vertices, one per wavefront
            for (int i = wave; i < U.cell_count; i += nwaves) batch_p1_vertex(I, U.cell_begin + i, lane);
            continue;
        }
        const int sub = lane / I.seg;
        const int lsub = lane - sub * I.seg;
        for (int grp = wave; grp * I.cpw < U.cell_count; grp += nwaves) {   // uniform over the wavefront
            const int slot = grp * I.cpw + sub;
            const bool valid = sub < I.cpw && slot < U.cell_count;
            const int32_t cell = valid ? U.cell_begin + slot : 0;
            int xb[3];
            double gx[3], gy[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xb[a] = valid ? I.xmap[(int64_t)cell * 6 + 2 * a] : 0;
                gx[a] = valid ? I.X[xb[a]] : 0.0;
                gy[a] = valid ? I.X[I.xn + xb[a]] : 0.0;
            }
            const int f0 = valid ? I.fmap[cell] : 0;
            for (int l0 = 0; l0 < I.n_layers; l0 += I.seg) {
                const int l = l0 + lsub;
                const bool act = valid && l < I.n_layers;
                const bool last = lsub == I.seg - 1 || l == I.n_layers - 1;
                batch_dg0_step(I, f0, xb, gx, gy, l, act, last);
            }
        }
    }
}

// The items of one kind on tiles (P1: owner tiles, DG0: tiles), one
// workgroup per (item, tile), every field of the item through one set-up.
struct TileSet {
    bool on = false;
    bool shared = false;           // P1: shared tiles (atomic adds into zeroed columns), else owner tiles
    DevBuf<BatchPipeItem> items;   // the kind's items, largest columns first
    DevBuf<int32_t> units;         // (item, tile) pairs
    DevBuf<const double*> ptrs;    // per item, inputs (f, w) then outputs (b, g)
    DevBuf<ZeroUnit> zero;         // shared tiles: the columns to zero before the walk
    DevBuf<int32_t> zstarts;       // ... their column starts
    int32_t n_units = 0, tile = 0, S = 0, cstride = 0, n_zero = 0, zero_out = 0;
    size_t lds = 0;
};

}  // namespace exm

using namespace exm;

struct exm_batch {
    int device = 0;
    hipStream_t cap = nullptr;
    hipStream_t side = nullptr;     // the DG0 items' branch
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf<BatchItemDev> items;
    DevBuf<Unit> units;
    DevBuf<int32_t> counter;
    DevBuf<const double*> ptrs;   // all field pointer arrays, item by item
    int64_t n_units = 0;
    int64_t n_units_p1 = 0;       // the P1 units come first in `units` (none when P1 is on tiles)
    TileSet tiles[2];             // P1 items, DG0 items on tiles (else work units)
    int32_t n_blocks = 0;
    int32_t unit_cells = 0;
    std::vector<int32_t> cpw;     // per item
    std::vector<bool> p1;         // per item: P1 x P1 (vertex units), else DG0 x DG0 (cell units)
    ~exm_batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (side) (void)hipStreamDestroy(side);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

int32_t batch_cpw(int32_t n_layers)
{
    // the cols_per_wave of the DIRECT schedule with the best lane use (<= 4)
    int32_t best = 1;
    double bu = 0.0;
    for (int32_t c = 1; c <= 4; ++c) {
        const int32_t seg = 64 / c;
        const int64_t steps = (n_layers + seg - 1) / seg;
        const double u = (double)c * n_layers / (64.0 * (double)steps);
        if (u > bu + 1e-9) {
            bu = u;
            best = c;
        }
    }
    return best;
}

// The items of one kind (P1: owner tiles, or shared tiles with `shared`;
// DG0: tiles) on tiles of about T cells with S-layer chunks: the item table,
// the units and the pass pointers (and for shared P1 tiles the columns to
// zero).  *fits stays false (and the set is left as it was) when some item's
// tiles exceed the kernel's limits or its pointers are not 16-byte aligned
// where the tile walk copies 16 bytes at a time.
int32_t build_tiles(exm_batch* B, bool p1, int32_t n_items, const exm_batch_item* items, int32_t T, int32_t S,
                    bool shared, bool* fits)
{
    shared = shared && p1;
    constexpr size_t kLds = 160 * 1024;
    const int32_t element = p1 ? EXM_ELEMENT_P1P1 : EXM_ELEMENT_DG0DG0;
    TileSet& ts = B->tiles[p1 ? 0 : 1];
    *fits = false;
    std::vector<int32_t> order;   // the kind's items, largest columns first
    for (int32_t m = 0; m < n_items; ++m)
        if (B->p1[m] == p1) order.push_back(m);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return items[a].space->mesh->n_layers > items[b].space->mesh->n_layers;
    });
    std::vector<const TilePlan*> plans;
    size_t lds = 0;
    int32_t cstride = 0;
    for (int32_t m : order) {
        const exm_batch_item& it = items[m];
        uintptr_t al = (uintptr_t)it.coords;
        if (p1)   // P1 fields are copied 16 bytes at a time too, at the coordinate field's column starts
            for (int32_t k = 0; k < it.n_fields; ++k) al |= (uintptr_t)it.f[k] | (it.w ? (uintptr_t)it.w[k] : 0);
        const bool same = !p1 || (!it.space->mixed && !it.coord_space->mixed &&
                                  it.space->base[0] == it.coord_space->base[0] &&
                                  it.space->col_size[0] == it.coord_space->col_size[0]);
        if ((al & 15) != 0 || !same) return EXM_OK;
        const TilePlan* plan = nullptr;
        int32_t s = p1 && !shared ? build_owner_plan(it.space->mesh, T, &plan)
                                  : build_tile_plan(it.space->mesh, T, &plan);
        if (s != EXM_OK) return s;
        const size_t l = pipe_lds_bytes(EXM_K_MASS, element, plan->max_verts, 0, plan->max_cells, S);
        if (plan->max_cells > pipe_max_tile_cells(EXM_K_MASS, element, S) ||
            (p1 && plan->max_verts > pipe_max_tile_verts(EXM_K_MASS, element, S)) || l > kLds)
            return EXM_OK;
        lds = std::max(lds, l);
        cstride = std::max(cstride, plan->max_cells);
        plans.push_back(plan);
    }
    std::vector<const double*> ptrs;
    std::vector<size_t> pbase;
    std::vector<int32_t> units;
    std::vector<int32_t> zstarts;
    std::vector<size_t> zbase;   // per item: its first entry in zstarts
    for (size_t i = 0; i < order.size(); ++i) {
        if (shared) {   // columns of the shared vertices and of those in no cell, in the P1 numbering
            const exm_batch_item& it = items[order[i]];
            zbase.push_back(zstarts.size());
            for (int32_t v : plans[i]->zero_verts)
                zstarts.push_back((int32_t)(it.space->base[0] + (int64_t)v * it.space->col_size[0]));
        }
        const exm_batch_item& it = items[order[i]];
        pbase.push_back(ptrs.size());
        for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.f[k]);
        if (it.w)
            for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.w[k]);
        for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.b[k]);
        if (it.g)
            for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.g[k]);
        for (int32_t k = 0; k < plans[i]->n_tiles; ++k) {
            units.push_back((int32_t)i);
            units.push_back(k);
        }
    }
    EXM_CHECK(units.size() / 2 < (size_t)INT32_MAX, EXM_EOVERFLOW, "too many tiles in the batch");
    int32_t s = ts.ptrs.upload(ptrs.data(), ptrs.size());
    if (s != EXM_OK) return s;
    std::vector<BatchPipeItem> dev(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
        const exm_batch_item& it = items[order[i]];
        const TilePlan* plan = plans[i];
        BatchPipeItem& d = dev[i];
        std::memset(&d, 0, sizeof(d));
        d.a.n_layers = it.space->mesh->n_layers;
        d.a.off = it.space->offsets[0];
        d.a.write = 1;
        d.a.xn = it.coord_space->n_dofs;
        d.a.fn = it.space->n_dofs;
        d.a.fmap = it.space->d_map.p;
        d.a.X = it.coords;
        d.t.vstride = plan->max_verts;
        d.t.tile_count = plan->n_tiles;
        d.t.cell_off = plan->cell_off.p;
        d.t.cells = plan->cells.p;
        d.t.vert_off = plan->vert_off.p;
        d.t.verts = plan->verts.p;
        d.t.lcv = plan->local_cv.p;
        d.t.owned = p1 && !shared ? plan->owned.p : nullptr;
        d.t.xstart = it.coord_space->d_starts[0].p;
        d.t.xbase = it.coord_space->base[0];
        d.t.xstep = it.coord_space->col_size[0];   // closed-form column starts: one layer count per mesh
        const int32_t np = it.w ? 2 * it.n_fields : it.n_fields;
        d.src = ts.ptrs.p + pbase[i];
        d.dst = (double* const*)(ts.ptrs.p + pbase[i] + np);
        d.n_pass = np;
    }
    if ((s = ts.items.upload(dev.data(), dev.size())) != EXM_OK) return s;
    if ((s = ts.units.upload(units.data(), units.size())) != EXM_OK) return s;
    ts.n_units = (int32_t)(units.size() / 2);
    ts.shared = shared;
    ts.n_zero = ts.zero_out = 0;
    if (shared) {   // zero units of up to 256 columns, every output of the item
        if (!zstarts.empty() && (s = ts.zstarts.upload(zstarts.data(), zstarts.size())) != EXM_OK) return s;
        std::vector<ZeroUnit> zu;
        for (size_t i = 0; i < order.size(); ++i) {
            const exm_batch_item& it = items[order[i]];
            const size_t b = zbase[i], e = i + 1 < order.size() ? zbase[i + 1] : zstarts.size();
            for (size_t k = b; k < e; k += 256)
                zu.push_back(ZeroUnit{dev[i].dst, ts.zstarts.p + k, dev[i].n_pass, (int32_t)std::min<size_t>(256, e - k),
                                      it.space->col_size[0]});
            ts.zero_out = std::max(ts.zero_out, dev[i].n_pass);
        }
        EXM_CHECK(zu.size() < (size_t)INT32_MAX, EXM_EOVERFLOW, "too many columns to zero");
        if (!zu.empty() && (s = ts.zero.upload(zu.data(), zu.size())) != EXM_OK) return s;
        ts.n_zero = (int32_t)zu.size();
    }
    ts.tile = T;
    ts.S = S;
    ts.cstride = cstride;
    ts.lds = lds;
    *fits = true;
    return EXM_OK;
}

int32_t launch_tiles(const TileSet& ts, bool p1, hipStream_t s)
{
    if (p1 && ts.shared) {
        const int32_t st = launch_zero_columns(ts.zero.p, ts.n_zero, ts.zero_out, s);
        if (st != EXM_OK) return st;
    }
    return p1 ? launch_batch_pipe_p1(ts.items.p, ts.units.p, ts.n_units, ts.S, ts.shared, ts.lds, s)
              : launch_batch_pipe_dg0(ts.items.p, ts.units.p, ts.n_units, ts.S, ts.cstride, ts.lds, s);
}

// The items of one kind: on tiles, or the persistent kernel over its units.
int32_t enqueue_kind(exm_batch* B, bool p1, hipStream_t s)
{
    if (B->tiles[p1 ? 0 : 1].on) return launch_tiles(B->tiles[p1 ? 0 : 1], p1, s);
    const int32_t n1 = (int32_t)B->n_units_p1, n0 = (int32_t)(B->n_units - B->n_units_p1);
    if (p1 && n1 > 0) {
        hipLaunchKernelGGL(k_batch<true>, dim3((unsigned)B->n_blocks), dim3(256), 0, s, B->items.p, B->units.p, n1,
                           B->counter.p);
        EXM_TRY_HIP(hipGetLastError());
    }
    if (!p1 && n0 > 0) {
        hipLaunchKernelGGL(k_batch<false>, dim3((unsigned)B->n_blocks), dim3(256), 0, s, B->items.p,
                           B->units.p + n1, n0, B->counter.p + 1);
        EXM_TRY_HIP(hipGetLastError());
    }
    return EXM_OK;
}

// The counter reset, then the P1 items on s and the DG0 items on a side
// stream forked after the reset and joined at the end (two branches of the
// graph), so that each kind's tail overlaps the other's work.
int32_t enqueue(exm_batch* B, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, B->counter.p);
    EXM_TRY_HIP(hipGetLastError());
    EXM_TRY_HIP(hipEventRecord(B->fork, s));
    EXM_TRY_HIP(hipStreamWaitEvent(B->side, B->fork, 0));
    int32_t st = enqueue_kind(B, true, s);
    if (st == EXM_OK) st = enqueue_kind(B, false, B->side);
    EXM_TRY_HIP(hipEventRecord(B->join, B->side));   // joined whatever happened, so a capture stays whole
    EXM_TRY_HIP(hipStreamWaitEvent(s, B->join, 0));
    return st;
}

int32_t build_units(exm_batch* B, const std::vector<int32_t>& n_cells, const std::vector<int32_t>& n_layers,
                    int32_t unit_cells)
{
    // units of about unit_cells entities (cells, or vertices for P1 items),
    // scaled so that every unit holds a similar number of layers in total
    // two lists, P1 units then DG0 units, each sorted largest first (that
    // keeps the tail of its kernel short)
    std::vector<Unit> lists[2];
    int64_t ref_layers = 64;
    for (size_t m = 0; m < n_cells.size(); ++m) {
        int64_t uc = std::max<int64_t>(1, unit_cells * ref_layers / std::max(1, n_layers[m]));
        uc = std::max<int64_t>(uc, B->cpw[m]);
        if (B->tiles[B->p1[m] ? 0 : 1].on) continue;   // on tiles
        std::vector<Unit>& units = lists[B->p1[m] ? 0 : 1];
        for (int64_t c = 0; c < n_cells[m]; c += uc)
            units.push_back(Unit{(int32_t)m, (int32_t)c, (int32_t)std::min<int64_t>(uc, n_cells[m] - c), 0});
    }
    for (std::vector<Unit>& units : lists)
        std::stable_sort(units.begin(), units.end(), [&](const Unit& a, const Unit& b) {
            return (int64_t)a.cell_count * n_layers[a.item] > (int64_t)b.cell_count * n_layers[b.item];
        });
    std::vector<Unit> units = lists[0];
    units.insert(units.end(), lists[1].begin(), lists[1].end());
    EXM_CHECK(units.size() < (size_t)INT32_MAX, EXM_EOVERFLOW, "too many work units");
    B->n_units = (int64_t)units.size();
    B->n_units_p1 = (int64_t)lists[0].size();
    B->unit_cells = unit_cells;
    return B->units.upload(units.data(), units.size());
}

}  // namespace

extern "C" {

int32_t exm_batch_create(int32_t n_items, const exm_batch_item* items, const exm_loop_opts* opts, void* stream,
                         exm_batch** out)
{
    clear_error();
    EXM_CHECK(out != nullptr, EXM_EINVAL, "out is NULL");
    *out = nullptr;
    EXM_CHECK(n_items >= 1 && items != nullptr, EXM_EINVAL, "need n_items >= 1 and an item array");
    EXM_CHECK(!opts || (opts->cols_per_wave >= 0 && opts->cols_per_wave <= 16), EXM_ERANGE,
              "cols_per_wave outside [0, 16]");
    EXM_CHECK(!opts || (opts->tile_cells >= 0 && opts->tile_cells <= 65536), EXM_ERANGE,
              "tile_cells (cells per work unit) outside [0, 65536]");
    auto B = std::make_unique<exm_batch>();
    EXM_TRY_HIP(hipGetDevice(&B->device));
    std::vector<BatchItemDev> dev(n_items);
    std::vector<const double*> ptrs;
    std::vector<int32_t> n_ent(n_items), n_layers(n_items);   // work entities (cells, or vertices for P1) per item
    std::vector<size_t> ptr_base(n_items);
    B->cpw.resize(n_items);
    B->p1.resize(n_items);
    for (int32_t m = 0; m < n_items; ++m) {
        const exm_batch_item& it = items[m];
        EXM_CHECK(it.space && it.coord_space && it.coords, EXM_EINVAL, "item %d: NULL space, coord_space or coords", m);
        EXM_CHECK(it.space->element == EXM_ELEMENT_P1P1 || it.space->element == EXM_ELEMENT_DG0DG0,
                  EXM_EUNSUPPORTED, "item %d: batched assembly supports P1xP1 and DG0xDG0 spaces", m);
        EXM_CHECK(!it.space->mesh->variable, EXM_EUNSUPPORTED,
                  "item %d: batches take meshes with one layer count per column", m);
        EXM_CHECK(it.coord_space->element == EXM_ELEMENT_P1P1 && it.coord_space->mesh == it.space->mesh, EXM_EINVAL,
                  "item %d: coord_space must be a P1xP1 space on the same mesh", m);
        EXM_CHECK(it.n_fields >= 1 && it.n_fields <= 64, EXM_ERANGE, "item %d: n_fields = %d outside [1, 64]", m,
                  it.n_fields);
        EXM_CHECK(it.f && it.b, EXM_EINVAL, "item %d: NULL f or b", m);
        EXM_CHECK((it.w == nullptr) == (it.g == nullptr), EXM_EINVAL, "item %d: w and g must both be given or both NULL",
                  m);
        for (int32_t k = 0; k < it.n_fields; ++k) {
            EXM_CHECK(it.f[k] && it.b[k], EXM_EINVAL, "item %d field %d: NULL pointer", m, k);
            EXM_CHECK(it.f[k] != it.b[k], EXM_EINVAL, "item %d field %d: b aliases f", m, k);
            if (it.w) {
                EXM_CHECK(it.w[k] && it.g[k], EXM_EINVAL, "item %d field %d: NULL pointer", m, k);
                EXM_CHECK(it.g[k] != it.b[k] && it.g[k] != it.w[k] && it.g[k] != it.f[k], EXM_EINVAL,
                          "item %d field %d: g aliases another field", m, k);
            }
        }
        int32_t vs = ensure_vertical(it.coord_space, it.coords, (hipStream_t)stream);
        if (vs != EXM_OK) return vs;
        const exm_mesh* mesh = it.space->mesh;
        const bool p1 = it.space->element == EXM_ELEMENT_P1P1;
        B->p1[m] = p1;
        n_ent[m] = p1 ? mesh->n[0] : mesh->n[2];
        n_layers[m] = mesh->n_layers;
        B->cpw[m] = opts && opts->cols_per_wave ? opts->cols_per_wave : batch_cpw(mesh->n_layers);
        BatchItemDev& d = dev[m];
        std::memset(&d, 0, sizeof(d));
        d.element = it.space->element;
        d.n_layers = mesh->n_layers;
        d.off = it.space->offsets[0];
        d.cpw = B->cpw[m];
        d.seg = 64 / d.cpw;
        d.n_fields = it.n_fields;
        d.adjoint = it.w ? 1 : 0;
        d.xn = it.coord_space->n_dofs;
        if (p1) {
            const VertexFans* fans = nullptr;
            int32_t st = build_vertex_fans(mesh, &fans);
            if (st != EXM_OK) return st;
            d.fan_off = fans->off.p;
            d.fan = fans->fan.p;
            d.fbase = it.space->base[0];
            d.xbase = it.coord_space->base[0];
        }
        d.fmap = it.space->d_map.p;
        d.xmap = it.coord_space->d_map.p;
        d.X = it.coords;
        ptr_base[m] = ptrs.size();
        for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.f[k]);
        for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.b[k]);
        if (it.w) {
            for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.w[k]);
            for (int32_t k = 0; k < it.n_fields; ++k) ptrs.push_back(it.g[k]);
        }
    }
    // Every output must be its own memory: no two outputs of any items may
    // overlap, and no output may overlap any input (fields, cotangents or
    // coordinates of any item), since tiles read neighbouring input columns
    // while other tiles store outputs.
    {
        struct Range { uintptr_t lo, hi; int32_t item; };
        std::vector<Range> outs, ins;
        for (int32_t m = 0; m < n_items; ++m) {
            const exm_batch_item& it = items[m];
            const uintptr_t bytes = (uintptr_t)it.space->n_dofs * sizeof(double);
            for (int32_t k = 0; k < it.n_fields; ++k) {
                outs.push_back({(uintptr_t)it.b[k], (uintptr_t)it.b[k] + bytes, m});
                ins.push_back({(uintptr_t)it.f[k], (uintptr_t)it.f[k] + bytes, m});
                if (it.w) {
                    outs.push_back({(uintptr_t)it.g[k], (uintptr_t)it.g[k] + bytes, m});
                    ins.push_back({(uintptr_t)it.w[k], (uintptr_t)it.w[k] + bytes, m});
                }
            }
            const uintptr_t xb = (uintptr_t)it.coord_space->n_dofs * 3 * sizeof(double);
            ins.push_back({(uintptr_t)it.coords, (uintptr_t)it.coords + xb, m});
        }
        std::sort(outs.begin(), outs.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
        for (size_t i = 1; i < outs.size(); ++i)
            EXM_CHECK(outs[i].lo >= outs[i - 1].hi, EXM_EINVAL, "outputs of items %d and %d overlap",
                      outs[i - 1].item, outs[i].item);
        for (const Range& r : ins) {
            // the first output ending after r.lo is the only candidate that can overlap r
            auto it = std::upper_bound(outs.begin(), outs.end(), r.lo,
                                       [](uintptr_t v, const Range& o) { return v < o.lo; });
            if (it != outs.begin()) {
                auto prev = std::prev(it);
                EXM_CHECK(prev->hi <= r.lo, EXM_EINVAL, "an output of item %d overlaps an input of item %d",
                          prev->item, r.item);
            }
            EXM_CHECK(it == outs.end() || it->lo >= r.hi, EXM_EINVAL,
                      "an output of item %d overlaps an input of item %d", it->item, r.item);
        }
    }
    int32_t s = B->ptrs.upload(ptrs.data(), ptrs.size());
    if (s != EXM_OK) return s;
    for (int32_t m = 0; m < n_items; ++m) {
        const double** p = B->ptrs.p + ptr_base[m];
        const int32_t nf = items[m].n_fields;
        dev[m].f = p;
        dev[m].b = (double* const*)(p + nf);
        if (items[m].w) {
            dev[m].w = p + 2 * nf;
            dev[m].g = (double* const*)(p + 3 * nf);
        }
    }
    if ((s = B->items.upload(dev.data(), dev.size())) != EXM_OK) return s;
    if ((s = B->counter.alloc(2)) != EXM_OK) return s;
    int cus = 0;
    EXM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
    B->n_blocks = std::max(1, cus) * 8;
    hipStream_t hs = (hipStream_t)stream;
    EXM_TRY_HIP(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
    EXM_TRY_HIP(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
    EXM_TRY_HIP(hipEventCreateWithFlags(&B->join, hipEventDisableTiming));
    // each kind on tiles unless GATHER is asked for: tile size and chunk
    // length timed on these buffers (the first that fits when the unit size
    // is given); work units where none fits
    for (int kind = 0; kind < 2 && !(opts && opts->schedule == EXM_SCHED_GATHER); ++kind) {
        const bool p1 = kind == 0;
        if (std::find(B->p1.begin(), B->p1.end(), p1) == B->p1.end()) continue;
        // (tile cells, chunk layers, shared tiles): P1 on owner tiles and on
        // shared tiles (race EXM_RACE_OWNER or EXM_RACE_ATOMIC picks one)
        struct Cand {
            int32_t T, S;
            bool shared;
        };
        std::vector<Cand> cand;
        if (p1) {
            const int32_t race = opts ? opts->race : 0;
            for (bool sh : {false, true}) {
                if ((race == EXM_RACE_ATOMIC && !sh) || (race == EXM_RACE_OWNER && sh)) continue;
                for (const auto& c : {std::make_pair(64, 16), std::make_pair(32, 16), std::make_pair(64, 8),
                                      std::make_pair(128, 8)})
                    cand.push_back(Cand{c.first, c.second, sh});
            }
        } else {
            for (const auto& c : {std::make_pair(32, 32), std::make_pair(30, 34), std::make_pair(32, 16),
                                  std::make_pair(64, 16), std::make_pair(64, 8)})
                cand.push_back(Cand{c.first, c.second, false});
        }
        const bool tune = !(opts && opts->tile_cells);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (tune) {
            EXM_TRY_HIP(hipEventCreate(&e0));
            EXM_TRY_HIP(hipEventCreate(&e1));
        }
        auto time_one = [&](float* ms) -> int32_t {   // one warm launch, one timed
            int32_t st = launch_tiles(B->tiles[kind], p1, hs);
            if (st != EXM_OK) return st;
            EXM_TRY_HIP(hipEventRecord(e0, hs));
            if ((st = launch_tiles(B->tiles[kind], p1, hs)) != EXM_OK) return st;
            EXM_TRY_HIP(hipEventRecord(e1, hs));
            EXM_TRY_HIP(hipEventSynchronize(e1));
            EXM_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
            return EXM_OK;
        };
        float best = 1e30f;
        int32_t bt = 0, bs = 0;
        bool bsh = false;
        for (const Cand& c : cand) {
            if (opts && opts->chunk_layers && opts->chunk_layers != c.S) continue;
            bool fits = false;
            if ((s = build_tiles(B.get(), p1, n_items, items, c.T, c.S, c.shared, &fits)) != EXM_OK) break;
            if (!fits) continue;
            if (!tune) {
                bt = c.T;
                bs = c.S;
                bsh = c.shared;
                break;
            }
            float ms = 0.f;
            if ((s = time_one(&ms)) != EXM_OK) break;
            if (ms < best) {
                best = ms;
                bt = c.T;
                bs = c.S;
                bsh = c.shared;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s != EXM_OK) return s;
        if (bt) {
            bool fits = false;
            if ((s = build_tiles(B.get(), p1, n_items, items, bt, bs, bsh, &fits)) != EXM_OK) return s;
            B->tiles[kind].on = fits;
        }
    }
    if (opts && opts->tile_cells) {
        if ((s = build_units(B.get(), n_ent, n_layers, opts->tile_cells)) != EXM_OK) return s;
    } else {
        // project autotuner: time the candidate unit sizes on these buffers
        // (the launch overwrites every output, so timing runs are harmless)
        hipEvent_t e0, e1;
        EXM_TRY_HIP(hipEventCreate(&e0));
        EXM_TRY_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        int32_t best_uc = 64;
        for (int32_t uc : {16, 64, 256}) {
            if ((s = build_units(B.get(), n_ent, n_layers, uc)) != EXM_OK) break;
            if ((s = enqueue(B.get(), hs)) != EXM_OK) break;
            EXM_TRY_HIP(hipEventRecord(e0, hs));
            if ((s = enqueue(B.get(), hs)) != EXM_OK) break;
            EXM_TRY_HIP(hipEventRecord(e1, hs));
            EXM_TRY_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            EXM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_uc = uc;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (s != EXM_OK) return s;
        if ((s = build_units(B.get(), n_ent, n_layers, best_uc)) != EXM_OK) return s;
    }
    // capture the counter reset and the two kinds' launches into a graph on a private stream
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    EXM_TRY_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    EXM_TRY_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
    s = enqueue(B.get(), B->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap, &g);
    if (s != EXM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return fail(EXM_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    B->graph = g;
    EXM_TRY_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    *out = B.release();
    return EXM_OK;
}

int32_t exm_batch_launch(exm_batch* batch, void* stream)
{
    clear_error();
    EXM_CHECK(batch != nullptr, EXM_EINVAL, "batch is NULL");
    int32_t s = check_pending();
    if (s != EXM_OK) return s;
    EXM_TRY_HIP(hipGraphLaunch(batch->exec, (hipStream_t)stream));
    return EXM_OK;
}

int32_t exm_batch_info(const exm_batch* batch, int64_t* n_units, int32_t* n_blocks)
{
    clear_error();
    EXM_CHECK(batch != nullptr, EXM_EINVAL, "batch is NULL");
    if (n_units) *n_units = batch->n_units;
    if (n_blocks) *n_blocks = batch->n_blocks;
    return EXM_OK;
}

int32_t exm_batch_tiles(const exm_batch* batch, int32_t element, int32_t* tile_cells, int32_t* chunk_layers)
{
    clear_error();
    EXM_CHECK(batch != nullptr, EXM_EINVAL, "batch is NULL");
    EXM_CHECK(element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_DG0DG0, EXM_EINVAL,
              "element must be EXM_ELEMENT_P1P1 or EXM_ELEMENT_DG0DG0");
    const TileSet& ts = batch->tiles[element == EXM_ELEMENT_P1P1 ? 0 : 1];
    if (tile_cells) *tile_cells = ts.on ? ts.tile : 0;
    if (chunk_layers) *chunk_layers = ts.on ? ts.S : 0;
    return EXM_OK;
}

void exm_batch_destroy(exm_batch* batch) { delete batch; }

}  // extern "C"
