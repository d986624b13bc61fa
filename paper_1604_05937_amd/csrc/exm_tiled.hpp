// Kernel arguments and launchers of the column loop (DIRECT and TILED schedules).
#pragma once

#include "exm_internal.hpp"

namespace exm {

// Arguments shared by every column-loop kernel.
struct ColArgs {
    int32_t n_layers;
    int32_t off;           // vertical offset of the field space (same for every list position)
    int32_t cpw, seg;      // columns per wavefront, lanes (layers per step) per column
    int32_t write;         // DG outputs: 1 WRITE, 0 INC
    int64_t xn;            // DoFs of the coordinate space (component stride of X)
    int64_t fn;            // DoFs of the field space (length of every field array)
    const int32_t* __restrict__ fmap;   // field explicit lists [n_cells * k]
    const int32_t* __restrict__ xmap;   // coordinate explicit lists [n_cells * 6]
    const double* __restrict__ X;       // coordinates, component-major [3 * xn]
    const double* __restrict__ in0;
    const double* __restrict__ in1;
    const double* __restrict__ in2;
    double* __restrict__ out0;
    double* __restrict__ out1;
    double* __restrict__ out2;
    const int32_t* __restrict__ cell_lam;   // layers of every cell column (a mesh with a range per column) or null
    const int32_t* __restrict__ list_off;   // start of every cell's list (a DoF count per entity) or null
    const int32_t* __restrict__ cells;  // DIRECT: cell list (one colour) or null
    int64_t cell_begin, cell_count;     // DIRECT: range of the list (or of the cells)
};

// TILED: the tile plan.
struct TileArgs {
    int32_t vstride;       // LDS entity slots for vertices (the plan's max_verts)
    int32_t estride;       // LDS entity slots for edges (the plan's max_edges)
    const int32_t* __restrict__ tiles;   // tile list (one colour) or null for tiles tile_begin ..
    int32_t tile_begin, tile_count;
    const int32_t* __restrict__ cell_off;
    const int32_t* __restrict__ cells;
    const int32_t* __restrict__ vert_off;
    const int32_t* __restrict__ verts;
    const int32_t* __restrict__ edge_off;
    const int32_t* __restrict__ edges;
    const uint16_t* __restrict__ lcv;
    const uint16_t* __restrict__ lce;
    const int32_t* __restrict__ xstart;    // coordinate column start of every base vertex
    const int32_t* __restrict__ fstart0;   // field column start of every base vertex
    const int32_t* __restrict__ fstart1;   // field column start of every base edge
    const int32_t* __restrict__ owned;     // owner plan: vertices each tile owns (else null)
    // Uniform meshes: the column starts in the closed form of Algorithm 1,
    // base + id * step, so that a kernel need not read the tables above
    // (step 0: read them).  Coordinate vertex columns, field vertex and edge columns.
    int64_t xbase, fbase0, fbase1;
    int32_t xstep, fstep0, fstep1;
    // a mesh with a layer range per cell column (else null): level range of
    // every base vertex, first layer of every base cell
    const int32_t* __restrict__ vlo;
    const int32_t* __restrict__ vhi;
    const int32_t* __restrict__ clo;
};

// Column start of entity `id` from its table or, on uniform meshes, in closed form.
__device__ __forceinline__ int32_t column_start(const int32_t* __restrict__ table, int64_t base, int32_t step,
                                                int32_t id)
{
    return step > 0 ? (int32_t)(base + (int64_t)id * step) : table[id];
}

// One item of a batch on tiles (P1 x P1: owner tiles; DG0 x DG0): lists,
// coordinates and layer count (a), its tile plan (t), and the input and
// output of every pass (forward fields, then adjoint ones).
struct BatchPipeItem {
    ColArgs a;
    TileArgs t;
    const double* const* src;
    double* const* dst;
    int32_t n_pass;
};
// shared: the items' tiles are shared tiles (shared vertices added
// atomically into zeroed columns), else owner tiles.
int32_t launch_batch_pipe_p1(const BatchPipeItem* items, const int32_t* units, int32_t n_units, int32_t S,
                             bool shared, size_t lds, hipStream_t s);

// A range of vertex columns to zero in every output of a batch item: column
// starts starts[0 .. count), len values each, in the n_out arrays dst.
struct ZeroUnit {
    double* const* dst;
    const int32_t* starts;
    int32_t n_out, count, len;
};
// max_out: the most outputs of any unit's item.
int32_t launch_zero_columns(const ZeroUnit* units, int32_t n_units, int32_t max_out, hipStream_t s);
// cstride: the largest tile of the DG0 items (cells).
int32_t launch_batch_pipe_dg0(const BatchPipeItem* items, const int32_t* units, int32_t n_units, int32_t S,
                              int32_t cstride, size_t lds, hipStream_t s);

ColArgs col_args(const LoopLaunch& P);
int32_t tiled_max_threads(int32_t kernel, int32_t element);
size_t staged_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t S);
bool staged_supported(int32_t kernel, int32_t element);
int32_t staged_max_tile_cells(int32_t S);
int32_t launch_staged(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t S, size_t lds, hipStream_t s);
size_t pipe_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t estride, int32_t cstride, int32_t S);
bool pipe_supported(int32_t kernel, int32_t element);
int32_t pipe_max_tile_cells(int32_t kernel, int32_t element, int32_t S);
int32_t pipe_max_tile_verts(int32_t kernel, int32_t element, int32_t S);
int32_t pipe_p1_wide_max_cells(int32_t S);
int32_t pipe_p1_wide_max_verts(int32_t S);
int32_t pipe_max_tile_entities(int32_t S);
bool pipe_chunk_ok(int32_t kernel, int32_t element, int32_t S);
// Chunk lengths the DG0 x DG0 tile walk takes beside 8, 16 and 32 on columns
// of one height (one layer per thread, so any even length): 20, 26 and 34
// layers cover 20, 50 and 100 layers in one, two and three chunk steps.
inline bool dg0_long_chunk(int32_t S) { return S == 20 || S == 26 || S == 34; }
int32_t launch_pipe(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t cstride, int32_t S, size_t lds,
                    hipStream_t s);
size_t chunk_lds_bytes(int32_t vstride, int32_t S);
int32_t chunk_count(int32_t n_layers, int32_t S);
int32_t launch_chunked(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t S, size_t lds, hipStream_t s);
bool gather_supported(int32_t kernel, int32_t element);
int32_t launch_gather(const LoopLaunch& P, const VertexFans* fans, int32_t wpb, hipStream_t s);
size_t tiled_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t estride, int32_t seg);
int32_t launch_tiled(const LoopLaunch& P, const TileArgs& t, int32_t threads, size_t lds, hipStream_t s);

}  // namespace exm
