// Internal declarations shared by the translation units of libexm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "exm.h"

namespace exm {

// ---------------------------------------------------------------------------
// Errors: a thread-local message plus the status code.

int32_t fail(int32_t code, const char* fmt, ...);
void clear_error();

#define EXM_TRY_HIP(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::exm::fail(EXM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define EXM_CHECK(cond, code, ...)                   \
    do {                                             \
        if (!(cond)) return ::exm::fail(code, __VA_ARGS__); \
    } while (0)

// Report an error from an earlier asynchronous launch, if any.
int32_t check_pending();

// ---------------------------------------------------------------------------
// Device buffers owned by the library.

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    int32_t alloc(size_t count) {
        reset();
        if (count == 0) return EXM_OK;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return fail(EXM_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
        }
        n = count;
        return EXM_OK;
    }
    int32_t upload(const T* host, size_t count) {
        int32_t s = alloc(count);
        if (s != EXM_OK) return s;
        if (count) EXM_TRY_HIP(hipMemcpy(p, host, count * sizeof(T), hipMemcpyHostToDevice));
        return EXM_OK;
    }
};

// ---------------------------------------------------------------------------
// Colouring of the base cells: no two cells of one colour share a vertex.

struct Colouring {
    int32_t n_colours = 0;
    std::vector<int64_t> offsets;   // [n_colours + 1] into cells
    DevBuf<int32_t> cells;          // cells grouped by colour, ascending within a colour
    std::vector<int32_t> host_cells;
};

// Tiles of compact groups of base cells for the LDS-staged column loop.
struct TilePlan {
    int32_t target = 0;          // requested cells per tile
    bool owner = false;          // owner plan: tiles own vertices, cells may repeat across tiles
    int32_t n_tiles = 0;
    int32_t max_cells = 0, max_verts = 0, max_edges = 0;
    int64_t n_tile_verts = 0;    // sum over tiles of their vertex counts
    int64_t n_shared_verts = 0;  // ... of which also touched by another tile
    bool has_edges = false;
    DevBuf<int32_t> cell_off;    // [n_tiles + 1] into cells / local_cv / local_ce
    DevBuf<int32_t> cells;       // base cells, tile by tile
    DevBuf<int32_t> vert_off;    // [n_tiles + 1] into verts
    DevBuf<int32_t> verts;       // base vertex ids; bit 31 set when shared with another tile
    DevBuf<int32_t> edge_off;    // [n_tiles + 1] into edges
    DevBuf<int32_t> edges;       // base edge ids; bit 31 set when shared
    DevBuf<uint16_t> local_cv;   // [n_cells * 3] tile-local vertex index of each cell vertex
    DevBuf<uint16_t> local_ce;   // [n_cells * 3] tile-local edge index of each cell edge
    int32_t n_colours = 0;
    std::vector<int64_t> colour_off;   // [n_colours + 1] into colour_tiles
    DevBuf<int32_t> colour_tiles;      // tiles grouped by colour
    DevBuf<int32_t> owned;             // owner plan: [n_tiles] vertices owned (the first of each vertex list)
    int64_t n_cell_entries = 0;        // owner plan: cells summed over tiles (>= n_cells)
    std::vector<int32_t> zero_verts;   // tile plan: the base vertices no single tile writes alone: touched
                                       // by more than one tile, or by none (host)
};

// Fans of base cells around every vertex (the GATHER schedule).
struct VertexFans {
    DevBuf<int32_t> off;   // [n_vertices + 1]
    DevBuf<int32_t> fan;   // neighbouring vertices in fan order; bit 31 flags the start of a fan
    DevBuf<int32_t> cell;  // the cell between an entry and the one before it (-1 at the start of a fan)
    int64_t n_entries = 0;
};

}  // namespace exm

struct exm_mesh {
    int32_t n[3] = {0, 0, 0};      // N_0, N_1, N_2
    int32_t n_layers = 0;          // the largest layer count (all of them unless `variable`)
    int device = 0;
    bool variable = false;         // each cell column has its own layer range
    std::vector<int32_t> lo[3], hi[3];   // variable: layer range [lo, hi) of every entity column
    exm::DevBuf<int32_t> d_cell_lam;     // variable: layers of every cell column
    exm::DevBuf<int32_t> d_cell_lo;      // variable: first layer of every cell column
    exm::DevBuf<int32_t> d_vert_lo, d_vert_hi;   // variable: level range of every vertex column
    exm::DevBuf<int32_t> d_edge_lo, d_edge_hi;   // variable: ... of every edge column
    exm::DevBuf<int32_t> d_cell_hi;              // variable: last layer + 1 of every cell column
    std::vector<int32_t> h_cell_vertex, h_cell_edge;
    exm::DevBuf<int32_t> d_cell_vertex, d_cell_edge;
    mutable std::mutex mu;
    mutable std::unique_ptr<exm::Colouring> colouring;   // built on first use
    mutable std::vector<std::unique_ptr<exm::TilePlan>> plans;
    mutable std::unique_ptr<exm::VertexFans> fans;        // built on first use
};

struct exm_space {
    const exm_mesh* mesh = nullptr;
    int32_t delta[6] = {0, 0, 0, 0, 0, 0};
    int32_t element = EXM_ELEMENT_NONE;
    int64_t n_dofs = 0;
    int32_t k = 0;
    int32_t col_size[3] = {0, 0, 0};   // DoFs in one column of a base entity of dimension d
    int64_t base[3] = {0, 0, 0};       // first DoF of the first column of dimension d
    std::vector<int32_t> offsets;      // [k], Algorithm 2
    std::vector<int32_t> entity_dim;   // [k]
    exm::DevBuf<int32_t> d_map;        // [n_cells * k], explicit lists of layer 0
    exm::DevBuf<int32_t> d_starts[3];  // column start of every base entity (-1: no column)
    // a DoF count per entity: lists of different lengths (d_map holds them
    // back to back), the start of every cell's list and the vertical offset
    // of every entry
    bool mixed = false;
    int64_t list_total = 0;
    exm::DevBuf<int32_t> d_list_off;   // [n_cells + 1]
    exm::DevBuf<int32_t> d_entry_off;  // [list_total]
    // a coordinate (P1xP1) space: addresses of fields found to have vertical
    // columns, and the device flag of that check
    mutable std::mutex coords_mu;
    mutable std::vector<const void*> coords_ok;
    mutable exm::DevBuf<int32_t> coords_flag;
};

namespace exm {

int32_t build_colouring(const exm_mesh* m, const Colouring** out);
int32_t build_tile_plan(const exm_mesh* m, int32_t target, const TilePlan** out);
int32_t build_owner_plan(const exm_mesh* m, int32_t target, const TilePlan** out);
int32_t build_vertex_fans(const exm_mesh* m, const VertexFans** out);

// Work decomposition of the column loop.
struct LoopShape {
    int32_t cpw;     // base-cell columns per wavefront
    int32_t seg;     // lanes (layers per step) per column
    int32_t wpb;     // wavefronts per workgroup
};

LoopShape default_shape(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells);
LoopShape shape_from_opts(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells,
                          const exm_loop_opts* opts);
int32_t lookup_tuned(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells, exm_loop_opts* out);

// Launch the column loop of one element kernel (validated arguments).
struct LoopLaunch {
    const exm_space* fspace;      // field space
    const exm_space* xspace;      // coordinate space
    int32_t kernel;
    int32_t element;
    int32_t race;
    LoopShape shape;
    int32_t n_layers;
    const int32_t* cell_lam;      // layers of every cell column, or null (all n_layers)
    const int32_t* list_off;      // a space with a DoF count per entity: start of every cell's list, else null
    int32_t field_offset;         // vertical offset of every position of the field space
    const int32_t* fmap;          // field explicit lists [n_cells * k]
    const int32_t* xmap;          // coordinate explicit lists [n_cells * 6]
    const double* X;              // coordinates [n * 3]
    const double* in[3];
    double* out[3];
    int32_t write;                // 1 WRITE, 0 INC
    int32_t n_cells;              // total base cells
    const int32_t* cells;         // cell list (colour mode) or null
    int64_t cell_begin, cell_count;  // range of the list (or of cells) handled by this launch
};
int32_t launch_column_loop(const LoopLaunch& L, hipStream_t stream);

// EXM_OK when the coordinate field X on `space` is known to have vertical
// columns (x, y constant along every vertex column); otherwise checks it on
// `stream` (synchronising it) and remembers the address if it passes.
// EXM_EUNSUPPORTED for a leaning column; EXM_EINVAL if the check would be
// needed while `stream` is being captured.
int32_t ensure_vertical(const exm_space* space, const void* X, hipStream_t stream);

}  // namespace exm
