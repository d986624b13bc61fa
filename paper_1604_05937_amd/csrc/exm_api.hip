// exm_par_loop: argument validation, schedule and race-strategy selection,
// and the autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>

#include "exm_internal.hpp"
#include "exm_tiled.hpp"

namespace exm {

// Largest LDS a workgroup may use; a chunk is shrunk until its staging fits.
static constexpr size_t kLdsLimit = 160 * 1024;
// Default LDS budget: two tile workgroups per compute unit.
static constexpr size_t kLdsDefault = 64 * 1024;

// ---------------------------------------------------------------------------
// DIRECT schedule shapes.  cols_per_wave = cpw columns share a wavefront; each
// gets seg = 64 / cpw lanes.  A column of lambda layers takes ceil(lambda /
// seg) steps, so the fraction of busy lanes is cpw lambda / (64 ceil(lambda / seg)).

static LoopShape make_shape(int32_t cpw, int32_t wpb)
{
    LoopShape s;
    s.cpw = std::max(1, std::min(cpw, 64));
    s.seg = 64 / s.cpw;
    s.wpb = std::max(1, std::min(wpb, 4));
    return s;
}

static double lane_use(int32_t cpw, int32_t lam)
{
    const int32_t seg = 64 / cpw;
    const int64_t steps = (lam + seg - 1) / seg;
    return (double)cpw * lam / (64.0 * (double)steps);
}

LoopShape default_shape(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells)
{
    (void)kernel;
    (void)element;
    (void)n_cells;
    // Wider lane groups per column keep accesses coalesced: at most four
    // columns per wavefront (16 lanes = 128 bytes of FP64 per column).
    int32_t best = 1;
    double bu = lane_use(1, n_layers);
    for (int32_t c = 2; c <= 4; ++c) {
        const double u = lane_use(c, n_layers);
        if (u > bu + 1e-9) {
            bu = u;
            best = c;
        }
    }
    return make_shape(best, 4);
}

// Tuned table: key (kernel, element, n_layers, log2 bucket of the cell count).
using TuneKey = std::tuple<int32_t, int32_t, int32_t, int32_t>;
static std::mutex g_tune_mu;
static std::map<TuneKey, exm_loop_opts> g_tuned;

static TuneKey tune_key(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells)
{
    int32_t b = 0;
    while ((int64_t(1) << (b + 1)) <= n_cells) ++b;
    return TuneKey(kernel, element, n_layers, b);
}

int32_t lookup_tuned(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells, exm_loop_opts* out)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(tune_key(kernel, element, n_layers, n_cells));
    if (it == g_tuned.end()) return 0;
    *out = it->second;
    return 1;
}

LoopShape shape_from_opts(int32_t kernel, int32_t element, int32_t n_layers, int64_t n_cells,
                          const exm_loop_opts* opts)
{
    LoopShape s = default_shape(kernel, element, n_layers, n_cells);
    if (opts && opts->cols_per_wave > 0) s = make_shape(opts->cols_per_wave, s.wpb);
    if (opts && opts->waves_per_block > 0) s = make_shape(s.cpw, opts->waves_per_block);
    return s;
}

// ---------------------------------------------------------------------------
// Argument signatures of the element kernels.

struct Signature {
    int32_t n_in, n_out;
};

static bool signature(int32_t kernel, Signature& s)
{
    switch (kernel) {
    case EXM_K_MASS: s = {1, 1}; return true;
    case EXM_K_CUBIC: s = {2, 1}; return true;
    case EXM_K_CUBIC_VJP: s = {2, 2}; return true;
    case EXM_K_CUBIC_FUSED: s = {3, 3}; return true;
    case EXM_K_FACET_JUMP: s = {1, 1}; return true;
    default: return false;
    }
}

// DoFs shared between cells (horizontally) or between layers (vertically)
static bool continuous(int32_t element)
{
    return element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_P2P2 || element == EXM_ELEMENT_P1DG0 ||
           element == EXM_ELEMENT_P1DG1 || element == EXM_ELEMENT_DG0P1 || element == EXM_ELEMENT_DG1P1;
}

// The tensor-product elements that run the generic DIRECT kernel only
static bool direct_only(int32_t element) { return element >= EXM_ELEMENT_P1DG0 && element <= EXM_ELEMENT_DGMIX; }

// Validate and fill everything but the schedule.
static int32_t prepare(int32_t kernel, const exm_mesh* m, int32_t nargs, const exm_arg* args, LoopLaunch& P)
{
    Signature sig;
    EXM_CHECK(signature(kernel, sig), EXM_EINVAL, "unknown kernel %d", kernel);
    EXM_CHECK(m != nullptr, EXM_EINVAL, "iterset is NULL");
    EXM_CHECK(args != nullptr, EXM_EINVAL, "args is NULL");
    EXM_CHECK(nargs == 1 + sig.n_in + sig.n_out, EXM_EINVAL, "kernel %d takes %d args, got %d", kernel,
              1 + sig.n_in + sig.n_out, nargs);
    const exm_arg& X = args[0];
    EXM_CHECK(X.space != nullptr && X.data != nullptr, EXM_EINVAL, "args[0] (coordinates) has a NULL space or data");
    EXM_CHECK(X.space->mesh == m, EXM_EINVAL, "coordinate space is on another mesh");
    EXM_CHECK(X.space->element == EXM_ELEMENT_P1P1, EXM_EINVAL, "coordinates must live on a P1xP1 space");
    EXM_CHECK(X.dim == 3, EXM_EINVAL, "coordinates must have dim 3 (got %d)", X.dim);
    EXM_CHECK(X.access == EXM_READ, EXM_EINVAL, "coordinates must be EXM_READ");
    const exm_space* V = args[1].space;
    EXM_CHECK(V != nullptr, EXM_EINVAL, "args[1] has a NULL space");
    EXM_CHECK(V->mesh == m, EXM_EINVAL, "field space is on another mesh");
    const int32_t el = V->element;
    EXM_CHECK(el != EXM_ELEMENT_NONE, EXM_EINVAL, "field space has no element");
    if (kernel == EXM_K_FACET_JUMP) {
        EXM_CHECK(el == EXM_ELEMENT_DG0DG0 || el == EXM_ELEMENT_DG1DG1 || el == EXM_ELEMENT_DG0DG1 ||
                      el == EXM_ELEMENT_DG1DG0 || el == EXM_ELEMENT_P1DG0 || el == EXM_ELEMENT_P1DG1,
                  EXM_EUNSUPPORTED, "the facet jump needs a space discontinuous across levels (element %d)", el);
        EXM_CHECK(!m->variable, EXM_EUNSUPPORTED, "the facet loop takes meshes with one layer count per column");
    } else if (kernel != EXM_K_MASS) {
        EXM_CHECK(el == EXM_ELEMENT_P1P1, EXM_EUNSUPPORTED, "kernel %d is implemented for P1xP1 only", kernel);
    }
    int32_t write = -1;
    for (int i = 1; i < nargs; ++i) {
        const exm_arg& A = args[i];
        const bool is_out = i > sig.n_in;
        EXM_CHECK(A.data != nullptr, EXM_EINVAL, "args[%d].data is NULL", i);
        EXM_CHECK(A.space != nullptr && A.space->mesh == m && A.space->element == el, EXM_EINVAL,
                  "args[%d] is not on the same space as args[1]", i);
        EXM_CHECK(A.dim == 1, EXM_EUNSUPPORTED, "args[%d].dim = %d: fields must be scalar", i, A.dim);
        if (!is_out) {
            EXM_CHECK(A.access == EXM_READ, EXM_EINVAL, "args[%d] must be EXM_READ", i);
        } else {
            EXM_CHECK(A.access == EXM_INC || A.access == EXM_WRITE, EXM_EINVAL, "args[%d] must be EXM_INC or EXM_WRITE",
                      i);
            if (A.access == EXM_WRITE)
                EXM_CHECK(!continuous(el), EXM_EINVAL,
                          "args[%d]: EXM_WRITE on a continuous space (DoFs shared between cells need EXM_INC)", i);
            const int32_t w = A.access == EXM_WRITE ? 1 : 0;
            EXM_CHECK(write < 0 || write == w, EXM_EINVAL, "outputs must all be WRITE or all INC");
            write = w;
        }
    }
    // an output may share no byte with another argument: the walks read
    // neighbouring columns of the inputs while other workgroups write outputs
    auto bytes = [&](int i) {   // dim components per DoF (three for the coordinate field)
        return (uintptr_t)args[i].dim * (uintptr_t)args[i].space->n_dofs * sizeof(double);
    };
    for (int i = 1 + sig.n_in; i < nargs; ++i)
        for (int j = 0; j < nargs; ++j) {
            const uintptr_t a0 = (uintptr_t)args[i].data, b0 = (uintptr_t)args[j].data;
            EXM_CHECK(i == j || a0 + bytes(i) <= b0 || b0 + bytes(j) <= a0, EXM_EINVAL,
                      "output args[%d] overlaps args[%d]", i, j);
        }
    std::memset(&P, 0, sizeof(P));
    P.fspace = V;
    P.xspace = X.space;
    P.kernel = kernel;
    P.element = el;
    P.n_layers = m->n_layers;
    P.cell_lam = m->variable ? m->d_cell_lam.p : nullptr;
    P.field_offset = V->offsets.empty() ? 0 : V->offsets[0];   // a mixed space has an offset per list entry
    P.list_off = V->mixed ? V->d_list_off.p : nullptr;
    P.fmap = V->d_map.p;
    P.xmap = X.space->d_map.p;
    P.X = (const double*)X.data;
    for (int i = 0; i < sig.n_in; ++i) P.in[i] = (const double*)args[1 + i].data;
    for (int i = 0; i < sig.n_out; ++i) P.out[i] = (double*)args[1 + sig.n_in + i].data;
    P.write = write;
    P.n_cells = m->n[2];
    P.cells = nullptr;
    P.cell_begin = 0;
    P.cell_count = m->n[2];
    return EXM_OK;
}

static int32_t default_tile_cells(const LoopLaunch& P)
{
    if (P.element == EXM_ELEMENT_P2P2 || P.kernel == EXM_K_CUBIC_FUSED) return 64;
    return 128;
}

// Lane layout of the TILED schedule: the requested columns per wavefront,
// else the fewest (longest steps) whose per-tile sums fit the default LDS
// budget; always within the hardware limit.  Returns cpw (0 if nothing fits).
static int32_t resolve_tiled_cpw(const LoopLaunch& P, const TilePlan* plan, int32_t requested, size_t* lds_out)
{
    auto bytes = [&](int32_t cpw) {
        return tiled_lds_bytes(P.kernel, P.element, plan->max_verts, plan->has_edges ? plan->max_edges : 0, 64 / cpw);
    };
    int32_t cpw = requested > 0 ? requested : default_shape(P.kernel, P.element, P.n_layers, P.n_cells).cpw;
    if (requested <= 0)
        while (cpw < 16 && bytes(cpw) > kLdsDefault) ++cpw;
    if (bytes(cpw) > kLdsLimit) return 0;
    *lds_out = bytes(cpw);
    return cpw;
}

static int32_t choose(const exm_mesh* mesh, const LoopLaunch& P, const exm_loop_opts* opts, exm_loop_opts& ch)
{
    exm_loop_opts d;
    std::memset(&d, 0, sizeof(d));
    // meshes with a layer range per column are tuned apart (negative layer key)
    if (!lookup_tuned(P.kernel, P.element, P.cell_lam ? -P.n_layers : P.n_layers, P.n_cells, &d)) {
        d.race = EXM_RACE_ATOMIC;
        d.schedule = EXM_SCHED_DIRECT;
    }
    if (opts) {
        EXM_CHECK(opts->race >= 0 && opts->race <= EXM_RACE_OWNER, EXM_EINVAL, "unknown race strategy %d", opts->race);
        EXM_CHECK(opts->schedule >= 0 && opts->schedule <= EXM_SCHED_GATHER, EXM_EINVAL, "unknown schedule %d",
                  opts->schedule);
        EXM_CHECK(opts->cols_per_wave >= 0 && opts->cols_per_wave <= 16, EXM_ERANGE,
                  "cols_per_wave = %d outside [0, 16]", opts->cols_per_wave);
        EXM_CHECK(opts->waves_per_block >= 0 && opts->waves_per_block <= 16, EXM_ERANGE,
                  "waves_per_block = %d outside [0, 16]", opts->waves_per_block);
        EXM_CHECK(opts->tile_cells == 0 || (opts->tile_cells >= 8 && opts->tile_cells <= 1024), EXM_ERANGE,
                  "tile_cells = %d outside [8, 1024]", opts->tile_cells);
        EXM_CHECK(opts->chunk_layers == 0 || opts->chunk_layers == 8 || opts->chunk_layers == 12 ||
                      opts->chunk_layers == 16 || opts->chunk_layers == 20 || opts->chunk_layers == 24 ||
                      opts->chunk_layers == 26 || opts->chunk_layers == 32 || opts->chunk_layers == 34 ||
                      opts->chunk_layers == 64,
                  EXM_ERANGE, "chunk_layers = %d: use 8, 12, 16, 20, 24, 26, 32, 34 or 64 (0 = choose)",
                  opts->chunk_layers);
        if (opts->race) d.race = opts->race;
        if (opts->schedule) {
            if (opts->schedule != d.schedule) {
                // a schedule switch drops the other schedule's tuned shape
                d.cols_per_wave = d.waves_per_block = d.tile_cells = d.chunk_layers = 0;
            }
            d.schedule = opts->schedule;
        }
        if (opts->cols_per_wave) d.cols_per_wave = opts->cols_per_wave;
        if (opts->waves_per_block) d.waves_per_block = opts->waves_per_block;
        if (opts->tile_cells) d.tile_cells = opts->tile_cells;
        if (opts->chunk_layers) d.chunk_layers = opts->chunk_layers;
    }
    if (!d.race) d.race = EXM_RACE_ATOMIC;
    if (!d.schedule) d.schedule = EXM_SCHED_DIRECT;
    // the P1xP1 and DG0xDG0 mass actions have PIPELINED kernels for columns of different heights
    const bool var_pipe = d.schedule == EXM_SCHED_PIPELINED && P.kernel == EXM_K_MASS &&
                          (P.element == EXM_ELEMENT_P1P1 || P.element == EXM_ELEMENT_DG0DG0) &&
                          mesh->n_layers <= 2000;
    EXM_CHECK(!mesh->variable || d.race != EXM_RACE_OWNER || d.schedule == EXM_SCHED_GATHER, EXM_EUNSUPPORTED,
              "owner-computes tiles need columns of one height; this mesh has a layer range per column");
    if (mesh->variable && !(d.schedule == EXM_SCHED_GATHER && gather_supported(P.kernel, P.element)) && !var_pipe) {
        // columns of different heights: the DIRECT schedule walks each on its own (or GATHER)
        if (d.schedule != EXM_SCHED_DIRECT) d.cols_per_wave = d.waves_per_block = 0;
        d.schedule = EXM_SCHED_DIRECT;
        d.tile_cells = d.chunk_layers = 0;
    }
    const bool gather = d.schedule == EXM_SCHED_GATHER && gather_supported(P.kernel, P.element);
    // the generic DIRECT kernels (tensor spaces the PIPELINED schedule also runs may ask for it)
    const bool pipe_ok = (d.schedule == EXM_SCHED_PIPELINED || d.schedule == EXM_SCHED_CHUNKED) &&
                         pipe_supported(P.kernel, P.element);   // CHUNKED runs PIPELINED off P1
    if ((direct_only(P.element) || P.kernel == EXM_K_FACET_JUMP) && !gather && !pipe_ok) {
        EXM_CHECK(d.race != EXM_RACE_OWNER, EXM_EUNSUPPORTED,
                  "owner-computes is not available for kernel %d on element %d", P.kernel, P.element);
        if (d.schedule != EXM_SCHED_DIRECT) d.cols_per_wave = d.waves_per_block = 0;
        d.schedule = EXM_SCHED_DIRECT;
        d.tile_cells = d.chunk_layers = 0;
    }
    if (d.schedule == EXM_SCHED_GATHER) {
        if (gather_supported(P.kernel, P.element)) {   // vertex columns own their outputs
            d.race = EXM_RACE_OWNER;
            d.cols_per_wave = d.tile_cells = d.chunk_layers = 0;
            if (!d.waves_per_block) d.waves_per_block = 4;
            EXM_CHECK(d.waves_per_block <= 4, EXM_ERANGE, "GATHER: waves_per_block = %d outside [0, 4]",
                      d.waves_per_block);
            ch = d;
            return EXM_OK;
        }
        d.schedule = EXM_SCHED_DIRECT;   // implemented for the P1xP1 mass action only
        d.cols_per_wave = d.waves_per_block = 0;
    }
    if (d.race == EXM_RACE_OWNER) {
        if (!continuous(P.element)) {
            d.race = EXM_RACE_ATOMIC;   // DG columns belong to one cell: nothing to own
        } else {
            EXM_CHECK(P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1, EXM_EUNSUPPORTED,
                      "owner-computes is implemented for the P1xP1 mass action (PIPELINED schedule)");
            if (d.schedule != EXM_SCHED_PIPELINED && d.schedule != EXM_SCHED_CHUNKED) {
                d.cols_per_wave = d.waves_per_block = d.tile_cells = 0;
                d.schedule = EXM_SCHED_PIPELINED;
            }
        }
    }
    if (d.schedule == EXM_SCHED_CHUNKED && !(P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1)) {
        d.schedule = EXM_SCHED_PIPELINED;
        d.tile_cells = 0;
    }
    if (d.schedule == EXM_SCHED_CHUNKED) {
        d.waves_per_block = 4;
        d.cols_per_wave = 0;
        if (!d.chunk_layers) d.chunk_layers = 16;
        EXM_CHECK(d.chunk_layers == 8 || d.chunk_layers == 16 || d.chunk_layers == 32, EXM_ERANGE,
                  "CHUNKED: chunk_layers = %d, use 8, 16 or 32", d.chunk_layers);
        if (!d.tile_cells) d.tile_cells = 64;
        const TilePlan* plan = nullptr;
        const bool owner = d.race == EXM_RACE_OWNER;
        int32_t s = owner ? build_owner_plan(mesh, d.tile_cells, &plan) : build_tile_plan(mesh, d.tile_cells, &plan);
        if (s != EXM_OK) return s;
        EXM_CHECK(plan->max_cells <= pipe_max_tile_cells(P.kernel, P.element, d.chunk_layers), EXM_EUNSUPPORTED,
                  "CHUNKED: tiles of about %d cells reach %d cells, more than %d with %d-layer chunks", d.tile_cells,
                  plan->max_cells, pipe_max_tile_cells(P.kernel, P.element, d.chunk_layers), d.chunk_layers);
        EXM_CHECK(chunk_lds_bytes(plan->max_verts, d.chunk_layers) <= kLdsLimit, EXM_EUNSUPPORTED,
                  "CHUNKED: tiles of %d cells with %d-layer chunks do not fit in LDS", d.tile_cells, d.chunk_layers);
        ch = d;
        return EXM_OK;
    }
    if (d.schedule == EXM_SCHED_PIPELINED && !pipe_supported(P.kernel, P.element)) {
        d.schedule = EXM_SCHED_STAGED;
        if (d.chunk_layers > 32) d.chunk_layers = 0;
    }
    if (d.schedule == EXM_SCHED_PIPELINED) {
        d.waves_per_block = 4;
        d.cols_per_wave = 0;
        const bool p2 = P.element == EXM_ELEMENT_P2P2;
        const bool one_layer = p2 || P.kernel != EXM_K_MASS || P.element == EXM_ELEMENT_P1DG0 ||
                               P.element == EXM_ELEMENT_P1DG1;   // one layer of one cell per thread
        if (!d.chunk_layers) d.chunk_layers = P.n_layers >= 12 && !one_layer ? 16 : 8;
        EXM_CHECK(pipe_chunk_ok(P.kernel, P.element, d.chunk_layers), EXM_ERANGE,
                  "PIPELINED: chunk_layers = %d, use 8, 12, 16, 20, 24 or 32 on P1xP1, 8 or 16 on P2xP2, CG1xDG* "
                  "and the cubic forms, and 8, 16 or 32 on the spaces discontinuous horizontally (20, 26 and 34 "
                  "also on DG0xDG0 with columns of one height)",
                  d.chunk_layers);
        EXM_CHECK(!(mesh->variable && P.element == EXM_ELEMENT_DG0DG0 && dg0_long_chunk(d.chunk_layers)), EXM_ERANGE,
                  "PIPELINED: chunk_layers = %d on DG0xDG0 needs columns of one height (use 8, 16 or 32)",
                  d.chunk_layers);
        // the fixed-height P1 x P1 walk takes larger tiles in wider workgroups
        const bool wide = P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1 && !mesh->variable &&
                          pipe_p1_wide_max_cells(d.chunk_layers) > 0;
        const int32_t max_cells =
            wide ? pipe_p1_wide_max_cells(d.chunk_layers) : pipe_max_tile_cells(P.kernel, P.element, d.chunk_layers);
        const int32_t max_verts =
            wide ? pipe_p1_wide_max_verts(d.chunk_layers) : pipe_max_tile_verts(P.kernel, P.element, d.chunk_layers);
        if (!d.tile_cells) d.tile_cells = std::min(one_layer ? 32 : 64, max_cells);
        EXM_CHECK(d.tile_cells <= max_cells, EXM_EUNSUPPORTED,
                  "PIPELINED: tiles of %d cells with %d-layer chunks exceed %d cells", d.tile_cells, d.chunk_layers,
                  max_cells);
        const TilePlan* plan = nullptr;
        const bool owner = d.race == EXM_RACE_OWNER;
        int32_t s = owner ? build_owner_plan(mesh, d.tile_cells, &plan) : build_tile_plan(mesh, d.tile_cells, &plan);
        if (s != EXM_OK) return s;
        EXM_CHECK(plan->max_cells <= max_cells, EXM_EUNSUPPORTED,
                  "PIPELINED: owner tiles of about %d cells reach %d cells with their neighbours, more than %d "
                  "with %d-layer chunks", d.tile_cells, plan->max_cells, max_cells, d.chunk_layers);
        if (P.element == EXM_ELEMENT_P1P1 || P.element == EXM_ELEMENT_P1DG0 || P.element == EXM_ELEMENT_P1DG1)
            EXM_CHECK(plan->max_verts <= max_verts, EXM_EUNSUPPORTED,
                      "PIPELINED: tiles of %d cells touch up to %d vertices, more than %d with %d-layer chunks",
                      d.tile_cells, plan->max_verts, max_verts, d.chunk_layers);
        if (p2) {
            EXM_CHECK(plan->has_edges, EXM_EINVAL, "P2 needs the mesh's cell_edge map");
            EXM_CHECK(plan->max_verts + plan->max_edges <= pipe_max_tile_entities(d.chunk_layers), EXM_EUNSUPPORTED,
                      "PIPELINED: tiles of %d cells touch up to %d vertices and %d edges, more than %d entities with "
                      "%d-layer chunks",
                      d.tile_cells, plan->max_verts, plan->max_edges, pipe_max_tile_entities(d.chunk_layers),
                      d.chunk_layers);
        }
        EXM_CHECK(pipe_lds_bytes(P.kernel, P.element, plan->max_verts, plan->has_edges ? plan->max_edges : 0,
                                 plan->max_cells, d.chunk_layers) <= kLdsLimit,
                  EXM_EUNSUPPORTED, "tiles of %d cells with %d-layer chunks do not fit in LDS", d.tile_cells,
                  d.chunk_layers);
        ch = d;
        return EXM_OK;
    }
    if (d.schedule == EXM_SCHED_STAGED)
        EXM_CHECK(d.chunk_layers % 8 == 0 && (d.chunk_layers & (d.chunk_layers - 1)) == 0, EXM_ERANGE,
                  "STAGED: chunk_layers = %d, use 8, 16, 32 or 64", d.chunk_layers);
    if (d.schedule == EXM_SCHED_STAGED && !staged_supported(P.kernel, P.element)) {
        d.schedule = EXM_SCHED_TILED;
        d.chunk_layers = 0;
    }
    // DG columns belong to one cell: nothing to sum per tile
    if (!continuous(P.element) && d.schedule == EXM_SCHED_TILED) {
        d.schedule = EXM_SCHED_DIRECT;
        d.tile_cells = 0;
        if (d.waves_per_block > 4) d.waves_per_block = 4;
    }
    if (d.schedule == EXM_SCHED_STAGED) {
        d.waves_per_block = 4;
        d.cols_per_wave = 0;
        if (!d.chunk_layers) d.chunk_layers = P.n_layers >= 12 ? 16 : 8;
        if (!d.tile_cells) d.tile_cells = std::min(64, staged_max_tile_cells(d.chunk_layers));
        EXM_CHECK(d.tile_cells <= staged_max_tile_cells(d.chunk_layers), EXM_EUNSUPPORTED,
                  "STAGED: tiles of %d cells need chunk_layers <= %d", d.tile_cells,
                  staged_max_tile_cells(d.chunk_layers));
        const TilePlan* plan = nullptr;
        int32_t s = build_tile_plan(mesh, d.tile_cells, &plan);
        if (s != EXM_OK) return s;
        EXM_CHECK(staged_lds_bytes(P.kernel, P.element, plan->max_verts, d.chunk_layers) <= kLdsLimit,
                  EXM_EUNSUPPORTED, "tiles of %d cells with %d-layer chunks do not fit in LDS", d.tile_cells,
                  d.chunk_layers);
        ch = d;
        return EXM_OK;
    }
    d.chunk_layers = 0;
    if (d.schedule == EXM_SCHED_DIRECT) {
        EXM_CHECK(d.waves_per_block <= 4, EXM_ERANGE, "DIRECT schedule: waves_per_block = %d outside [0, 4]",
                  d.waves_per_block);
        LoopShape s = shape_from_opts(P.kernel, P.element, P.n_layers, P.n_cells, &d);
        d.cols_per_wave = s.cpw;
        d.waves_per_block = s.wpb;
        d.tile_cells = 0;
    } else {
        if (!d.tile_cells) d.tile_cells = default_tile_cells(P);
        if (!d.waves_per_block) d.waves_per_block = 4;
        d.waves_per_block = std::min(d.waves_per_block, tiled_max_threads(P.kernel, P.element) / 64);
        const TilePlan* plan = nullptr;
        int32_t s = build_tile_plan(mesh, d.tile_cells, &plan);
        if (s != EXM_OK) return s;
        size_t lds = 0;
        const int32_t cpw = resolve_tiled_cpw(P, plan, d.cols_per_wave, &lds);
        EXM_CHECK(cpw > 0, EXM_EUNSUPPORTED, "tiles of %d cells do not fit in LDS; use smaller tile_cells or more "
                  "cols_per_wave", d.tile_cells);
        d.cols_per_wave = cpw;
    }
    ch = d;
    return EXM_OK;
}

static int32_t run_direct(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    P.race = ch.race;
    P.shape = make_shape(ch.cols_per_wave, ch.waves_per_block);
    if (P.race == EXM_RACE_COLOUR && continuous(P.element)) {
        const Colouring* col = nullptr;
        int32_t s = build_colouring(mesh, &col);
        if (s != EXM_OK) return s;
        P.cells = col->cells.p;
        for (int32_t k = 0; k < col->n_colours; ++k) {
            P.cell_begin = col->offsets[k];
            P.cell_count = col->offsets[k + 1] - col->offsets[k];
            s = launch_column_loop(P, stream);
            if (s != EXM_OK) return s;
        }
        return EXM_OK;
    }
    P.race = EXM_RACE_ATOMIC;
    P.cells = nullptr;
    P.cell_begin = 0;
    P.cell_count = P.n_cells;
    return launch_column_loop(P, stream);
}

static void fill_tile_args(const TilePlan* plan, const LoopLaunch& P, TileArgs& t)
{
    std::memset(&t, 0, sizeof(t));
    t.vstride = plan->max_verts;
    t.estride = plan->has_edges ? plan->max_edges : 0;
    t.cell_off = plan->cell_off.p;
    t.cells = plan->cells.p;
    t.vert_off = plan->vert_off.p;
    t.verts = plan->verts.p;
    t.edge_off = plan->has_edges ? plan->edge_off.p : nullptr;
    t.edges = plan->has_edges ? plan->edges.p : nullptr;
    t.lcv = plan->local_cv.p;
    t.lce = plan->has_edges ? plan->local_ce.p : nullptr;
    t.xstart = P.xspace->d_starts[0].p;
    t.fstart0 = P.fspace->d_starts[0].p;
    t.fstart1 = P.fspace->d_starts[1].p;
    t.owned = plan->owner ? plan->owned.p : nullptr;
    // closed-form column starts where Algorithm 1 gives one: one layer count
    // and one DoF count per entity type
    const bool uniform = !P.fspace->mesh->variable;
    const bool xok = uniform && !P.xspace->mixed && P.xspace->col_size[0] > 0;
    const bool fok = uniform && !P.fspace->mixed;
    t.xbase = P.xspace->base[0];
    t.xstep = xok ? P.xspace->col_size[0] : 0;
    t.fbase0 = P.fspace->base[0];
    t.fstep0 = fok && P.fspace->col_size[0] > 0 ? P.fspace->col_size[0] : 0;
    t.fbase1 = P.fspace->base[1];
    t.fstep1 = fok && P.fspace->col_size[1] > 0 ? P.fspace->col_size[1] : 0;
    const exm_mesh* m = P.fspace->mesh;
    t.vlo = m->variable ? m->d_vert_lo.p : nullptr;
    t.vhi = m->variable ? m->d_vert_hi.p : nullptr;
    t.clo = m->variable ? m->d_cell_lo.p : nullptr;
}

static int32_t run_tiled(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    const TilePlan* plan = nullptr;
    int32_t s = build_tile_plan(mesh, ch.tile_cells, &plan);
    if (s != EXM_OK) return s;
    size_t lds = 0;
    const int32_t cpw = resolve_tiled_cpw(P, plan, ch.cols_per_wave, &lds);
    EXM_CHECK(cpw > 0, EXM_EUNSUPPORTED, "tiles of %d cells do not fit in LDS", ch.tile_cells);
    if (P.element == EXM_ELEMENT_P2P2) EXM_CHECK(plan->has_edges, EXM_EINVAL, "P2 needs the mesh's cell_edge map");
    P.race = ch.race;
    P.shape = make_shape(cpw, 1);
    TileArgs t;
    fill_tile_args(plan, P, t);
    const int32_t threads = 64 * std::max(1, std::min(ch.waves_per_block, 16));
    if (ch.race == EXM_RACE_COLOUR) {
        t.tiles = plan->colour_tiles.p;
        for (int32_t k = 0; k < plan->n_colours; ++k) {
            t.tile_begin = (int32_t)plan->colour_off[k];
            t.tile_count = (int32_t)(plan->colour_off[k + 1] - plan->colour_off[k]);
            s = launch_tiled(P, t, threads, lds, stream);
            if (s != EXM_OK) return s;
        }
        return EXM_OK;
    }
    t.tiles = nullptr;
    t.tile_begin = 0;
    t.tile_count = plan->n_tiles;
    return launch_tiled(P, t, threads, lds, stream);
}

static int32_t run_staged(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    const TilePlan* plan = nullptr;
    int32_t s = build_tile_plan(mesh, ch.tile_cells, &plan);
    if (s != EXM_OK) return s;
    const size_t lds = staged_lds_bytes(P.kernel, P.element, plan->max_verts, ch.chunk_layers);
    EXM_CHECK(lds <= kLdsLimit, EXM_EUNSUPPORTED, "staging does not fit in LDS");
    P.race = ch.race;
    P.shape = make_shape(1, 1);
    const ColArgs a = col_args(P);
    TileArgs t;
    fill_tile_args(plan, P, t);
    if (ch.race == EXM_RACE_COLOUR && continuous(P.element)) {
        t.tiles = plan->colour_tiles.p;
        for (int32_t k = 0; k < plan->n_colours; ++k) {
            t.tile_begin = (int32_t)plan->colour_off[k];
            t.tile_count = (int32_t)(plan->colour_off[k + 1] - plan->colour_off[k]);
            s = launch_staged(P, a, t, ch.chunk_layers, lds, stream);
            if (s != EXM_OK) return s;
        }
        return EXM_OK;
    }
    if (!continuous(P.element)) P.race = EXM_RACE_ATOMIC;   // nothing is shared
    t.tiles = nullptr;
    t.tile_begin = 0;
    t.tile_count = plan->n_tiles;
    return launch_staged(P, a, t, ch.chunk_layers, lds, stream);
}

static int32_t run_pipe(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    const TilePlan* plan = nullptr;
    const bool owner = ch.race == EXM_RACE_OWNER;
    int32_t s = owner ? build_owner_plan(mesh, ch.tile_cells, &plan) : build_tile_plan(mesh, ch.tile_cells, &plan);
    if (s != EXM_OK) return s;
    const size_t lds = pipe_lds_bytes(P.kernel, P.element, plan->max_verts, plan->has_edges ? plan->max_edges : 0,
                                      plan->max_cells, ch.chunk_layers);
    P.race = ch.race;
    P.shape = make_shape(1, 1);
    const ColArgs a = col_args(P);
    TileArgs t;
    fill_tile_args(plan, P, t);
    if (ch.race == EXM_RACE_COLOUR && continuous(P.element)) {
        t.tiles = plan->colour_tiles.p;
        for (int32_t k = 0; k < plan->n_colours; ++k) {
            t.tile_begin = (int32_t)plan->colour_off[k];
            t.tile_count = (int32_t)(plan->colour_off[k + 1] - plan->colour_off[k]);
            s = launch_pipe(P, a, t, plan->max_cells, ch.chunk_layers, lds, stream);
            if (s != EXM_OK) return s;
        }
        return EXM_OK;
    }
    t.tiles = nullptr;
    t.tile_begin = 0;
    t.tile_count = plan->n_tiles;
    if (!continuous(P.element)) P.race = EXM_RACE_ATOMIC;   // nothing is shared
    return launch_pipe(P, a, t, plan->max_cells, ch.chunk_layers, lds, stream);
}

static int32_t run_chunked(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    const TilePlan* plan = nullptr;
    const bool owner = ch.race == EXM_RACE_OWNER;
    int32_t s = owner ? build_owner_plan(mesh, ch.tile_cells, &plan) : build_tile_plan(mesh, ch.tile_cells, &plan);
    if (s != EXM_OK) return s;
    const size_t lds = chunk_lds_bytes(plan->max_verts, ch.chunk_layers);
    P.race = ch.race;
    P.shape = make_shape(1, 1);
    const ColArgs a = col_args(P);
    TileArgs t;
    fill_tile_args(plan, P, t);
    if (ch.race == EXM_RACE_COLOUR) {
        t.tiles = plan->colour_tiles.p;
        for (int32_t k = 0; k < plan->n_colours; ++k) {
            t.tile_begin = (int32_t)plan->colour_off[k];
            t.tile_count = (int32_t)(plan->colour_off[k + 1] - plan->colour_off[k]);
            s = launch_chunked(P, a, t, ch.chunk_layers, lds, stream);
            if (s != EXM_OK) return s;
        }
        return EXM_OK;
    }
    t.tiles = nullptr;
    t.tile_begin = 0;
    t.tile_count = plan->n_tiles;
    return launch_chunked(P, a, t, ch.chunk_layers, lds, stream);
}

static int32_t run_gather(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    const VertexFans* fans = nullptr;
    int32_t s = build_vertex_fans(mesh, &fans);
    if (s != EXM_OK) return s;
    P.race = EXM_RACE_OWNER;
    return launch_gather(P, fans, ch.waves_per_block, stream);
}

static int32_t run_on_mesh(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
{
    if (ch.schedule == EXM_SCHED_GATHER) return run_gather(mesh, P, ch, stream);
    if (ch.schedule == EXM_SCHED_CHUNKED) return run_chunked(mesh, P, ch, stream);
    if (ch.schedule == EXM_SCHED_DIRECT) return run_direct(mesh, P, ch, stream);
    if (ch.schedule == EXM_SCHED_PIPELINED) return run_pipe(mesh, P, ch, stream);
    if (ch.schedule == EXM_SCHED_STAGED) return run_staged(mesh, P, ch, stream);
    return run_tiled(mesh, P, ch, stream);
}

}  // namespace exm

using namespace exm;

extern "C" {

int32_t exm_par_loop(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args,
                     const exm_loop_opts* opts, void* stream)
{
    clear_error();
    LoopLaunch P;
    int32_t s = prepare(kernel, iterset, nargs, args, P);
    if (s != EXM_OK) return s;
    exm_loop_opts ch;
    s = choose(iterset, P, opts, ch);
    if (s != EXM_OK) return s;
    s = check_pending();
    if (s != EXM_OK) return s;
    s = ensure_vertical(P.xspace, P.X, (hipStream_t)stream);
    if (s != EXM_OK) return s;
    return run_on_mesh(iterset, P, ch, (hipStream_t)stream);
}

int32_t exm_par_loop_config(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args,
                            const exm_loop_opts* opts, exm_loop_opts* chosen)
{
    clear_error();
    EXM_CHECK(chosen != nullptr, EXM_EINVAL, "chosen is NULL");
    LoopLaunch P;
    int32_t s = prepare(kernel, iterset, nargs, args, P);
    if (s != EXM_OK) return s;
    return choose(iterset, P, opts, *chosen);
}

int32_t exm_autotune(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args, void* stream,
                     exm_loop_opts* best)
{
    clear_error();
    LoopLaunch P;
    int32_t s = prepare(kernel, iterset, nargs, args, P);
    if (s != EXM_OK) return s;
    hipStream_t hs = (hipStream_t)stream;
    s = ensure_vertical(P.xspace, P.X, hs);
    if (s != EXM_OK) return s;
    // Scratch outputs so the caller's buffers stay untouched.
    Signature sig;
    signature(kernel, sig);
    const int64_t n = args[1].space->n_dofs;
    DevBuf<double> scratch[3];
    for (int i = 0; i < sig.n_out; ++i) {
        s = scratch[i].alloc((size_t)n);
        if (s != EXM_OK) return s;
        EXM_TRY_HIP(hipMemsetAsync(scratch[i].p, 0, sizeof(double) * (size_t)n, hs));
        P.out[i] = scratch[i].p;
    }
    std::vector<exm_loop_opts> cand;
    const bool cg = continuous(P.element);
    const int32_t races[2] = {EXM_RACE_ATOMIC, EXM_RACE_COLOUR};
    for (int r = 0; r < (cg ? 2 : 1); ++r) {
        for (int32_t c : {1, 2, 3, 4}) cand.push_back(exm_loop_opts{races[r], EXM_SCHED_DIRECT, c, 4, 0, 0});
        if (iterset->variable) {   // columns of different heights run DIRECT, GATHER or (P1, DG0 mass) PIPELINED
            for (int32_t c : {1, 2, 4}) cand.push_back(exm_loop_opts{races[r], EXM_SCHED_DIRECT, c, 2, 0, 0});
            if (r == 0 && gather_supported(P.kernel, P.element))
                for (int32_t w : {1, 2, 4}) cand.push_back(exm_loop_opts{EXM_RACE_OWNER, EXM_SCHED_GATHER, 0, w, 0, 0});
            if (P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1)
                for (int32_t tc : {32, 48, 64})
                    for (int32_t S : {8, 16}) cand.push_back(exm_loop_opts{races[r], EXM_SCHED_PIPELINED, 0, 4, tc, S});
            if (P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_DG0DG0)
                for (int32_t tc : {32, 64})
                    for (int32_t S : {16, 32})
                        if (tc <= pipe_max_tile_cells(P.kernel, P.element, S))
                            cand.push_back(exm_loop_opts{races[r], EXM_SCHED_PIPELINED, 0, 4, tc, S});
            continue;
        }
        if (r == 0 && gather_supported(P.kernel, P.element))
            for (int32_t w : {1, 2, 4}) cand.push_back(exm_loop_opts{EXM_RACE_OWNER, EXM_SCHED_GATHER, 0, w, 0, 0});
        if (staged_supported(P.kernel, P.element))
            for (int32_t tc : {32, 64, 128, 256})
                for (int32_t S : {8, 16, 32, 64})
                    if (tc <= staged_max_tile_cells(S))
                        cand.push_back(exm_loop_opts{races[r], EXM_SCHED_STAGED, 0, 4, tc, S});
        if (pipe_supported(P.kernel, P.element))
            for (int32_t tc : {16, 24, 30, 32, 38, 48, 50, 64, 96, 128, 256})
                for (int32_t S : {8, 12, 16, 20, 24, 26, 32, 34}) {
                    const bool p1 = P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1;
                    const int32_t narrow = pipe_max_tile_cells(P.kernel, P.element, S);
                    // 30, 38 and 50 cells: the full tiles of DG0's 34-, 26- and 20-layer chunks
                    const bool full_dg0 = P.element == EXM_ELEMENT_DG0DG0 && dg0_long_chunk(S) && tc == narrow;
                    if ((tc == 30 || tc == 38 || tc == 50) && !full_dg0) continue;
                    const int32_t limit = p1 ? std::max(narrow, pipe_p1_wide_max_cells(S)) : narrow;
                    if (pipe_chunk_ok(P.kernel, P.element, S) && tc <= limit &&
                        (tc >= 32 || full_dg0 || P.element == EXM_ELEMENT_P2P2 || P.kernel != EXM_K_MASS)) {
                        cand.push_back(exm_loop_opts{races[r], EXM_SCHED_PIPELINED, 0, 4, tc, S});
                        if (r == 0 && p1) cand.push_back(exm_loop_opts{EXM_RACE_OWNER, EXM_SCHED_PIPELINED, 0, 4, tc, S});
                        if (p1 && (S & (S - 1)) == 0 && tc <= narrow) {
                            cand.push_back(exm_loop_opts{races[r], EXM_SCHED_CHUNKED, 0, 4, tc, S});
                            if (r == 0) cand.push_back(exm_loop_opts{EXM_RACE_OWNER, EXM_SCHED_CHUNKED, 0, 4, tc, S});
                        }
                    }
                }
        if (cg)
            for (int32_t t : {8, 16, 24, 32, 64, 128, 256})
                for (int32_t c : {0, 1, 2, 4})
                    for (int32_t w : {4, 8}) cand.push_back(exm_loop_opts{races[r], EXM_SCHED_TILED, c, w, t, 0});
    }
    hipEvent_t e0, e1;
    EXM_TRY_HIP(hipEventCreate(&e0));
    EXM_TRY_HIP(hipEventCreate(&e1));
    // bring the clocks to their steady state before the first candidate is
    // timed: about a quarter second of the first candidate, untimed
    {
        exm_loop_opts ch0;
        if (choose(iterset, P, &cand[0], ch0) == EXM_OK) {
            float spent = 0.0f;
            for (int round = 0; round < 64 && spent < 250.0f && s == EXM_OK; ++round) {
                EXM_TRY_HIP(hipEventRecord(e0, hs));
                for (int i = 0; i < 8 && s == EXM_OK; ++i) {
                    LoopLaunch Q = P;
                    s = run_on_mesh(iterset, Q, ch0, hs);
                }
                EXM_TRY_HIP(hipEventRecord(e1, hs));
                EXM_TRY_HIP(hipEventSynchronize(e1));
                float ms = 0;
                EXM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
                spent += ms;
            }
            if (s != EXM_OK) return s;
        }
    }
    float best_ms = 1e30f;
    exm_loop_opts best_opts = cand[0];
    for (const exm_loop_opts& c : cand) {
        exm_loop_opts ch;
        if (choose(iterset, P, &c, ch) != EXM_OK) continue;   // e.g. a tile too large for LDS
        LoopLaunch Q = P;
        s = run_on_mesh(iterset, Q, ch, hs);   // warm-up
        if (s != EXM_OK) break;
        float t_min = 1e30f;
        for (int rep = 0; rep < 3 && s == EXM_OK; ++rep) {
            EXM_TRY_HIP(hipEventRecord(e0, hs));
            Q = P;
            s = run_on_mesh(iterset, Q, ch, hs);
            EXM_TRY_HIP(hipEventRecord(e1, hs));
            EXM_TRY_HIP(hipEventSynchronize(e1));
            float ms = 0;
            EXM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            t_min = std::min(t_min, ms);
        }
        if (s != EXM_OK) break;
        if (t_min < best_ms) {
            best_ms = t_min;
            best_opts = ch;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != EXM_OK) return s;
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[tune_key(P.kernel, P.element, P.cell_lam ? -P.n_layers : P.n_layers, P.n_cells)] = best_opts;
    }
    if (best) *best = best_opts;
    return EXM_OK;
}

int32_t exm_autotune_save(const char* path)
{
    clear_error();
    EXM_CHECK(path != nullptr, EXM_EINVAL, "path is NULL");
    std::ofstream f(path);
    EXM_CHECK(f.good(), EXM_EINVAL, "cannot open %s", path);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    f << "# kernel element n_layers log2_cells race schedule cols_per_wave waves_per_block tile_cells chunk_layers\n";
    for (auto& kv : g_tuned)
        f << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' ' << std::get<2>(kv.first) << ' '
          << std::get<3>(kv.first) << ' ' << kv.second.race << ' ' << kv.second.schedule << ' '
          << kv.second.cols_per_wave << ' ' << kv.second.waves_per_block << ' ' << kv.second.tile_cells << ' '
          << kv.second.chunk_layers << '\n';
    return EXM_OK;
}

int32_t exm_autotune_load(const char* path)
{
    clear_error();
    EXM_CHECK(path != nullptr, EXM_EINVAL, "path is NULL");
    std::ifstream f(path);
    EXM_CHECK(f.good(), EXM_EINVAL, "cannot open %s", path);
    std::string line;
    std::map<TuneKey, exm_loop_opts> table;
    int ln = 0;
    while (std::getline(f, line)) {
        ++ln;
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        int32_t k, e, l, b;
        exm_loop_opts o;
        EXM_CHECK((bool)(is >> k >> e >> l >> b >> o.race >> o.schedule >> o.cols_per_wave >> o.waves_per_block >>
                         o.tile_cells >> o.chunk_layers),
                  EXM_EINVAL, "%s:%d: malformed line", path, ln);
        EXM_CHECK((o.race == EXM_RACE_ATOMIC || o.race == EXM_RACE_COLOUR || o.race == EXM_RACE_OWNER) &&
                      o.schedule >= EXM_SCHED_DIRECT && o.schedule <= EXM_SCHED_GATHER && o.cols_per_wave >= 0 &&
                      o.cols_per_wave <= 16 && o.waves_per_block >= 1 && o.waves_per_block <= 16 &&
                      o.tile_cells >= 0 && o.tile_cells <= 1024 &&
                      (o.chunk_layers == 0 || o.chunk_layers == 8 || o.chunk_layers == 12 || o.chunk_layers == 16 ||
                       o.chunk_layers == 20 || o.chunk_layers == 24 || o.chunk_layers == 26 || o.chunk_layers == 32 ||
                       o.chunk_layers == 34 || o.chunk_layers == 64),
                  EXM_ERANGE, "%s:%d: values out of range", path, ln);
        table[TuneKey(k, e, l, b)] = o;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& kv : table) g_tuned[kv.first] = kv.second;
    return EXM_OK;
}

}  // extern "C"
