// Handles, validation and the numbering builder (Algorithms 1 and 2) of
// libexm.so, plus the base-cell colouring and the STREAM triad.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>

#include "exm_internal.hpp"

namespace exm {

static thread_local std::string g_error;

int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

int32_t check_pending()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(EXM_EHIP, "earlier device work failed: %s", hipGetErrorString(e));
    return EXM_OK;
}

// ---------------------------------------------------------------------------
// Numbering kernels.
//
// With a constant layer count the counter of Algorithm 1 advances by the same
// amount for every entity of one dimension: the column of base entity (d, i)
// holds (lambda + 1) delta(d,0) + lambda delta(d,1) DoFs and starts at
// base[d] + i * col_size[d], base[d] being the DoFs of all columns of lower
// dimension.  Inside a column, level l starts at l (delta(d,0) + delta(d,1))
// and the vertical entity over interval l follows its bottom level.

__global__ void k_column_starts(int32_t n, int64_t base, int32_t col_size, int32_t* dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = col_size ? (int32_t)(base + i * (int64_t)col_size) : -1;
}

// One position of the explicit list: closure entity e (0..2 vertex, 3..5 edge,
// 6 cell) and the DoF offset inside that entity's column for layer 0.
struct StencilPos {
    int32_t entity;
    int32_t shift;
};

__global__ void k_bottom_map(int32_t n_cells, int32_t k, const StencilPos* __restrict__ pos,
                             const int32_t* __restrict__ cell_vertex, const int32_t* __restrict__ cell_edge,
                             int64_t base0, int64_t base1, int64_t base2, int32_t cs0, int32_t cs1, int32_t cs2,
                             int32_t* __restrict__ map)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)n_cells * k;
    if (t >= total) return;
    int64_t c = t / k;
    int32_t p = (int32_t)(t - c * k);
    StencilPos sp = pos[p];
    int64_t start;
    if (sp.entity < 3) start = base0 + (int64_t)cell_vertex[c * 3 + sp.entity] * cs0;
    else if (sp.entity < 6) start = base1 + (int64_t)cell_edge[c * 3 + sp.entity - 3] * cs1;
    else start = base2 + c * (int64_t)cs2;
    map[t] = (int32_t)(start + sp.shift);
}

// ---------------------------------------------------------------------------
// Greedy base-cell colouring (host): cells are visited in base order and take
// the smallest colour not used by an already coloured cell sharing a vertex.

int32_t build_colouring(const exm_mesh* m, const Colouring** out)
{
    std::lock_guard<std::mutex> lock(m->mu);
    if (m->colouring) {
        *out = m->colouring.get();
        return EXM_OK;
    }
    const int32_t nv = m->n[0], nc = m->n[2];
    const int32_t* cv = m->h_cell_vertex.data();
    // vertex -> cells adjacency (CSR)
    std::vector<int64_t> vstart(nv + 1, 0);
    for (int64_t i = 0; i < (int64_t)nc * 3; ++i) vstart[cv[i] + 1]++;
    for (int32_t v = 0; v < nv; ++v) vstart[v + 1] += vstart[v];
    std::vector<int32_t> vcells(vstart[nv]);
    std::vector<int64_t> fill(vstart.begin(), vstart.end() - 1);
    for (int32_t c = 0; c < nc; ++c)
        for (int a = 0; a < 3; ++a) vcells[fill[cv[c * 3 + a]]++] = c;
    std::vector<int32_t> colour(nc, -1);
    std::vector<int32_t> mark;   // mark[col] == c when colour col is taken by a neighbour of c
    int32_t ncol = 0;
    for (int32_t c = 0; c < nc; ++c) {
        for (int a = 0; a < 3; ++a) {
            int32_t v = cv[c * 3 + a];
            for (int64_t j = vstart[v]; j < vstart[v + 1]; ++j) {
                int32_t o = colour[vcells[j]];
                if (o >= 0) mark[o] = c;
            }
        }
        int32_t col = 0;
        while (col < ncol && mark[col] == c) ++col;
        if (col == ncol) {
            ++ncol;
            mark.push_back(-1);
        }
        colour[c] = col;
    }
    auto col = std::make_unique<Colouring>();
    col->n_colours = ncol;
    col->offsets.assign(ncol + 1, 0);
    for (int32_t c = 0; c < nc; ++c) col->offsets[colour[c] + 1]++;
    for (int32_t k = 0; k < ncol; ++k) col->offsets[k + 1] += col->offsets[k];
    col->host_cells.resize(nc);
    std::vector<int64_t> f2(col->offsets.begin(), col->offsets.end() - 1);
    for (int32_t c = 0; c < nc; ++c) col->host_cells[f2[colour[c]]++] = c;
    int32_t s = col->cells.upload(col->host_cells.data(), col->host_cells.size());
    if (s != EXM_OK) return s;
    m->colouring = std::move(col);
    *out = m->colouring.get();
    return EXM_OK;
}

// ---------------------------------------------------------------------------
// STREAM triad.

__global__ void k_triad(double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ c,
                        double alpha, int64_t n)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        a[i] = b[i] + alpha * c[i];
}

// The same on 16-byte pairs with non-temporal loads and stores (arrays
// 16-byte aligned): the faster of the two on gfx950 by about 8 %, so the
// yardstick is not set low by the access width.
typedef double double2v __attribute__((ext_vector_type(2)));
__global__ void k_triad2(double* __restrict__ a, const double* __restrict__ b, const double* __restrict__ c,
                         double alpha, int64_t n)
{
    const int64_t np = n / 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < np; i += stride) {
        const double2v x = __builtin_nontemporal_load((const double2v*)b + i);
        const double2v y = __builtin_nontemporal_load((const double2v*)c + i);
        __builtin_nontemporal_store(x + alpha * y, (double2v*)a + i);
    }
    if (t0 == 0 && (n & 1)) a[n - 1] = b[n - 1] + alpha * c[n - 1];
}

}  // namespace exm

using namespace exm;

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* exm_last_error(void) { return g_error.c_str(); }

int32_t exm_abi_version(void) { return EXM_ABI_VERSION; }

int32_t exm_sync(void* stream)
{
    clear_error();
    EXM_TRY_HIP(hipStreamSynchronize((hipStream_t)stream));
    return check_pending();
}

static int32_t mesh_create(int32_t n_vertices, int32_t n_edges, int32_t n_cells, const int32_t* cell_vertex,
                           const int32_t* cell_edge, int32_t n_layers, const int32_t* layers, exm_mesh** out)
{
    EXM_CHECK(out != nullptr, EXM_EINVAL, "out is NULL");
    *out = nullptr;
    EXM_CHECK(cell_vertex != nullptr, EXM_EINVAL, "cell_vertex is NULL");
    EXM_CHECK(n_vertices >= 3 && n_cells >= 1 && n_edges >= 0, EXM_ERANGE,
              "need n_vertices >= 3, n_cells >= 1, n_edges >= 0 (got %d, %d, %d)", n_vertices, n_cells, n_edges);
    EXM_CHECK(n_layers >= 1, EXM_ERANGE, "n_layers must be >= 1 (got %d)", n_layers);
    EXM_CHECK(cell_edge == nullptr || n_edges >= 3, EXM_ERANGE, "cell_edge given but n_edges = %d", n_edges);
    for (int64_t i = 0; i < (int64_t)n_cells * 3; ++i)
        EXM_CHECK(cell_vertex[i] >= 0 && cell_vertex[i] < n_vertices, EXM_ERANGE,
                  "cell_vertex[%lld] = %d outside [0, %d)", (long long)i, cell_vertex[i], n_vertices);
    for (int64_t c = 0; c < n_cells; ++c) {
        const int32_t* v = cell_vertex + c * 3;
        EXM_CHECK(v[0] != v[1] && v[1] != v[2] && v[0] != v[2], EXM_EINVAL,
                  "cell %lld repeats a vertex", (long long)c);
    }
    if (cell_edge) {
        for (int64_t i = 0; i < (int64_t)n_cells * 3; ++i)
            EXM_CHECK(cell_edge[i] >= 0 && cell_edge[i] < n_edges, EXM_ERANGE,
                      "cell_edge[%lld] = %d outside [0, %d)", (long long)i, cell_edge[i], n_edges);
        // edge a of a cell joins its vertices (a + 1) % 3 and (a + 2) % 3: every
        // cell that lists an edge must see the same two vertices, and no two
        // edges may join the same pair (a shared edge would get two columns)
        std::vector<int64_t> ends((size_t)n_edges, -1);
        for (int64_t c = 0; c < n_cells; ++c)
            for (int a = 0; a < 3; ++a) {
                const int32_t e = cell_edge[c * 3 + a];
                const int64_t u = cell_vertex[c * 3 + (a + 1) % 3], w = cell_vertex[c * 3 + (a + 2) % 3];
                const int64_t key = std::min(u, w) * n_vertices + std::max(u, w);
                EXM_CHECK(ends[e] < 0 || ends[e] == key, EXM_EINVAL,
                          "cell_edge: edge %d, opposite local vertex %d of cell %lld, joins vertices %lld and %lld "
                          "there but %lld and %lld in an earlier cell",
                          e, a, (long long)c, (long long)u, (long long)w, (long long)(ends[e] / n_vertices),
                          (long long)(ends[e] % n_vertices));
                ends[e] = key;
            }
        std::vector<int64_t> sorted;
        sorted.reserve(ends.size());
        for (int64_t k : ends)
            if (k >= 0) sorted.push_back(k);
        std::sort(sorted.begin(), sorted.end());
        const auto dup = std::adjacent_find(sorted.begin(), sorted.end());
        EXM_CHECK(dup == sorted.end(), EXM_EINVAL, "cell_edge: two edges join vertices %lld and %lld",
                  (long long)(dup == sorted.end() ? 0 : *dup / n_vertices),
                  (long long)(dup == sorted.end() ? 0 : *dup % n_vertices));
    }
    if (layers)
        for (int64_t c = 0; c < n_cells; ++c)
            EXM_CHECK(layers[2 * c] >= 0 && layers[2 * c] < layers[2 * c + 1] && layers[2 * c + 1] <= n_layers,
                      EXM_ERANGE, "layers of cell %lld = [%d, %d) not inside [0, %d) or empty", (long long)c,
                      layers[2 * c], layers[2 * c + 1], n_layers);
    auto m = std::make_unique<exm_mesh>();
    m->n[0] = n_vertices;
    m->n[1] = n_edges;
    m->n[2] = n_cells;
    m->n_layers = n_layers;
    EXM_TRY_HIP(hipGetDevice(&m->device));
    m->h_cell_vertex.assign(cell_vertex, cell_vertex + (size_t)n_cells * 3);
    int32_t s = m->d_cell_vertex.upload(cell_vertex, (size_t)n_cells * 3);
    if (s != EXM_OK) return s;
    if (cell_edge) {
        m->h_cell_edge.assign(cell_edge, cell_edge + (size_t)n_cells * 3);
        s = m->d_cell_edge.upload(cell_edge, (size_t)n_cells * 3);
        if (s != EXM_OK) return s;
    }
    if (layers) {
        // entity columns: a cell's own range; a vertex or edge column spans
        // the union of the ranges of the cells around it
        m->variable = true;
        for (int d = 0; d < 3; ++d) {
            m->lo[d].assign(m->n[d], n_layers);
            m->hi[d].assign(m->n[d], 0);
        }
        std::vector<int32_t> lam(n_cells);
        for (int64_t c = 0; c < n_cells; ++c) {
            const int32_t b = layers[2 * c], t = layers[2 * c + 1];
            lam[c] = t - b;
            m->lo[2][c] = b;
            m->hi[2][c] = t;
            for (int a = 0; a < 3; ++a) {
                const int32_t v = cell_vertex[c * 3 + a];
                m->lo[0][v] = std::min(m->lo[0][v], b);
                m->hi[0][v] = std::max(m->hi[0][v], t);
                if (cell_edge) {
                    const int32_t e = cell_edge[c * 3 + a];
                    m->lo[1][e] = std::min(m->lo[1][e], b);
                    m->hi[1][e] = std::max(m->hi[1][e], t);
                }
            }
        }
        for (int32_t v = 0; v < n_vertices; ++v)
            EXM_CHECK(m->lo[0][v] < m->hi[0][v], EXM_EINVAL, "vertex %d belongs to no cell", v);
        if (!cell_edge) {
            m->lo[1].assign(m->n[1], 0);
            m->hi[1].assign(m->n[1], n_layers);
        }
        s = m->d_cell_lam.upload(lam.data(), lam.size());
        if (s != EXM_OK) return s;
        if ((s = m->d_cell_lo.upload(m->lo[2].data(), m->lo[2].size())) != EXM_OK) return s;
        if ((s = m->d_vert_lo.upload(m->lo[0].data(), m->lo[0].size())) != EXM_OK) return s;
        if ((s = m->d_vert_hi.upload(m->hi[0].data(), m->hi[0].size())) != EXM_OK) return s;
        if ((s = m->d_cell_hi.upload(m->hi[2].data(), m->hi[2].size())) != EXM_OK) return s;
        if (n_edges > 0) {
            if ((s = m->d_edge_lo.upload(m->lo[1].data(), m->lo[1].size())) != EXM_OK) return s;
            if ((s = m->d_edge_hi.upload(m->hi[1].data(), m->hi[1].size())) != EXM_OK) return s;
        }
    }
    *out = m.release();
    return EXM_OK;
}

int32_t exm_mesh_create(int32_t n_vertices, int32_t n_edges, int32_t n_cells, const int32_t* cell_vertex,
                        const int32_t* cell_edge, int32_t n_layers, exm_mesh** out)
{
    clear_error();
    return mesh_create(n_vertices, n_edges, n_cells, cell_vertex, cell_edge, n_layers, nullptr, out);
}

int32_t exm_mesh_create_var(int32_t n_vertices, int32_t n_edges, int32_t n_cells, const int32_t* cell_vertex,
                            const int32_t* cell_edge, int32_t n_layers, const int32_t* layers, exm_mesh** out)
{
    clear_error();
    EXM_CHECK(layers != nullptr, EXM_EINVAL, "layers is NULL");
    return mesh_create(n_vertices, n_edges, n_cells, cell_vertex, cell_edge, n_layers, layers, out);
}

int32_t exm_mesh_create_device(int32_t n_vertices, int32_t n_edges, int32_t n_cells, const int32_t* cell_vertex,
                               const int32_t* cell_edge, int32_t n_layers, const int32_t* layers, exm_mesh** out)
{
    clear_error();
    EXM_CHECK(out != nullptr, EXM_EINVAL, "out is NULL");
    *out = nullptr;
    EXM_CHECK(cell_vertex != nullptr, EXM_EINVAL, "cell_vertex is NULL");
    EXM_CHECK(n_vertices >= 3 && n_cells >= 1 && n_edges >= 0, EXM_ERANGE,
              "need n_vertices >= 3, n_cells >= 1, n_edges >= 0 (got %d, %d, %d)", n_vertices, n_cells, n_edges);
    int32_t s = check_pending();
    if (s != EXM_OK) return s;
    // The plans (colouring, tiles, fans) are built on the host, so the
    // adjacency comes back once; every array must be device memory.
    const int32_t* arrays[3] = {cell_vertex, cell_edge, layers};
    const char* names[3] = {"cell_vertex", "cell_edge", "layers"};
    const size_t counts[3] = {(size_t)n_cells * 3, (size_t)n_cells * 3, (size_t)n_cells * 2};
    std::vector<int32_t> host[3];
    for (int a = 0; a < 3; ++a) {
        if (!arrays[a]) continue;
        hipPointerAttribute_t attr;
        hipError_t e = hipPointerGetAttributes(&attr, arrays[a]);
        (void)hipGetLastError();   // an unknown (host) pointer leaves an error behind
        EXM_CHECK(e == hipSuccess && (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged),
                  EXM_EINVAL, "%s is not device memory", names[a]);
        host[a].resize(counts[a]);
        EXM_TRY_HIP(hipMemcpy(host[a].data(), arrays[a], counts[a] * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return mesh_create(n_vertices, n_edges, n_cells, host[0].data(), cell_edge ? host[1].data() : nullptr, n_layers,
                       layers ? host[2].data() : nullptr, out);
}

int32_t exm_mesh_entity_layers(const exm_mesh* mesh, int32_t d1, int32_t* lo, int32_t* hi)
{
    clear_error();
    EXM_CHECK(mesh != nullptr, EXM_EINVAL, "mesh is NULL");
    EXM_CHECK(d1 >= 0 && d1 <= 2, EXM_ERANGE, "d1 = %d outside [0, 2]", d1);
    for (int32_t i = 0; i < mesh->n[d1]; ++i) {
        if (lo) lo[i] = mesh->variable ? mesh->lo[d1][i] : 0;
        if (hi) hi[i] = mesh->variable ? mesh->hi[d1][i] : mesh->n_layers;
    }
    return EXM_OK;
}

void exm_mesh_destroy(exm_mesh* mesh) { delete mesh; }

static bool element_delta(int32_t element, int32_t d[6])
{
    for (int i = 0; i < 6; ++i) d[i] = 0;
    switch (element) {
    case EXM_ELEMENT_P1P1: d[0] = 1; return true;
    case EXM_ELEMENT_DG0DG0: d[5] = 1; return true;
    case EXM_ELEMENT_DG1DG1: d[5] = 6; return true;
    case EXM_ELEMENT_P2P2: d[0] = d[1] = d[2] = d[3] = 1; return true;
    case EXM_ELEMENT_P1DG0: d[1] = 1; return true;
    case EXM_ELEMENT_P1DG1: d[1] = 2; return true;
    case EXM_ELEMENT_DG0P1: d[4] = 1; return true;
    case EXM_ELEMENT_DG0DG1: d[5] = 2; return true;
    case EXM_ELEMENT_DG1P1: d[4] = 3; return true;
    case EXM_ELEMENT_DG1DG0: d[5] = 3; return true;
    default: return false;
    }
}

// Algorithm 1 with a layer range per entity column: column sizes differ, so
// the column starts are one exclusive prefix sum of the column sizes over the
// entities in the order Algorithm 1 visits them (dimension-major, then by
// index); the explicit list of a cell is that of its bottom prism, so that
// L(c) + l * offset still addresses layer l of the cell's column.  Built on
// the device: the sizes, the scan, then the lists and the int32 starts.

// Size of the column of entity i (levels lo .. hi, hi - lo layers).
__global__ void k_var_col_sizes(int32_t n, const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                                int32_t dh, int32_t dv, int64_t* __restrict__ size)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nl = (int64_t)hi[i] - lo[i];
    size[i] = (nl + 1) * dh + nl * dv;
}

__global__ void k_var_starts(int32_t n, const int64_t* __restrict__ start, int32_t has, int32_t* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = has ? (int32_t)start[i] : -1;
}

// One position of a cell's explicit list on columns of different heights:
// closure entity e (0..2 vertex, 3..5 edge, 6 cell), its DoFs per level
// (Algorithm 2's offset) and the DoF's place within the level.
struct VarPos {
    int32_t entity;
    int32_t per_level;
    int32_t shift;
};

// start: the column starts of all entities in visiting order (vertices, then
// edges from first_edge, then cells from first_cell); lo: the first level of
// every entity column, per dimension.
__global__ void k_var_bottom_map(int32_t n_cells, int32_t k, const VarPos* __restrict__ pos,
                                 const int32_t* __restrict__ cell_vertex, const int32_t* __restrict__ cell_edge,
                                 const int64_t* __restrict__ start, int64_t first_edge, int64_t first_cell,
                                 const int32_t* __restrict__ lo0, const int32_t* __restrict__ lo1,
                                 const int32_t* __restrict__ lo2, int32_t* __restrict__ map)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_cells * k) return;
    const int64_t c = t / k;
    const int32_t p = (int32_t)(t - c * k);
    const VarPos vp = pos[p];
    const int32_t b = lo2[c];   // the cell's first layer
    int64_t s;
    int32_t l;
    if (vp.entity < 3) {
        const int32_t v = cell_vertex[c * 3 + vp.entity];
        s = start[v];
        l = lo0[v];
    } else if (vp.entity < 6) {
        const int32_t e = cell_edge[c * 3 + vp.entity - 3];
        s = start[first_edge + e];
        l = lo1[e];
    } else {
        s = start[first_cell + c];
        l = b;
    }
    map[t] = (int32_t)(s + (int64_t)(b - l) * vp.per_level + vp.shift);
}

static int32_t space_create_var(const exm_mesh* mesh, const int32_t* delta, std::unique_ptr<exm_space> s,
                                hipStream_t hs, exm_space** out)
{
    const int64_t n0 = mesh->n[0], n1 = mesh->n[1], n2 = mesh->n[2];
    const int64_t ntot = n0 + n1 + n2;
    EXM_CHECK(ntot < INT32_MAX, EXM_EOVERFLOW, "%lld entity columns exceed the int32 range", (long long)ntot);
    DevBuf<int64_t> size, start;
    int32_t st;
    if ((st = size.alloc((size_t)ntot)) != EXM_OK) return st;
    if ((st = start.alloc((size_t)ntot)) != EXM_OK) return st;
    const int bs = 256;
    const int32_t* los[3] = {mesh->d_vert_lo.p, mesh->d_edge_lo.p, mesh->d_cell_lo.p};
    const int32_t* his[3] = {mesh->d_vert_hi.p, mesh->d_edge_hi.p, mesh->d_cell_hi.p};
    const int64_t first[3] = {0, n0, n0 + n1};
    for (int d = 0; d < 3; ++d) {
        const int32_t n = mesh->n[d];
        if (n == 0) continue;
        if (delta[2 * d] + delta[2 * d + 1] == 0) {   // no DoFs: columns of size 0
            EXM_TRY_HIP(hipMemsetAsync(size.p + first[d], 0, sizeof(int64_t) * (size_t)n, hs));
            continue;
        }
        EXM_CHECK(los[d] && his[d], EXM_EINVAL, "dimension %d carries DoFs but the mesh has no ranges for it", d);
        hipLaunchKernelGGL(k_var_col_sizes, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, hs, n, los[d], his[d],
                           delta[2 * d], delta[2 * d + 1], size.p + first[d]);
        EXM_TRY_HIP(hipGetLastError());
    }
    size_t tmp_bytes = 0;
    EXM_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, size.p, start.p, (int)ntot, hs));
    DevBuf<unsigned char> tmp;
    if ((st = tmp.alloc(tmp_bytes)) != EXM_OK) return st;
    EXM_TRY_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, size.p, start.p, (int)ntot, hs));
    // read back: the last start and size (the DoF count) and where each dimension begins
    int64_t last[2], dim0[3] = {0, -1, -1};
    EXM_TRY_HIP(hipMemcpyAsync(&last[0], start.p + ntot - 1, sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    EXM_TRY_HIP(hipMemcpyAsync(&last[1], size.p + ntot - 1, sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    for (int d = 1; d < 3; ++d)
        if (first[d] < ntot)
            EXM_TRY_HIP(hipMemcpyAsync(&dim0[d], start.p + first[d], sizeof(int64_t), hipMemcpyDeviceToHost, hs));
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    s->n_dofs = last[0] + last[1];
    EXM_CHECK(s->n_dofs < (int64_t)INT32_MAX, EXM_EOVERFLOW,
              "space has %lld DoFs; the int32 numbering allows at most %d", (long long)s->n_dofs, INT32_MAX - 1);
    for (int d = 0; d < 3; ++d) {
        s->base[d] = dim0[d] < 0 ? s->n_dofs : dim0[d];
        s->col_size[d] = -1;   // columns differ in size: the starts are a table
    }
    // stencil layout and offsets (Algorithm 2), as for uniform columns
    std::vector<VarPos> pos;
    for (int e = 0; e < 7; ++e) {
        const int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
        const int nh = delta[2 * d], nv = delta[2 * d + 1];
        for (int part = 0; part < 3; ++part) {
            const int cnt = part < 2 ? nh : nv;
            for (int j = 0; j < cnt; ++j) {
                // bottom level: j; top level: the next level's horizontal DoFs; vertical entity: after nh
                pos.push_back({e, nh + nv, (part == 1 ? nh + nv : (part == 2 ? nh : 0)) + j});
                s->offsets.push_back(nh + nv);
                s->entity_dim.push_back(d);
            }
        }
    }
    s->k = (int32_t)s->offsets.size();
    const int64_t nmap = n2 * s->k;
    if ((st = s->d_map.alloc((size_t)nmap)) != EXM_OK) return st;
    DevBuf<VarPos> dpos;
    if ((st = dpos.upload(pos.data(), pos.size())) != EXM_OK) return st;
    if (nmap > 0) {
        hipLaunchKernelGGL(k_var_bottom_map, dim3((unsigned)((nmap + bs - 1) / bs)), dim3(bs), 0, hs, mesh->n[2], s->k,
                           dpos.p, mesh->d_cell_vertex.p, mesh->d_cell_edge.p, start.p, first[1], first[2],
                           mesh->d_vert_lo.p, mesh->d_edge_lo.p, mesh->d_cell_lo.p, s->d_map.p);
        EXM_TRY_HIP(hipGetLastError());
    }
    for (int d = 0; d < 3; ++d) {
        const int32_t n = mesh->n[d];
        if (n == 0) continue;
        if ((st = s->d_starts[d].alloc((size_t)n)) != EXM_OK) return st;
        hipLaunchKernelGGL(k_var_starts, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, hs, n, start.p + first[d],
                           delta[2 * d] + delta[2 * d + 1] > 0 ? 1 : 0, s->d_starts[d].p);
        EXM_TRY_HIP(hipGetLastError());
    }
    // the scan buffers are freed on return: wait for the kernels that read them
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    *out = s.release();
    return EXM_OK;
}

int32_t exm_space_create(const exm_mesh* mesh, const int32_t* delta, int32_t element, void* stream,
                         exm_space** out)
{
    clear_error();
    EXM_CHECK(out != nullptr, EXM_EINVAL, "out is NULL");
    *out = nullptr;
    EXM_CHECK(mesh != nullptr && delta != nullptr, EXM_EINVAL, "mesh or delta is NULL");
    int32_t total = 0;
    for (int i = 0; i < 6; ++i) {
        EXM_CHECK(delta[i] >= 0 && delta[i] <= 64, EXM_ERANGE, "delta[%d] = %d outside [0, 64]", i, delta[i]);
        total += delta[i];
    }
    EXM_CHECK(total > 0, EXM_EINVAL, "delta table is all zero");
    if (element != EXM_ELEMENT_NONE) {
        int32_t want[6];
        EXM_CHECK(element_delta(element, want), EXM_EINVAL, "unknown element %d", element);
        for (int i = 0; i < 6; ++i)
            EXM_CHECK(want[i] == delta[i], EXM_EINVAL, "delta[%d] = %d does not match element %d (expects %d)", i,
                      delta[i], element, want[i]);
    }
    EXM_CHECK(delta[2] + delta[3] == 0 || !mesh->h_cell_edge.empty(), EXM_EINVAL,
              "space has DoFs on edges but the mesh has no cell_edge map");
    const int64_t lam = mesh->n_layers;
    auto s = std::make_unique<exm_space>();
    s->mesh = mesh;
    s->element = element;
    std::memcpy(s->delta, delta, sizeof(s->delta));
    if (mesh->variable) return space_create_var(mesh, delta, std::move(s), (hipStream_t)stream, out);
    int64_t base = 0;
    for (int d = 0; d < 3; ++d) {
        int64_t cs = (lam + 1) * delta[2 * d] + lam * delta[2 * d + 1];
        EXM_CHECK(cs < INT32_MAX, EXM_EOVERFLOW, "column size too large");
        s->col_size[d] = (int32_t)cs;
        s->base[d] = base;
        base += (int64_t)mesh->n[d] * cs;
    }
    s->n_dofs = base;
    EXM_CHECK(s->n_dofs < (int64_t)INT32_MAX, EXM_EOVERFLOW,
              "space has %lld DoFs; the int32 numbering allows at most %d", (long long)s->n_dofs, INT32_MAX - 1);
    // Stencil layout and Algorithm 2 offsets.
    std::vector<StencilPos> pos;
    for (int e = 0; e < 7; ++e) {
        int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
        int nh = delta[2 * d], nv = delta[2 * d + 1];
        for (int j = 0; j < nh; ++j) pos.push_back({e, j});                 // bottom level
        for (int j = 0; j < nh; ++j) pos.push_back({e, nh + nv + j});       // top level
        for (int j = 0; j < nv; ++j) pos.push_back({e, nh + j});            // vertical entity
        for (int j = 0; j < 2 * nh + nv; ++j) {
            s->offsets.push_back(nh + nv);
            s->entity_dim.push_back(d);
        }
    }
    s->k = (int32_t)pos.size();
    const int64_t nmap = (int64_t)mesh->n[2] * s->k;
    int32_t st = s->d_map.alloc((size_t)nmap);
    if (st != EXM_OK) return st;
    DevBuf<StencilPos> dpos;
    st = dpos.upload(pos.data(), pos.size());
    if (st != EXM_OK) return st;
    hipStream_t hs = (hipStream_t)stream;
    const int bs = 256;
    hipLaunchKernelGGL(k_bottom_map, dim3((unsigned)((nmap + bs - 1) / bs)), dim3(bs), 0, hs, mesh->n[2], s->k,
                       dpos.p, mesh->d_cell_vertex.p, mesh->d_cell_edge.p, s->base[0], s->base[1], s->base[2],
                       s->col_size[0], s->col_size[1], s->col_size[2], s->d_map.p);
    EXM_TRY_HIP(hipGetLastError());
    for (int d = 0; d < 3; ++d) {
        const int32_t n = mesh->n[d];
        if (n == 0) continue;
        st = s->d_starts[d].alloc((size_t)n);
        if (st != EXM_OK) return st;
        hipLaunchKernelGGL(k_column_starts, dim3((n + bs - 1) / bs), dim3(bs), 0, hs, n, s->base[d], s->col_size[d],
                           s->d_starts[d].p);
        EXM_TRY_HIP(hipGetLastError());
    }
    // dpos is freed on return: wait for the kernel that reads it.
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    *out = s.release();
    return EXM_OK;
}

int32_t exm_space_info(const exm_space* space, int64_t* n_dofs, int32_t* arity)
{
    clear_error();
    EXM_CHECK(space != nullptr, EXM_EINVAL, "space is NULL");
    if (n_dofs) *n_dofs = space->n_dofs;
    if (arity) *arity = space->k;
    return EXM_OK;
}

int32_t exm_space_create_mixed(const exm_mesh* mesh, const int32_t* dofs_v, const int32_t* dofs_e,
                               const int32_t* dofs_c, int32_t element, void* stream, exm_space** out)
{
    clear_error();
    EXM_CHECK(mesh != nullptr && out != nullptr, EXM_EINVAL, "mesh or out is NULL");
    EXM_CHECK(dofs_v != nullptr && dofs_c != nullptr, EXM_EINVAL, "dofs_v or dofs_c is NULL");
    EXM_CHECK(!mesh->variable, EXM_EUNSUPPORTED, "a DoF count per entity takes meshes with one layer count");
    EXM_CHECK(element == EXM_ELEMENT_NONE || element == EXM_ELEMENT_DGMIX, EXM_EINVAL,
              "element %d: a space with a DoF count per entity is EXM_ELEMENT_NONE or EXM_ELEMENT_DGMIX", element);
    const int32_t* dofs[3] = {dofs_v, dofs_e, dofs_c};
    for (int d = 0; d < 3; ++d) {
        if (!dofs[d]) continue;
        for (int64_t i = 0; i < 2 * (int64_t)mesh->n[d]; ++i)
            EXM_CHECK(dofs[d][i] >= 0 && dofs[d][i] <= 64, EXM_ERANGE, "dofs of entity %lld (dimension %d) = %d "
                      "outside [0, 64]", (long long)(i / 2), d, dofs[d][i]);
    }
    bool edge_dofs = false;
    if (dofs_e)
        for (int64_t i = 0; i < 2 * (int64_t)mesh->n[1] && !edge_dofs; ++i) edge_dofs = dofs_e[i] > 0;
    EXM_CHECK(!edge_dofs || !mesh->h_cell_edge.empty(), EXM_EINVAL,
              "edges carry DoFs but the mesh has no cell_edge map");
    if (element == EXM_ELEMENT_DGMIX) {
        for (int64_t i = 0; i < 2 * (int64_t)mesh->n[0]; ++i)
            EXM_CHECK(dofs_v[i] == 0, EXM_EINVAL, "EXM_ELEMENT_DGMIX: vertex DoFs must be 0");
        EXM_CHECK(!edge_dofs, EXM_EINVAL, "EXM_ELEMENT_DGMIX: edge DoFs must be 0");
        for (int32_t c = 0; c < mesh->n[2]; ++c)
            EXM_CHECK(dofs_c[2 * c] == 0 && (dofs_c[2 * c + 1] == 1 || dofs_c[2 * c + 1] == 6), EXM_EINVAL,
                      "EXM_ELEMENT_DGMIX: cell %d carries (%d, %d); use (0, 1) or (0, 6)", c, dofs_c[2 * c],
                      dofs_c[2 * c + 1]);
    }
    const int64_t lam = mesh->n_layers;
    auto s = std::make_unique<exm_space>();
    s->mesh = mesh;
    s->element = element;
    s->mixed = true;
    auto nh = [&](int d, int64_t i) { return dofs[d] ? dofs[d][2 * i] : 0; };
    auto nv = [&](int d, int64_t i) { return dofs[d] ? dofs[d][2 * i + 1] : 0; };
    // Algorithm 1: column starts as a prefix sum over the entities in visiting order
    std::vector<int64_t> start[3];
    int64_t c = 0;
    for (int d = 0; d < 3; ++d) {
        s->base[d] = c;
        s->col_size[d] = -1;   // columns differ in size
        start[d].resize(mesh->n[d]);
        for (int32_t i = 0; i < mesh->n[d]; ++i) {
            start[d][i] = c;
            c += (lam + 1) * nh(d, i) + lam * nv(d, i);
        }
    }
    s->n_dofs = c;
    EXM_CHECK(s->n_dofs < (int64_t)INT32_MAX, EXM_EOVERFLOW,
              "space has %lld DoFs; the int32 numbering allows at most %d", (long long)s->n_dofs, INT32_MAX - 1);
    // lists of layer 0, cell by cell, with the vertical offset of every entry
    const int32_t ncell = mesh->n[2];
    const int32_t* cv = mesh->h_cell_vertex.data();
    const int32_t* ce = mesh->h_cell_edge.empty() ? nullptr : mesh->h_cell_edge.data();
    std::vector<int32_t> off(ncell + 1, 0), map, eoff;
    int32_t kmax = 0;
    for (int32_t cell = 0; cell < ncell; ++cell) {
        for (int ent = 0; ent < 7; ++ent) {
            const int d = ent < 3 ? 0 : (ent < 6 ? 1 : 2);
            if (d == 1 && !ce) continue;
            const int32_t i = d == 0 ? cv[cell * 3 + ent] : (d == 1 ? ce[cell * 3 + (ent - 3)] : cell);
            const int h = nh(d, i), v = nv(d, i);
            const int64_t S = start[d][i];
            for (int j = 0; j < h; ++j) { map.push_back((int32_t)(S + j)); eoff.push_back(h + v); }           // bottom
            for (int j = 0; j < h; ++j) { map.push_back((int32_t)(S + h + v + j)); eoff.push_back(h + v); }   // top
            for (int j = 0; j < v; ++j) { map.push_back((int32_t)(S + h + j)); eoff.push_back(h + v); }       // vertical
        }
        EXM_CHECK(map.size() < (size_t)INT32_MAX, EXM_EOVERFLOW, "lists exceed the int32 range");
        off[cell + 1] = (int32_t)map.size();
        kmax = std::max(kmax, off[cell + 1] - off[cell]);
    }
    s->k = kmax;
    s->list_total = (int64_t)map.size();
    int32_t st;
    if ((st = s->d_map.upload(map.data(), map.size())) != EXM_OK) return st;
    if ((st = s->d_list_off.upload(off.data(), off.size())) != EXM_OK) return st;
    if ((st = s->d_entry_off.upload(eoff.data(), eoff.size())) != EXM_OK) return st;
    for (int d = 0; d < 3; ++d) {
        if (mesh->n[d] == 0) continue;
        std::vector<int32_t> h(mesh->n[d]);
        for (int32_t i = 0; i < mesh->n[d]; ++i) h[i] = (int32_t)start[d][i];
        if ((st = s->d_starts[d].upload(h.data(), h.size())) != EXM_OK) return st;
    }
    (void)stream;
    *out = s.release();
    return EXM_OK;
}

int32_t exm_space_list_size(const exm_space* space, int64_t* total)
{
    clear_error();
    EXM_CHECK(space != nullptr && total != nullptr, EXM_EINVAL, "space or total is NULL");
    *total = space->mixed ? space->list_total : (int64_t)space->mesh->n[2] * space->k;
    return EXM_OK;
}

__global__ void k_uniform_lists(int32_t n_cells, int32_t k, const int32_t* __restrict__ offsets, int32_t* list_off,
                                int32_t* entry_off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n_cells) list_off[i] = (int32_t)(i * k);
    if (i < (int64_t)n_cells * k) entry_off[i] = offsets[i % k];
}

int32_t exm_space_lists(const exm_space* space, int32_t* list_off, int32_t* lists, int32_t* entry_offsets,
                        void* stream)
{
    clear_error();
    EXM_CHECK(space != nullptr && list_off != nullptr, EXM_EINVAL, "space or list_off is NULL");
    int64_t total = 0;
    int32_t st = exm_space_list_size(space, &total);
    if (st != EXM_OK) return st;
    EXM_CHECK(total == 0 || (lists != nullptr && entry_offsets != nullptr), EXM_EINVAL, "lists or entry_offsets is NULL");
    hipStream_t hs = (hipStream_t)stream;
    const int32_t nc = space->mesh->n[2];
    if (total) EXM_TRY_HIP(hipMemcpyAsync(lists, space->d_map.p, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToDevice, hs));
    if (space->mixed) {
        EXM_TRY_HIP(hipMemcpyAsync(list_off, space->d_list_off.p, sizeof(int32_t) * (size_t)(nc + 1),
                                   hipMemcpyDeviceToDevice, hs));
        if (total)
            EXM_TRY_HIP(hipMemcpyAsync(entry_offsets, space->d_entry_off.p, sizeof(int32_t) * (size_t)total,
                                       hipMemcpyDeviceToDevice, hs));
        return EXM_OK;
    }
    DevBuf<int32_t> offs;
    if ((st = offs.upload(space->offsets.data(), space->offsets.size())) != EXM_OK) return st;
    const int64_t n = std::max<int64_t>(nc + 1, total);
    const int bs = 256;
    hipLaunchKernelGGL(k_uniform_lists, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, hs, nc, space->k,
                       offs.p, list_off, entry_offsets);
    EXM_TRY_HIP(hipGetLastError());
    // offs is freed on return: wait for the kernel that reads it
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    return EXM_OK;
}

int32_t exm_space_offsets(const exm_space* space, int32_t* offsets)
{
    clear_error();
    EXM_CHECK(space != nullptr && offsets != nullptr, EXM_EINVAL, "space or offsets is NULL");
    EXM_CHECK(!space->mixed, EXM_EUNSUPPORTED, "the space has a DoF count per entity: use exm_space_lists");
    std::memcpy(offsets, space->offsets.data(), sizeof(int32_t) * space->offsets.size());
    return EXM_OK;
}

int32_t exm_space_column_starts(const exm_space* space, int32_t d1, int32_t* dst, void* stream)
{
    clear_error();
    EXM_CHECK(space != nullptr && dst != nullptr, EXM_EINVAL, "space or dst is NULL");
    EXM_CHECK(d1 >= 0 && d1 <= 2, EXM_ERANGE, "d1 = %d outside [0, 2]", d1);
    const int32_t n = space->mesh->n[d1];
    if (n == 0) return EXM_OK;
    // the starts the space keeps (closed form, or a prefix sum over the ranges of a variable mesh)
    EXM_TRY_HIP(hipMemcpyAsync(dst, space->d_starts[d1].p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
    return EXM_OK;
}

int32_t exm_space_bottom_map(const exm_space* space, int32_t* dst, void* stream)
{
    clear_error();
    EXM_CHECK(space != nullptr && dst != nullptr, EXM_EINVAL, "space or dst is NULL");
    EXM_CHECK(!space->mixed, EXM_EUNSUPPORTED, "the space has a DoF count per entity: use exm_space_lists");
    size_t bytes = sizeof(int32_t) * space->d_map.n;
    if (bytes)
        EXM_TRY_HIP(hipMemcpyAsync(dst, space->d_map.p, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return EXM_OK;
}

void exm_space_destroy(exm_space* space) { delete space; }

int32_t exm_mesh_colours(const exm_mesh* mesh, int32_t* n_colours)
{
    clear_error();
    EXM_CHECK(mesh != nullptr && n_colours != nullptr, EXM_EINVAL, "mesh or n_colours is NULL");
    const Colouring* c = nullptr;
    int32_t s = build_colouring(mesh, &c);
    if (s != EXM_OK) return s;
    *n_colours = c->n_colours;
    return EXM_OK;
}

int32_t exm_stream_triad(double* a, const double* b, const double* c, double alpha, int64_t n, int32_t block,
                         int32_t grid, void* stream)
{
    clear_error();
    EXM_CHECK(a && b && c, EXM_EINVAL, "null array");
    EXM_CHECK(a != b && a != c && b != c, EXM_EINVAL, "arrays must be distinct");
    EXM_CHECK(n >= 0, EXM_ERANGE, "n < 0");
    EXM_CHECK(block >= 64 && block <= 1024 && block % 64 == 0, EXM_ERANGE, "block = %d not a multiple of 64 in [64, 1024]", block);
    EXM_CHECK(grid >= 0, EXM_ERANGE, "grid < 0");
    if (n == 0) return EXM_OK;
    const bool pairs = (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) == 0 && n >= 2;
    const int64_t items = pairs ? n / 2 : n;
    int64_t g = grid ? grid : (items + block - 1) / block;
    EXM_CHECK(g <= INT32_MAX, EXM_ERANGE, "grid too large");
    if (pairs)
        hipLaunchKernelGGL(k_triad2, dim3((unsigned)g), dim3(block), 0, (hipStream_t)stream, a, b, c, alpha, n);
    else
        hipLaunchKernelGGL(k_triad, dim3((unsigned)g), dim3(block), 0, (hipStream_t)stream, a, b, c, alpha, n);
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

}  // extern "C"
