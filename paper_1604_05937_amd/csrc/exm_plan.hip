// Tile plans for the LDS-staged column loop (host code).
//
// A tile is a compact group of base cells grown by breadth-first search over
// the cells sharing a vertex, seeded at the lowest-numbered unassigned cell, so
// it follows the locality of the base ordering.  For every tile the plan lists
// the base vertices (and, if asked, edges) its cells touch; each is flagged
// when another tile touches it too.  Tiles are also greedily coloured so that
// tiles of one colour share no vertex.
#include <algorithm>
#include <cstring>
#include <deque>

#include "exm_internal.hpp"

namespace exm {

namespace {

struct Csr {
    std::vector<int64_t> start;
    std::vector<int32_t> items;
};

Csr vertex_cells(const exm_mesh* m)
{
    const int32_t nv = m->n[0], nc = m->n[2];
    const int32_t* cv = m->h_cell_vertex.data();
    Csr r;
    r.start.assign(nv + 1, 0);
    for (int64_t i = 0; i < (int64_t)nc * 3; ++i) r.start[cv[i] + 1]++;
    for (int32_t v = 0; v < nv; ++v) r.start[v + 1] += r.start[v];
    r.items.resize(r.start[nv]);
    std::vector<int64_t> fill(r.start.begin(), r.start.end() - 1);
    for (int32_t c = 0; c < nc; ++c)
        for (int a = 0; a < 3; ++a) r.items[fill[cv[c * 3 + a]]++] = c;
    return r;
}

}  // namespace

int32_t build_tile_plan(const exm_mesh* m, int32_t target, const TilePlan** out)
{
    std::lock_guard<std::mutex> lock(m->mu);
    for (auto& p : m->plans)
        if (p->target == target && !p->owner) {
            *out = p.get();
            return EXM_OK;
        }
    const int32_t nv = m->n[0], ne = m->n[1], nc = m->n[2];
    const int32_t* cv = m->h_cell_vertex.data();
    const bool edges = !m->h_cell_edge.empty();
    const int32_t* ce = edges ? m->h_cell_edge.data() : nullptr;
    Csr vc = vertex_cells(m);

    // 1. grow tiles
    std::vector<int32_t> tile_of(nc, -1);
    auto plan = std::make_unique<TilePlan>();
    plan->target = target;
    std::vector<int32_t> order;
    order.reserve(nc);
    std::vector<int64_t> tile_cell_off(1, 0);
    std::deque<int32_t> q;
    int32_t nt = 0;
    for (int32_t s = 0; s < nc; ++s) {
        if (tile_of[s] >= 0) continue;
        int32_t cnt = 0;
        q.clear();
        q.push_back(s);
        tile_of[s] = nt;
        order.push_back(s);
        ++cnt;
        while (!q.empty() && cnt < target) {
            const int32_t c = q.front();
            q.pop_front();
            // vertex neighbours: cells sharing a vertex with c.  Growing over
            // edge neighbours only leaves pockets between earlier tiles that
            // later tiles cannot fill: on triangulated squares that gives
            // tiles of about 40 cells for a target of 64, with more vertices
            // per cell; over vertex neighbours the tiles fill.
            for (int a = 0; a < 3 && cnt < target; ++a) {
                const int32_t p = cv[c * 3 + a];
                for (int64_t j = vc.start[p]; j < vc.start[p + 1] && cnt < target; ++j) {
                    const int32_t o = vc.items[j];
                    if (tile_of[o] >= 0) continue;
                    tile_of[o] = nt;
                    order.push_back(o);
                    q.push_back(o);
                    ++cnt;
                }
            }
        }
        tile_cell_off.push_back((int64_t)order.size());
        ++nt;
    }
    plan->n_tiles = nt;

    // 2. per-tile vertex and edge lists with local indices
    std::vector<int32_t> touch_v(nv, 0), touch_e(edges ? ne : 0, 0);
    std::vector<int32_t> stamp_v(nv, -1), local_v(nv, 0), stamp_e(edges ? ne : 0, -1), local_e(edges ? ne : 0, 0);
    std::vector<int64_t> voff(1, 0), eoff(1, 0);
    std::vector<int32_t> verts, edgs;
    std::vector<uint16_t> lcv((size_t)nc * 3), lce(edges ? (size_t)nc * 3 : 0);
    int32_t maxc = 0, maxv = 0, maxe = 0;
    for (int32_t t = 0; t < nt; ++t) {
        const int64_t b = tile_cell_off[t], e = tile_cell_off[t + 1];
        maxc = std::max<int32_t>(maxc, (int32_t)(e - b));
        int32_t nvl = 0, nel = 0;
        for (int64_t i = b; i < e; ++i) {
            const int32_t c = order[i];
            for (int a = 0; a < 3; ++a) {
                const int32_t v = cv[(int64_t)c * 3 + a];
                if (stamp_v[v] != t) {
                    stamp_v[v] = t;
                    local_v[v] = nvl++;
                    verts.push_back(v);
                    touch_v[v]++;
                }
                lcv[(size_t)i * 3 + a] = (uint16_t)local_v[v];
                if (edges) {
                    const int32_t g = ce[(int64_t)c * 3 + a];
                    if (stamp_e[g] != t) {
                        stamp_e[g] = t;
                        local_e[g] = nel++;
                        edgs.push_back(g);
                        touch_e[g]++;
                    }
                    lce[(size_t)i * 3 + a] = (uint16_t)local_e[g];
                }
            }
        }
        EXM_CHECK(nvl < 65535 && nel < 65535, EXM_ERANGE, "tile too large");
        maxv = std::max(maxv, nvl);
        maxe = std::max(maxe, nel);
        voff.push_back((int64_t)verts.size());
        eoff.push_back((int64_t)edgs.size());
    }
    plan->max_cells = maxc;
    plan->max_verts = maxv;
    plan->max_edges = maxe;
    // shared flag in bit 31 of the stored id
    std::vector<int32_t> vflag(verts.size()), eflag(edgs.size());
    int64_t shared_v = 0;
    for (size_t i = 0; i < verts.size(); ++i) {
        const bool sh = touch_v[verts[i]] > 1;
        shared_v += sh;
        vflag[i] = verts[i] | (sh ? (int32_t)0x80000000 : 0);
    }
    for (size_t i = 0; i < edgs.size(); ++i) eflag[i] = edgs[i] | (touch_e[edgs[i]] > 1 ? (int32_t)0x80000000 : 0);
    plan->n_tile_verts = (int64_t)verts.size();
    plan->n_shared_verts = shared_v;
    for (int32_t v = 0; v < nv; ++v)
        if (touch_v[v] != 1) plan->zero_verts.push_back(v);

    // 3. greedy tile colouring: tiles sharing a vertex differ in colour
    std::vector<int32_t> tcol(nt, -1), mark;
    int32_t ncol = 0;
    for (int32_t t = 0; t < nt; ++t) {
        for (int64_t i = voff[t]; i < voff[t + 1]; ++i) {
            const int32_t v = verts[i];
            for (int64_t j = vc.start[v]; j < vc.start[v + 1]; ++j) {
                const int32_t o = tcol[tile_of[vc.items[j]]];
                if (o >= 0) mark[o] = t;
            }
        }
        int32_t col = 0;
        while (col < ncol && mark[col] == t) ++col;
        if (col == ncol) {
            ++ncol;
            mark.push_back(-1);
        }
        tcol[t] = col;
    }
    plan->n_colours = ncol;
    plan->colour_off.assign(ncol + 1, 0);
    for (int32_t t = 0; t < nt; ++t) plan->colour_off[tcol[t] + 1]++;
    for (int32_t k = 0; k < ncol; ++k) plan->colour_off[k + 1] += plan->colour_off[k];
    std::vector<int32_t> tiles_by_colour(nt);
    {
        std::vector<int64_t> f(plan->colour_off.begin(), plan->colour_off.end() - 1);
        for (int32_t t = 0; t < nt; ++t) tiles_by_colour[f[tcol[t]]++] = t;
    }

    // 4. device copies
    std::vector<int32_t> tco(tile_cell_off.begin(), tile_cell_off.end());
    std::vector<int32_t> vo(voff.begin(), voff.end()), eo(eoff.begin(), eoff.end());
    EXM_CHECK(tile_cell_off.back() < INT32_MAX && voff.back() < INT32_MAX && eoff.back() < INT32_MAX, EXM_EOVERFLOW,
              "plan too large");
    int32_t s;
    if ((s = plan->cell_off.upload(tco.data(), tco.size())) != EXM_OK) return s;
    if ((s = plan->cells.upload(order.data(), order.size())) != EXM_OK) return s;
    if ((s = plan->vert_off.upload(vo.data(), vo.size())) != EXM_OK) return s;
    if ((s = plan->verts.upload(vflag.data(), vflag.size())) != EXM_OK) return s;
    if ((s = plan->local_cv.upload(lcv.data(), lcv.size())) != EXM_OK) return s;
    if (edges) {
        if ((s = plan->edge_off.upload(eo.data(), eo.size())) != EXM_OK) return s;
        if ((s = plan->edges.upload(eflag.data(), eflag.size())) != EXM_OK) return s;
        if ((s = plan->local_ce.upload(lce.data(), lce.size())) != EXM_OK) return s;
    }
    if ((s = plan->colour_tiles.upload(tiles_by_colour.data(), tiles_by_colour.size())) != EXM_OK) return s;
    plan->has_edges = edges;
    m->plans.push_back(std::move(plan));
    *out = m->plans.back().get();
    return EXM_OK;
}

// Owner plan: the base vertices are split into compact tiles of about
// target / 2 vertices (a triangulation has about half as many vertices as
// cells), grown breadth-first over the vertex graph from the lowest-numbered
// unassigned vertex.  A tile owns its vertices: it is the only one that sums
// and writes their columns.  Its cell list holds every cell with an owned
// vertex, so a cell on a tile boundary appears in each tile that owns one of
// its vertices and is computed there again; its vertex list holds the owned
// vertices first, then the other vertices of those cells (read, never
// written).
int32_t build_owner_plan(const exm_mesh* m, int32_t target, const TilePlan** out)
{
    std::lock_guard<std::mutex> lock(m->mu);
    for (auto& p : m->plans)
        if (p->target == target && p->owner) {
            *out = p.get();
            return EXM_OK;
        }
    const int32_t nv = m->n[0], nc = m->n[2];
    const int32_t* cv = m->h_cell_vertex.data();
    Csr vc = vertex_cells(m);
    const int32_t tv = std::max(1, target / 2);

    // 1. grow vertex tiles over the vertex graph (vertices sharing a cell)
    std::vector<int32_t> tile_of(nv, -1), vorder;
    vorder.reserve(nv);
    std::vector<int64_t> own_off(1, 0);
    std::deque<int32_t> q;
    int32_t nt = 0;
    for (int32_t s0 = 0; s0 < nv; ++s0) {
        if (tile_of[s0] >= 0) continue;
        int32_t cnt = 0;
        q.clear();
        q.push_back(s0);
        tile_of[s0] = nt;
        vorder.push_back(s0);
        ++cnt;
        while (!q.empty() && cnt < tv) {
            const int32_t v = q.front();
            q.pop_front();
            for (int64_t jx = vc.start[v]; jx < vc.start[v + 1] && cnt < tv; ++jx) {
                const int32_t c = vc.items[jx];
                for (int a = 0; a < 3 && cnt < tv; ++a) {
                    const int32_t w = cv[(int64_t)c * 3 + a];
                    if (tile_of[w] >= 0) continue;
                    tile_of[w] = nt;
                    vorder.push_back(w);
                    q.push_back(w);
                    ++cnt;
                }
            }
        }
        own_off.push_back((int64_t)vorder.size());
        ++nt;
    }

    // 2. per tile: cells touching an owned vertex, vertex list (owned first)
    auto plan = std::make_unique<TilePlan>();
    plan->target = target;
    plan->owner = true;
    plan->n_tiles = nt;
    std::vector<int32_t> cstamp(nc, -1), vstamp(nv, -1), local(nv, 0);
    std::vector<int32_t> cells, verts, owned(nt);
    std::vector<int64_t> coff(1, 0), voff(1, 0);
    std::vector<uint16_t> lcv;
    int32_t maxc = 0, maxv = 0;
    for (int32_t t = 0; t < nt; ++t) {
        int32_t nvl = 0;
        for (int64_t i = own_off[t]; i < own_off[t + 1]; ++i) {
            const int32_t v = vorder[i];
            vstamp[v] = t;
            local[v] = nvl++;
            verts.push_back(v);
        }
        owned[t] = nvl;
        const int64_t c0 = (int64_t)cells.size();
        for (int64_t i = own_off[t]; i < own_off[t + 1]; ++i) {
            const int32_t v = vorder[i];
            for (int64_t jx = vc.start[v]; jx < vc.start[v + 1]; ++jx) {
                const int32_t c = vc.items[jx];
                if (cstamp[c] == t) continue;
                cstamp[c] = t;
                cells.push_back(c);
                for (int a = 0; a < 3; ++a) {
                    const int32_t w = cv[(int64_t)c * 3 + a];
                    if (vstamp[w] != t) {
                        vstamp[w] = t;
                        local[w] = nvl++;
                        verts.push_back(w);
                    }
                    lcv.push_back((uint16_t)local[w]);
                }
            }
        }
        EXM_CHECK(nvl < 65535, EXM_ERANGE, "tile too large");
        maxc = std::max<int32_t>(maxc, (int32_t)((int64_t)cells.size() - c0));
        maxv = std::max(maxv, nvl);
        coff.push_back((int64_t)cells.size());
        voff.push_back((int64_t)verts.size());
    }
    plan->max_cells = maxc;
    plan->max_verts = maxv;
    plan->max_edges = 0;
    plan->n_tile_verts = (int64_t)verts.size();
    plan->n_shared_verts = 0;
    plan->n_cell_entries = (int64_t)cells.size();
    plan->n_colours = 1;
    plan->colour_off = {0, nt};

    EXM_CHECK(coff.back() < INT32_MAX && voff.back() < INT32_MAX, EXM_EOVERFLOW, "plan too large");
    std::vector<int32_t> co(coff.begin(), coff.end()), vo(voff.begin(), voff.end()), all(nt);
    for (int32_t t = 0; t < nt; ++t) all[t] = t;
    int32_t s;
    if ((s = plan->cell_off.upload(co.data(), co.size())) != EXM_OK) return s;
    if ((s = plan->cells.upload(cells.data(), cells.size())) != EXM_OK) return s;
    if ((s = plan->vert_off.upload(vo.data(), vo.size())) != EXM_OK) return s;
    if ((s = plan->verts.upload(verts.data(), verts.size())) != EXM_OK) return s;
    if ((s = plan->local_cv.upload(lcv.data(), lcv.size())) != EXM_OK) return s;
    if ((s = plan->owned.upload(owned.data(), owned.size())) != EXM_OK) return s;
    if ((s = plan->colour_tiles.upload(all.data(), all.size())) != EXM_OK) return s;
    plan->has_edges = false;
    m->plans.push_back(std::move(plan));
    *out = m->plans.back().get();
    return EXM_OK;
}

}  // namespace exm

// ---------------------------------------------------------------------------
// Read-out of the plans, so that callers and tests can check them.

using namespace exm;

namespace {

template <class T>
int32_t copy_back(T* dst, const DevBuf<T>& src, size_t count)
{
    if (!dst || count == 0) return EXM_OK;
    EXM_CHECK(src.p != nullptr && src.n >= count, EXM_EINVAL, "plan array missing");
    EXM_TRY_HIP(hipMemcpy(dst, src.p, count * sizeof(T), hipMemcpyDeviceToHost));
    return EXM_OK;
}

int32_t find_plan(const exm_mesh* m, int32_t kind, int32_t target, const Colouring** col, const TilePlan** plan)
{
    *col = nullptr;
    *plan = nullptr;
    EXM_CHECK(m != nullptr, EXM_EINVAL, "mesh is NULL");
    switch (kind) {
    case EXM_PLAN_CELL_COLOURS: return build_colouring(m, col);
    case EXM_PLAN_TILES:
        EXM_CHECK(target >= 1 && target <= 65536, EXM_ERANGE, "target = %d outside [1, 65536]", target);
        return build_tile_plan(m, target, plan);
    case EXM_PLAN_OWNER:
        EXM_CHECK(target >= 2 && target <= 65536, EXM_ERANGE, "target = %d outside [2, 65536]", target);
        return build_owner_plan(m, target, plan);
    default: return fail(EXM_EINVAL, "unknown plan kind %d", kind);
    }
}

}  // namespace

extern "C" {

int32_t exm_mesh_plan_info(const exm_mesh* mesh, int32_t kind, int32_t target, exm_plan_info* info)
{
    clear_error();
    EXM_CHECK(info != nullptr, EXM_EINVAL, "info is NULL");
    const Colouring* col;
    const TilePlan* plan;
    int32_t s = find_plan(mesh, kind, target, &col, &plan);
    if (s != EXM_OK) return s;
    std::memset(info, 0, sizeof(*info));
    if (col) {
        info->n_units = mesh->n[2];
        info->n_colours = col->n_colours;
        info->n_cell_entries = mesh->n[2];
        info->n_vert_entries = (int64_t)mesh->n[2] * 3;
        return EXM_OK;
    }
    info->n_units = plan->n_tiles;
    info->n_colours = plan->n_colours;
    info->n_cell_entries = (int64_t)plan->cells.n;
    info->n_vert_entries = plan->n_tile_verts;
    info->n_edge_entries = plan->has_edges ? (int64_t)plan->edges.n : 0;
    return EXM_OK;
}

int32_t exm_mesh_plan_read(const exm_mesh* mesh, int32_t kind, int32_t target, const exm_plan_arrays* out)
{
    clear_error();
    EXM_CHECK(out != nullptr, EXM_EINVAL, "out is NULL");
    int32_t s = check_pending();
    if (s != EXM_OK) return s;
    const Colouring* col;
    const TilePlan* plan;
    if ((s = find_plan(mesh, kind, target, &col, &plan)) != EXM_OK) return s;
    const int32_t nc = mesh->n[2];
    const int32_t* cv = mesh->h_cell_vertex.data();
    if (col) {
        // units are single cells, in base order
        for (int32_t k = 0; k < col->n_colours; ++k)
            for (int64_t i = col->offsets[k]; i < col->offsets[k + 1]; ++i)
                if (out->colour) out->colour[col->host_cells[i]] = k;
        for (int32_t c = 0; c < nc; ++c) {
            if (out->cell_off) out->cell_off[c] = c;
            if (out->cells) out->cells[c] = c;
            if (out->vert_off) out->vert_off[c] = 3 * c;
            for (int a = 0; a < 3; ++a) {
                if (out->verts) out->verts[3 * (int64_t)c + a] = cv[3 * (int64_t)c + a];
                if (out->local_cv) out->local_cv[3 * (int64_t)c + a] = (uint16_t)a;
            }
            if (out->owned) out->owned[c] = 0;
        }
        if (out->cell_off) out->cell_off[nc] = nc;
        if (out->vert_off) out->vert_off[nc] = 3 * nc;
        EXM_CHECK(!out->edge_off && !out->edges && !out->local_ce, EXM_EINVAL, "the cell colouring lists no edges");
        return EXM_OK;
    }
    const int32_t nt = plan->n_tiles;
    if (out->colour) {
        std::vector<int32_t> by_colour(nt);
        if ((s = copy_back(by_colour.data(), plan->colour_tiles, (size_t)nt)) != EXM_OK) return s;
        for (int32_t k = 0; k < plan->n_colours; ++k)
            for (int64_t i = plan->colour_off[k]; i < plan->colour_off[k + 1]; ++i) out->colour[by_colour[i]] = k;
    }
    if ((s = copy_back(out->cell_off, plan->cell_off, (size_t)nt + 1)) != EXM_OK) return s;
    if ((s = copy_back(out->cells, plan->cells, plan->cells.n)) != EXM_OK) return s;
    if ((s = copy_back(out->vert_off, plan->vert_off, (size_t)nt + 1)) != EXM_OK) return s;
    if ((s = copy_back(out->verts, plan->verts, plan->verts.n)) != EXM_OK) return s;
    if ((s = copy_back(out->local_cv, plan->local_cv, plan->local_cv.n)) != EXM_OK) return s;
    if (out->owned) {
        if (plan->owner) {
            if ((s = copy_back(out->owned, plan->owned, (size_t)nt)) != EXM_OK) return s;
        } else {
            for (int32_t t = 0; t < nt; ++t) out->owned[t] = 0;
        }
    }
    if (out->edge_off || out->edges || out->local_ce) {
        EXM_CHECK(plan->has_edges, EXM_EINVAL, "this plan lists no edges (the mesh has no cell_edge, or owner plan)");
        if ((s = copy_back(out->edge_off, plan->edge_off, (size_t)nt + 1)) != EXM_OK) return s;
        if ((s = copy_back(out->edges, plan->edges, plan->edges.n)) != EXM_OK) return s;
        if ((s = copy_back(out->local_ce, plan->local_ce, plan->local_ce.n)) != EXM_OK) return s;
    }
    return EXM_OK;
}

}  // extern "C"
