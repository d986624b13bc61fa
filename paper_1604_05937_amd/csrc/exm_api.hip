// exm_par_loop: argument validation, launch-shape selection, race strategy,
// and the autotuner.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <tuple>

#include "exm_internal.hpp"

namespace exm {

// ---------------------------------------------------------------------------
// Launch shapes.  cols_per_wave = cpw columns share a wavefront; each gets
// seg = 64 / cpw lanes.  A column of lambda layers takes ceil(lambda / seg)
// steps, so the fraction of busy lanes is cpw lambda / (64 ceil(lambda / seg)).

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
    // Wider groups of lanes per column keep the accesses coalesced; consider
    // at most four columns per wavefront (16 lanes = 128 bytes of FP64).
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
    exm_loop_opts tuned;
    if (lookup_tuned(kernel, element, n_layers, n_cells, &tuned)) s = make_shape(tuned.cols_per_wave, tuned.waves_per_block);
    if (opts) {
        if (opts->cols_per_wave > 0) s = make_shape(opts->cols_per_wave, s.wpb);
        if (opts->waves_per_block > 0) s = make_shape(s.cpw, opts->waves_per_block);
    }
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
    default: return false;
    }
}

static bool continuous(int32_t element) { return element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_P2P2; }

// Validate and fill everything but the race strategy and shape.
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
    if (kernel != EXM_K_MASS)
        EXM_CHECK(el == EXM_ELEMENT_P1P1, EXM_EUNSUPPORTED, "kernel %d is implemented for P1xP1 only", kernel);
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
            EXM_CHECK(A.access == EXM_INC || A.access == EXM_WRITE, EXM_EINVAL, "args[%d] must be EXM_INC or EXM_WRITE", i);
            if (A.access == EXM_WRITE)
                EXM_CHECK(!continuous(el), EXM_EINVAL,
                          "args[%d]: EXM_WRITE on a continuous space (DoFs shared between cells need EXM_INC)", i);
            const int32_t w = A.access == EXM_WRITE ? 1 : 0;
            EXM_CHECK(write < 0 || write == w, EXM_EINVAL, "outputs must all be WRITE or all INC");
            write = w;
        }
    }
    for (int i = 1 + sig.n_in; i < nargs; ++i)
        for (int j = 0; j < nargs; ++j)
            EXM_CHECK(i == j || args[i].data != args[j].data, EXM_EINVAL, "output args[%d] aliases args[%d]", i, j);
    std::memset(&P, 0, sizeof(P));
    P.kernel = kernel;
    P.element = el;
    P.n_layers = m->n_layers;
    P.field_offset = V->offsets[0];
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

static int32_t choose(const LoopLaunch& P, const exm_loop_opts* opts, exm_loop_opts& ch)
{
    exm_loop_opts tuned;
    const bool have_tuned = lookup_tuned(P.kernel, P.element, P.n_layers, P.n_cells, &tuned) != 0;
    ch.race = opts && opts->race ? opts->race : (have_tuned && tuned.race ? tuned.race : EXM_RACE_ATOMIC);
    EXM_CHECK(ch.race == EXM_RACE_ATOMIC || ch.race == EXM_RACE_COLOUR, EXM_EINVAL, "unknown race strategy %d", ch.race);
    EXM_CHECK(!opts || (opts->cols_per_wave >= 0 && opts->cols_per_wave <= 64), EXM_ERANGE,
              "cols_per_wave = %d outside [0, 64]", opts->cols_per_wave);
    EXM_CHECK(!opts || (opts->waves_per_block >= 0 && opts->waves_per_block <= 4), EXM_ERANGE,
              "waves_per_block = %d outside [0, 4]", opts->waves_per_block);
    LoopShape s = shape_from_opts(P.kernel, P.element, P.n_layers, P.n_cells, opts);
    ch.cols_per_wave = s.cpw;
    ch.waves_per_block = s.wpb;
    ch.reserved = 0;
    return EXM_OK;
}

static int32_t run_on_mesh(const exm_mesh* mesh, LoopLaunch& P, const exm_loop_opts& ch, hipStream_t stream)
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
    P.cells = nullptr;
    P.cell_begin = 0;
    P.cell_count = P.n_cells;
    return launch_column_loop(P, stream);
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
    s = choose(P, opts, ch);
    if (s != EXM_OK) return s;
    s = check_pending();
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
    return choose(P, opts, *chosen);
}

int32_t exm_autotune(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args, void* stream,
                     exm_loop_opts* best)
{
    clear_error();
    LoopLaunch P;
    int32_t s = prepare(kernel, iterset, nargs, args, P);
    if (s != EXM_OK) return s;
    hipStream_t hs = (hipStream_t)stream;
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
    const int32_t races[2] = {EXM_RACE_ATOMIC, EXM_RACE_COLOUR};
    const int nr = continuous(P.element) ? 2 : 1;
    const int32_t cpws[] = {1, 2, 3, 4, 5, 6, 8};
    const int32_t wpbs[] = {1, 2, 4};
    for (int r = 0; r < nr; ++r)
        for (int32_t c : cpws)
            for (int32_t w : wpbs) cand.push_back(exm_loop_opts{races[r], c, w, 0});
    hipEvent_t e0, e1;
    EXM_TRY_HIP(hipEventCreate(&e0));
    EXM_TRY_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    exm_loop_opts best_opts = cand[0];
    for (const exm_loop_opts& c : cand) {
        LoopLaunch Q = P;
        s = run_on_mesh(iterset, Q, c, hs);   // warm-up
        if (s != EXM_OK) break;
        float t_min = 1e30f;
        for (int rep = 0; rep < 3 && s == EXM_OK; ++rep) {
            EXM_TRY_HIP(hipEventRecord(e0, hs));
            Q = P;
            s = run_on_mesh(iterset, Q, c, hs);
            EXM_TRY_HIP(hipEventRecord(e1, hs));
            EXM_TRY_HIP(hipEventSynchronize(e1));
            float ms = 0;
            EXM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
            t_min = std::min(t_min, ms);
        }
        if (s != EXM_OK) break;
        if (t_min < best_ms) {
            best_ms = t_min;
            best_opts = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != EXM_OK) return s;
    EXM_TRY_HIP(hipStreamSynchronize(hs));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[tune_key(P.kernel, P.element, P.n_layers, P.n_cells)] = best_opts;
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
    f << "# kernel element n_layers log2_cells race cols_per_wave waves_per_block\n";
    for (auto& kv : g_tuned)
        f << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' ' << std::get<2>(kv.first) << ' '
          << std::get<3>(kv.first) << ' ' << kv.second.race << ' ' << kv.second.cols_per_wave << ' '
          << kv.second.waves_per_block << '\n';
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
        int32_t k, e, l, b, r, c, w;
        EXM_CHECK((bool)(is >> k >> e >> l >> b >> r >> c >> w), EXM_EINVAL, "%s:%d: malformed line", path, ln);
        EXM_CHECK((r == EXM_RACE_ATOMIC || r == EXM_RACE_COLOUR) && c >= 1 && c <= 64 && w >= 1 && w <= 4,
                  EXM_ERANGE, "%s:%d: values out of range", path, ln);
        table[TuneKey(k, e, l, b)] = exm_loop_opts{r, c, w, 0};
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& kv : table) g_tuned[kv.first] = kv.second;
    return EXM_OK;
}

}  // extern "C"
