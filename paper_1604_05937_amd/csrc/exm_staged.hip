// STAGED schedule of the column loop: tiles of base cells whose column
// segments are copied once into LDS.
//
// Why: in the DIRECT schedule each prism gathers its three vertex columns
// itself, so a vertex column shared by about six base cells crosses the
// vector-memory address path about six times, and that path, not HBM, limits
// the loop.  Here one workgroup owns a compact tile of base cells and walks its
// layers in chunks of S layers.  Per chunk it copies every column segment the
// tile touches (z coordinates and input fields, contiguous thanks to the
// vertical-innermost numbering) into LDS once; the element kernels of all
// (cell, layer) pairs read LDS only and sum their element vectors into LDS;
// the workgroup then adds every (vertex, level) sum to HBM once, and in the
// same phase copies the next chunk in.
//
// Everything that does not change along the column is fetched once per tile:
// the column starts, shared flags and (x, y) of the tile's vertices go to LDS,
// and each thread keeps the tile-local vertices of its (at most NP) cells in
// registers for all chunks -- thread t owns layer t % S of cells t / S + k *
// (256 / S).  Columns are vertical, so (x, y) is the same at every level.
//
// Shared vertices (touched by another tile) are updated with FP64 atomics, or
// with plain read-add-write when one launch holds one colour of tiles.
#include "exm_elements.hpp"
#include "exm_tiled.hpp"

namespace exm {

namespace {

constexpr int kThreads = 256;
constexpr int kPasses = 4;   // cells per thread: tile_cells <= kPasses * 256 / S

__device__ __forceinline__ unsigned xcd_block_s(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ int32_t eid(int32_t tagged) { return tagged & 0x7fffffff; }
__device__ __forceinline__ bool eshared(int32_t tagged) { return tagged < 0; }

struct Tile {
    int32_t cb, nc, vb, nv;
};

__device__ __forceinline__ Tile tile_of(const TileArgs& t)
{
    const int32_t b = (int32_t)xcd_block_s(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + b] : t.tile_begin + b;
    Tile r;
    r.cb = t.cell_off[tile];
    r.nc = t.cell_off[tile + 1] - r.cb;
    r.vb = t.vert_off[tile];
    r.nv = t.vert_off[tile + 1] - r.vb;
    return r;
}

template <int S>
struct Log2 {
    static constexpr int v = S == 8 ? 3 : (S == 16 ? 4 : (S == 32 ? 5 : 6));
};

// Per-tile vertex data in LDS: tag (id | shared bit), coordinate and field
// column starts, x and y.
struct VertLds {
    int32_t* tag;
    int32_t* xst;
    int32_t* fst;
    double* xs;
    double* ys;
};

__device__ __forceinline__ void load_vertices(const ColArgs& a, const TileArgs& t, const Tile& T, const VertLds& V,
                                              bool with_field)
{
    for (int v = threadIdx.x; v < T.nv; v += blockDim.x) {
        const int32_t tag = t.verts[T.vb + v];
        const int32_t xs = t.xstart[eid(tag)];
        V.tag[v] = tag;
        V.xst[v] = xs;
        V.fst[v] = with_field ? t.fstart0[eid(tag)] : 0;
        V.xs[v] = a.X[xs];
        V.ys[v] = a.X[a.xn + xs];
    }
}

// Copy levels l0 .. l0 + nl of NA vertex-column arrays into st[k][v * L + j]
// (array 0 is z, the others are inputs on the field space).
template <int S, int NA>
__device__ __forceinline__ void stage(const Tile& T, const VertLds& V, int l0, int nl, const double* const src[NA],
                                      double* st, int VL)
{
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    const int nvS = T.nv << LS;
    for (int it = threadIdx.x; it < nvS; it += blockDim.x) {
        const int v = it >> LS;
        const int j = it & (S - 1);
        if (j > nl) continue;
        const int64_t xo = (int64_t)V.xst[v] + l0 + j;
        const int64_t fo = (int64_t)V.fst[v] + l0 + j;
#pragma unroll
        for (int k = 0; k < NA; ++k) st[k * VL + v * L + j] = src[k][k == 0 ? xo : fo];
    }
    if (nl == S)   // the chunk's top level
        for (int v = threadIdx.x; v < T.nv; v += blockDim.x) {
            const int64_t xo = (int64_t)V.xst[v] + l0 + S;
            const int64_t fo = (int64_t)V.fst[v] + l0 + S;
#pragma unroll
            for (int k = 0; k < NA; ++k) st[k * VL + v * L + S] = src[k][k == 0 ? xo : fo];
        }
}

template <int FORM>
struct Form {
    static constexpr int NIN = FORM == 0 ? 1 : (FORM == 3 ? 3 : 2);
    static constexpr int NOUT = FORM == 0 ? 1 : (FORM == 1 ? 1 : (FORM == 2 ? 2 : 3));
};

template <int FORM>
__device__ __forceinline__ void element(double twoA, const double h[3], const double b[][3], const double tp[][3],
                                        double yb[][3], double yt[][3])
{
    if constexpr (FORM == 0)
        p1_mass(twoA, h, b[0], tp[0], yb[0], yt[0]);
    else
        cubic_element<FORM>(twoA, h, b, tp, yb, yt);
}

}  // namespace

// P1 x P1 forms.  LDS: ints tag/xst/fst [vstride]; doubles xs, ys [vstride],
// st [1 + NIN][vstride * L] (z, then the inputs), acc [2][NOUT][vstride * L]
// (this chunk and the next).
template <int FORM, bool ATOMIC, int S>
__global__ void __launch_bounds__(kThreads) k_staged_p1(const ColArgs a, const TileArgs t)
{
    constexpr int NIN = Form<FORM>::NIN;
    constexpr int NOUT = Form<FORM>::NOUT;
    constexpr int NA = 1 + NIN;
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    constexpr int CPP = kThreads >> LS;   // cells per pass
    extern __shared__ double lds[];
    const Tile T = tile_of(t);
    const int VL = t.vstride * L;
    VertLds V;
    V.xs = lds;
    V.ys = V.xs + t.vstride;
    double* st = V.ys + t.vstride;
    double* accb[2] = {st + NA * VL, st + NA * VL + NOUT * VL};
    V.tag = (int32_t*)(accb[1] + NOUT * VL);
    V.xst = V.tag + t.vstride;
    V.fst = V.xst + t.vstride;
    const double* const ins[3] = {a.in0, a.in1, a.in2};
    const double* src[NA];
    src[0] = a.X + 2 * a.xn;
#pragma unroll
    for (int k = 0; k < NIN; ++k) src[1 + k] = ins[k];
    double* const out[3] = {a.out0, a.out1, a.out2};
    const int lane = threadIdx.x & 63;
    const int j = threadIdx.x & (S - 1);

    // the thread's cells (tile-local vertex indices), fixed for all chunks
    int lv[kPasses][3];
    bool has[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        const int c = (threadIdx.x >> LS) + p * CPP;
        has[p] = c < T.nc;
#pragma unroll
        for (int q = 0; q < 3; ++q) lv[p][q] = has[p] ? t.lcv[(int64_t)(T.cb + c) * 3 + q] : 0;
    }
    const int npass = (T.nc + CPP - 1) / CPP;   // uniform over the workgroup

    load_vertices(a, t, T, V, true);
    __syncthreads();
    stage<S, NA>(T, V, 0, min(S, a.n_layers), src, st, VL);
    for (int i = threadIdx.x; i < NOUT * VL; i += blockDim.x) accb[0][i] = 0.0;
    __syncthreads();
    int cur = 0;
    for (int l0 = 0; l0 < a.n_layers; l0 += S) {
        const int nl = min(S, a.n_layers - l0);
        const bool last_chunk = l0 + nl == a.n_layers;
        double* acc = accb[cur];
        // element kernels; lanes hold consecutive layers of a cell, so the
        // top contribution of layer j - 1 comes from the previous lane
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            if (p >= npass) break;
            const bool act = has[p] && j < nl;
            double yb[NOUT][3], yt[NOUT][3];
#pragma unroll
            for (int o = 0; o < NOUT; ++o)
#pragma unroll
                for (int q = 0; q < 3; ++q) yb[o][q] = yt[o][q] = 0.0;
            if (act) {
                double x[3], y[3], h[3], b[NIN][3], tp[NIN][3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int o = lv[p][q] * L + j;
                    x[q] = V.xs[lv[p][q]];
                    y[q] = V.ys[lv[p][q]];
                    h[q] = st[o + 1] - st[o];
#pragma unroll
                    for (int k = 0; k < NIN; ++k) {
                        b[k][q] = st[(1 + k) * VL + o];
                        tp[k][q] = st[(1 + k) * VL + o + 1];
                    }
                }
                element<FORM>(twice_area(x, y), h, b, tp, yb, yt);
            }
#pragma unroll
            for (int o = 0; o < NOUT; ++o)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double below = __shfl_up(yt[o][q], 1, 64);
                    if (act) {
                        double* ptr = acc + o * VL + lv[p][q] * L + j;
                        atomicAdd(ptr, yb[o][q] + (j > 0 ? below : 0.0));
                        if (j == nl - 1) atomicAdd(ptr + 1, yt[o][q]);
                    }
                }
        }
        __syncthreads();
        // one update per (vertex, level); the chunk's top level is carried into
        // the other accumulator, which is cleared for the next chunk
        double* nxt = accb[cur ^ 1];
        const int nvS = T.nv << LS;
        for (int it = threadIdx.x; it < nvS; it += blockDim.x) {
            const int v = it >> LS;
            const int jj = it & (S - 1);
            if (jj < nl) {
                const int32_t tag = V.tag[v];
                const int64_t d = (int64_t)V.fst[v] + l0 + jj;
#pragma unroll
                for (int o = 0; o < NOUT; ++o) {
                    const double s = acc[o * VL + v * L + jj];
                    if (ATOMIC && eshared(tag))
                        unsafeAtomicAdd(out[o] + d, s);
                    else
                        out[o][d] += s;
                }
            }
            if (!last_chunk)
#pragma unroll
                for (int o = 0; o < NOUT; ++o) nxt[o * VL + v * L + jj] = jj == 0 ? acc[o * VL + v * L + nl] : 0.0;
        }
        for (int v = threadIdx.x; v < T.nv; v += blockDim.x) {
            if (last_chunk) {   // the column's top level
                const int32_t tag = V.tag[v];
                const int64_t d = (int64_t)V.fst[v] + l0 + nl;
#pragma unroll
                for (int o = 0; o < NOUT; ++o) {
                    const double s = acc[o * VL + v * L + nl];
                    if (ATOMIC && eshared(tag))
                        unsafeAtomicAdd(out[o] + d, s);
                    else
                        out[o][d] += s;
                }
            } else {
#pragma unroll
                for (int o = 0; o < NOUT; ++o) nxt[o * VL + v * L + S] = 0.0;
            }
        }
        if (last_chunk) break;
        stage<S, NA>(T, V, l0 + S, min(S, a.n_layers - l0 - S), src, st, VL);
        cur ^= 1;
        __syncthreads();
    }
    (void)lane;
}

// DG0 x DG0 and DG1 x DG1: only z is staged (two buffers, so the next chunk
// is copied in while this one is computed); the cell's own DoFs are
// consecutive in layers and read / written directly.
template <int NDOF, int S>
__global__ void __launch_bounds__(kThreads) k_staged_dg(const ColArgs a, const TileArgs t)
{
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    constexpr int CPP = kThreads >> LS;
    extern __shared__ double lds[];
    const Tile T = tile_of(t);
    const int VL = t.vstride * L;
    VertLds V;
    V.xs = lds;
    V.ys = V.xs + t.vstride;
    double* zb[2] = {V.ys + t.vstride, V.ys + t.vstride + VL};
    V.tag = (int32_t*)(zb[1] + VL);
    V.xst = V.tag + t.vstride;
    V.fst = V.xst + t.vstride;
    const double* const src[1] = {a.X + 2 * a.xn};
    const int j = threadIdx.x & (S - 1);
    int lv[kPasses][3];
    int64_t d0[kPasses];
    bool has[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        const int c = (threadIdx.x >> LS) + p * CPP;
        has[p] = c < T.nc;
#pragma unroll
        for (int q = 0; q < 3; ++q) lv[p][q] = has[p] ? t.lcv[(int64_t)(T.cb + c) * 3 + q] : 0;
        d0[p] = has[p] ? (int64_t)a.fmap[(int64_t)t.cells[T.cb + c] * NDOF] : 0;
    }
    const int npass = (T.nc + CPP - 1) / CPP;
    load_vertices(a, t, T, V, false);
    __syncthreads();
    stage<S, 1>(T, V, 0, min(S, a.n_layers), src, zb[0], VL);
    __syncthreads();
    int cur = 0;
    for (int l0 = 0; l0 < a.n_layers; l0 += S) {
        const int nl = min(S, a.n_layers - l0);
        const bool last_chunk = l0 + nl == a.n_layers;
        if (!last_chunk) stage<S, 1>(T, V, l0 + S, min(S, a.n_layers - l0 - S), src, zb[cur ^ 1], VL);
        const double* zs = zb[cur];
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            if (p >= npass) break;
            if (!(has[p] && j < nl)) continue;
            double x[3], y[3], h[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                x[q] = V.xs[lv[p][q]];
                y[q] = V.ys[lv[p][q]];
                h[q] = zs[lv[p][q] * L + j + 1] - zs[lv[p][q] * L + j];
            }
            const double twoA = twice_area(x, y);
            const int64_t d = d0[p] + (int64_t)(l0 + j) * a.off;
            if constexpr (NDOF == 1) {
                const double yv = dg0_mass(twoA, h, a.in0[d]);
                if (a.write)
                    a.out0[d] = yv;
                else
                    a.out0[d] += yv;
            } else {
                double xb[3], xt[3], yb[3], yt[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    xb[q] = a.in0[d + 2 * q];
                    xt[q] = a.in0[d + 2 * q + 1];
                }
                p1_mass(twoA, h, xb, xt, yb, yt);
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
        if (last_chunk) break;
        cur ^= 1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------

size_t staged_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t S)
{
    const size_t VL = (size_t)vstride * (S + 1);
    const size_t per_vertex = 2 * sizeof(double) + 3 * sizeof(int32_t);
    if (element == EXM_ELEMENT_DG0DG0 || element == EXM_ELEMENT_DG1DG1)
        return sizeof(double) * 2 * VL + per_vertex * vstride;
    if (element != EXM_ELEMENT_P1P1) return 0;
    int nin = 1, nout = 1;
    if (kernel == EXM_K_CUBIC) nin = 2;
    if (kernel == EXM_K_CUBIC_VJP) nin = 2, nout = 2;
    if (kernel == EXM_K_CUBIC_FUSED) nin = 3, nout = 3;
    return sizeof(double) * (1 + nin + 2 * nout) * VL + per_vertex * vstride;
}

int32_t staged_max_tile_cells(int32_t S) { return kPasses * (kThreads / S); }

bool staged_supported(int32_t kernel, int32_t element)
{
    return kernel != EXM_K_FACET_JUMP &&
           (element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_DG0DG0 || element == EXM_ELEMENT_DG1DG1);
}

template <int S>
static int32_t launch_staged_s(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    dim3 grid((unsigned)t.tile_count), block(kThreads);
    const bool atomic = P.race == EXM_RACE_ATOMIC;
#define EXM_SL(K) hipLaunchKernelGGL(K, grid, block, lds, s, a, t)
#define EXM_SL_RACE(F)                                   \
    do {                                                 \
        if (atomic) EXM_SL((k_staged_p1<F, true, S>));   \
        else EXM_SL((k_staged_p1<F, false, S>));         \
    } while (0)
    switch (P.element) {
    case EXM_ELEMENT_P1P1:
        switch (P.kernel) {
        case EXM_K_MASS: EXM_SL_RACE(0); break;
        case EXM_K_CUBIC: EXM_SL_RACE(1); break;
        case EXM_K_CUBIC_VJP: EXM_SL_RACE(2); break;
        case EXM_K_CUBIC_FUSED: EXM_SL_RACE(3); break;
        default: return fail(EXM_EUNSUPPORTED, "kernel %d not available on P1xP1", P.kernel);
        }
        break;
    case EXM_ELEMENT_DG0DG0: EXM_SL((k_staged_dg<1, S>)); break;
    case EXM_ELEMENT_DG1DG1: EXM_SL((k_staged_dg<6, S>)); break;
    default: return fail(EXM_EUNSUPPORTED, "element %d has no staged kernels", P.element);
    }
#undef EXM_SL_RACE
#undef EXM_SL
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t launch_staged(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t S, size_t lds, hipStream_t s)
{
    if (t.tile_count <= 0) return EXM_OK;
    switch (S) {
    case 8: return launch_staged_s<8>(P, a, t, lds, s);
    case 16: return launch_staged_s<16>(P, a, t, lds, s);
    case 32: return launch_staged_s<32>(P, a, t, lds, s);
    case 64: return launch_staged_s<64>(P, a, t, lds, s);
    default: return fail(EXM_ERANGE, "chunk_layers = %d: the STAGED schedule takes 8, 16, 32 or 64", S);
    }
}

}  // namespace exm
