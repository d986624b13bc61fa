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
// same phase copies the next chunk in.  The (x, y) of every tile vertex is
// read once per tile: columns are vertical.
//
// Shared vertices (touched by another tile) are updated with FP64 atomics, or
// with plain read-add-write when one launch holds one colour of tiles.
//
// Index maps use shifts only: S is a power of two, items (row, j) with j in
// [0, S) fastest, and the chunk's top level handled by its own short loop.
#include "exm_elements.hpp"
#include "exm_tiled.hpp"

namespace exm {

namespace {

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

// Copy levels l0 .. l0 + nl of NA vertex-column arrays into st[k][v * L + j].
// Array k < NZ is the z coordinate (k == 0), the others are inputs.
template <int S, int NA>
__device__ __forceinline__ void stage(const ColArgs& a, const TileArgs& t, const Tile& T, int l0, int nl,
                                      const double* const src[NA], const int32_t* const* starts, double* st, int VL)
{
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    const int nvS = T.nv << LS;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int32_t* sk = starts[k];
        for (int it = threadIdx.x; it < nvS; it += blockDim.x) {
            const int v = it >> LS;
            const int j = it & (S - 1);
            if (j <= nl) st[k * VL + v * L + j] = src[k][(int64_t)sk[eid(t.verts[T.vb + v])] + l0 + j];
        }
        if (nl == S)   // the chunk's top level
            for (int v = threadIdx.x; v < T.nv; v += blockDim.x)
                st[k * VL + v * L + S] = src[k][(int64_t)sk[eid(t.verts[T.vb + v])] + l0 + S];
    }
}

// (x, y) of every tile vertex, once.
__device__ __forceinline__ void stage_xy(const ColArgs& a, const TileArgs& t, const Tile& T, double* xs, double* ys)
{
    for (int v = threadIdx.x; v < T.nv; v += blockDim.x) {
        const int64_t d = t.xstart[eid(t.verts[T.vb + v])];
        xs[v] = a.X[d];
        ys[v] = a.X[a.xn + d];
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
    if constexpr (FORM == 0) {
        p1_mass(twoA, h, b[0], tp[0], yb[0], yt[0]);
    } else {
        CubicRule Q;
        cubic_rule(Q);
        double W[7][3], uq[7][3];
        cubic_weights(Q, twoA, h, W);
        p1_at_points(Q, b[0], tp[0], uq);
        if constexpr (FORM == 1 || FORM == 3) {
            double fq[7][3], s[7][3];
            p1_at_points(Q, b[1], tp[1], fq);
#pragma unroll
            for (int i = 0; i < 7; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) s[i][j] = W[i][j] * (uq[i][j] * uq[i][j] * uq[i][j] - fq[i][j]);
            p1_test(Q, s, yb[0], yt[0]);
        }
        if constexpr (FORM == 2 || FORM == 3) {
            constexpr int wi = FORM == 2 ? 1 : 2;
            constexpr int og = FORM == 2 ? 0 : 1;
            double wq[7][3], s[7][3], mb[3], mt[3];
            p1_at_points(Q, b[wi], tp[wi], wq);
#pragma unroll
            for (int i = 0; i < 7; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) s[i][j] = W[i][j] * 3.0 * uq[i][j] * uq[i][j] * wq[i][j];
            p1_test(Q, s, yb[og], yt[og]);
            p1_mass(twoA, h, b[wi], tp[wi], mb, mt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                yb[og + 1][q] = -mb[q];
                yt[og + 1][q] = -mt[q];
            }
        }
    }
}

}  // namespace

// P1 x P1 forms.  LDS (doubles): xs, ys [vstride]; st [1 + NIN][vstride * L]
// (z, then the inputs); acc [2][NOUT][vstride * L] (two chunks in flight).
template <int FORM, bool ATOMIC, int S>
__global__ void __launch_bounds__(256) k_staged_p1(const ColArgs a, const TileArgs t)
{
    constexpr int NIN = Form<FORM>::NIN;
    constexpr int NOUT = Form<FORM>::NOUT;
    constexpr int NA = 1 + NIN;
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    extern __shared__ double lds[];
    const Tile T = tile_of(t);
    const int VL = t.vstride * L;
    double* xs = lds;
    double* ys = xs + t.vstride;
    double* st = ys + t.vstride;
    double* accb[2] = {st + NA * VL, st + NA * VL + NOUT * VL};
    const double* const ins[3] = {a.in0, a.in1, a.in2};
    const double* src[NA];
    const int32_t* starts[NA];
    src[0] = a.X + 2 * a.xn;
    starts[0] = t.xstart;
#pragma unroll
    for (int k = 0; k < NIN; ++k) {
        src[1 + k] = ins[k];
        starts[1 + k] = t.fstart0;
    }
    double* const out[3] = {a.out0, a.out1, a.out2};
    const int lane = threadIdx.x & 63;

    stage_xy(a, t, T, xs, ys);
    stage<S, NA>(a, t, T, 0, min(S, a.n_layers), src, starts, st, VL);
    for (int i = threadIdx.x; i < NOUT * VL; i += blockDim.x) accb[0][i] = 0.0;
    __syncthreads();
    int cur = 0;
    for (int l0 = 0; l0 < a.n_layers; l0 += S) {
        const int nl = min(S, a.n_layers - l0);
        const bool last_chunk = l0 + nl == a.n_layers;
        double* acc = accb[cur];
        // element kernels of the chunk; item (cell, j) with j fastest, so a
        // wavefront holds consecutive layers of a cell and a shuffle adds the
        // top contribution of layer j - 1 to the bottom of layer j.
        const int nitems = T.nc << LS;
        const int wave_base = threadIdx.x - lane;
        for (int base = wave_base; base < nitems; base += blockDim.x) {   // uniform over the wavefront
            const int it = base + lane;
            const int c = it >> LS;
            const int j = it & (S - 1);
            const bool act = it < nitems && j < nl;
            int lv[3] = {0, 0, 0};
            double yb[NOUT][3], yt[NOUT][3];
#pragma unroll
            for (int o = 0; o < NOUT; ++o)
#pragma unroll
                for (int q = 0; q < 3; ++q) yb[o][q] = yt[o][q] = 0.0;
            if (act) {
                double x[3], y[3], h[3], b[NIN][3], tp[NIN][3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    lv[q] = t.lcv[(int64_t)(T.cb + c) * 3 + q];
                    const int o = lv[q] * L + j;
                    x[q] = xs[lv[q]];
                    y[q] = ys[lv[q]];
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
                        double* p = acc + o * VL + lv[q] * L + j;
                        atomicAdd(p, yb[o][q] + (j > 0 ? below : 0.0));
                        if (j == nl - 1) atomicAdd(p + 1, yt[o][q]);
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
            const int j = it & (S - 1);
            if (j < nl) {
                const int32_t tag = t.verts[T.vb + v];
                const int64_t d = (int64_t)t.fstart0[eid(tag)] + l0 + j;
#pragma unroll
                for (int o = 0; o < NOUT; ++o) {
                    const double s = acc[o * VL + v * L + j];
                    if (ATOMIC && eshared(tag))
                        unsafeAtomicAdd(out[o] + d, s);
                    else
                        out[o][d] += s;
                }
            }
            if (!last_chunk)
#pragma unroll
                for (int o = 0; o < NOUT; ++o) nxt[o * VL + v * L + j] = j == 0 ? acc[o * VL + v * L + nl] : 0.0;
        }
        for (int v = threadIdx.x; v < T.nv; v += blockDim.x) {
            if (last_chunk) {   // the column's top level
                const int32_t tag = t.verts[T.vb + v];
                const int64_t d = (int64_t)t.fstart0[eid(tag)] + l0 + nl;
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
        stage<S, NA>(a, t, T, l0 + S, min(S, a.n_layers - l0 - S), src, starts, st, VL);
        cur ^= 1;
        __syncthreads();
    }
}

// DG0 x DG0 and DG1 x DG1: only z is staged (two buffers, so the next chunk
// is copied in while this one is computed); the cell's own DoFs are
// consecutive in layers and read / written directly.
template <int NDOF, int S>
__global__ void __launch_bounds__(256) k_staged_dg(const ColArgs a, const TileArgs t)
{
    constexpr int L = S + 1;
    constexpr int LS = Log2<S>::v;
    extern __shared__ double lds[];
    const Tile T = tile_of(t);
    const int VL = t.vstride * L;
    double* xs = lds;
    double* ys = xs + t.vstride;
    double* zb[2] = {ys + t.vstride, ys + t.vstride + VL};
    const double* const src[1] = {a.X + 2 * a.xn};
    const int32_t* const starts[1] = {t.xstart};
    stage_xy(a, t, T, xs, ys);
    stage<S, 1>(a, t, T, 0, min(S, a.n_layers), src, starts, zb[0], VL);
    __syncthreads();
    int cur = 0;
    for (int l0 = 0; l0 < a.n_layers; l0 += S) {
        const int nl = min(S, a.n_layers - l0);
        const bool last_chunk = l0 + nl == a.n_layers;
        if (!last_chunk) stage<S, 1>(a, t, T, l0 + S, min(S, a.n_layers - l0 - S), src, starts, zb[cur ^ 1], VL);
        const double* zs = zb[cur];
        const int nitems = T.nc << LS;
        for (int it = threadIdx.x; it < nitems; it += blockDim.x) {
            const int c = it >> LS;
            const int j = it & (S - 1);
            if (j >= nl) continue;
            double x[3], y[3], h[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int lv = t.lcv[(int64_t)(T.cb + c) * 3 + q];
                x[q] = xs[lv];
                y[q] = ys[lv];
                h[q] = zs[lv * L + j + 1] - zs[lv * L + j];
            }
            const double twoA = twice_area(x, y);
            const int32_t cell = t.cells[T.cb + c];
            const int64_t d0 = (int64_t)a.fmap[(int64_t)cell * NDOF] + (int64_t)(l0 + j) * a.off;
            if constexpr (NDOF == 1) {
                const double yv = dg0_mass(twoA, h, a.in0[d0]);
                if (a.write)
                    a.out0[d0] = yv;
                else
                    a.out0[d0] += yv;
            } else {
                double xb[3], xt[3], yb[3], yt[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    xb[q] = a.in0[d0 + 2 * q];
                    xt[q] = a.in0[d0 + 2 * q + 1];
                }
                p1_mass(twoA, h, xb, xt, yb, yt);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (a.write) {
                        a.out0[d0 + 2 * q] = yb[q];
                        a.out0[d0 + 2 * q + 1] = yt[q];
                    } else {
                        a.out0[d0 + 2 * q] += yb[q];
                        a.out0[d0 + 2 * q + 1] += yt[q];
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
    const size_t xy = 2 * (size_t)vstride;
    if (element == EXM_ELEMENT_DG0DG0 || element == EXM_ELEMENT_DG1DG1) return sizeof(double) * (xy + 2 * VL);
    if (element != EXM_ELEMENT_P1P1) return 0;
    int nin = 1, nout = 1;
    if (kernel == EXM_K_CUBIC) nin = 2;
    if (kernel == EXM_K_CUBIC_VJP) nin = 2, nout = 2;
    if (kernel == EXM_K_CUBIC_FUSED) nin = 3, nout = 3;
    return sizeof(double) * (xy + (1 + nin + 2 * nout) * VL);
}

bool staged_supported(int32_t kernel, int32_t element)
{
    (void)kernel;
    return element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_DG0DG0 || element == EXM_ELEMENT_DG1DG1;
}

template <int S>
static int32_t launch_staged_s(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    dim3 grid((unsigned)t.tile_count), block(256);
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
