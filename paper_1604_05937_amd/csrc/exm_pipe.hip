// PIPELINED schedule of the column loop: the tile walk of the STAGED
// schedule, with every column segment copied into LDS by the asynchronous
// global-to-LDS loads of gfx950 (16 bytes per lane, no registers involved),
// issued one chunk of layers ahead of its use.
//
// One workgroup owns a compact tile of base cells (the tile plan) and walks
// its columns in chunks of S layers.  Per chunk and per tile vertex, the
// segment of levels l0 .. l0 + S of z, of the input field and of the INC
// output (y) lands in LDS.  The vertical-innermost numbering makes each
// segment contiguous in HBM, so the copy is a handful of 16-byte transfers per
// vertex, and every level of every array crosses the memory path once per
// tile.
//
// Per chunk k the workgroup, after one wait for its own copies and one
// barrier:
//   1. writes chunk k-1 back: every (vertex, level) sum goes to HBM once, a
//      plain store for vertices only this tile touches (whose LDS slot
//      started from the old output value) and an FP64 atomic add for shared
//      vertices (whose slot started from zero); the chunk's top level carries
//      into level 0 of chunk k;
//   2. barrier, then issues the copies of chunk k+1 into the other buffers;
//   3. computes chunk k from LDS: each thread owns R consecutive layers of a
//      few cells (fixed for the whole column, with 2A in registers), adds
//      the top contribution of layer r to the bottom one of layer r + 1 in
//      registers, and sends each level's sum to LDS with one LDS atomic.
// The copies of chunk k+1 and the stores of chunk k-1 are in flight while
// chunk k computes; the wait at the top of the next chunk finds them done.
//
// Copies are 16-byte aligned: a vertex's LDS slot starts at the even global
// index at or below its first level, so the slot holds one extra level below
// when the column start is odd (the parity is fixed because S is even).
// Base pointers must be 16-byte aligned; the host checks.
#include <algorithm>
#include <type_traits>

#include "exm_elements.hpp"
#include "exm_tiled.hpp"

namespace exm {

namespace {

constexpr int kThreads = 256;
constexpr int kPasses = 2;   // cells per thread: tile_cells <= kPasses * 256 * kLayers / S
constexpr int kLayers = 4;   // consecutive layers of one cell per thread

__device__ __forceinline__ unsigned xcd_block_p(unsigned b, unsigned G)
{
    const unsigned q = G >> 3, r = G & 7u, x = b & 7u, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Barrier for LDS traffic only: this wave's LDS reads and writes are done
// before any wave passes.  Asynchronous copies are waited for separately, and
// outstanding global stores are not waited for.
__device__ __forceinline__ void lds_barrier()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __asm__ __volatile__("" ::: "memory");
}

// All vector-memory operations of this wave are complete (copies landed in
// LDS, stores acknowledged).
__device__ __forceinline__ void wait_copies()
{
    __asm__ __volatile__("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
    __asm__ __volatile__("" ::: "memory");
}

// Copy 16 bytes from src to LDS at wave_base + 16 * (lane id), asynchronously.
// wave_base must be the same for every lane of the wavefront.
__device__ __forceinline__ void copy16(const double* src, double* wave_base)
{
    __builtin_amdgcn_global_load_lds((const void*)src,
                                     (__attribute__((address_space(3))) void*)wave_base, 16, 0, 0);
}

// FP64 add into LDS (no return value).  Written in assembly so that the
// compiler does not hold it until the asynchronous copies in flight have
// landed (they target the other buffers); lds_barrier() waits for it.
__device__ __forceinline__ void lds_add(double* p, double v)
{
    const uint32_t a = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) double*)p;
    __asm__ __volatile__("ds_add_f64 %0, %1" : : "v"(a), "v"(v));
}

__device__ __forceinline__ int32_t vid(int32_t tagged) { return tagged & 0x7fffffff; }
__device__ __forceinline__ bool vshared(int32_t tagged) { return tagged < 0; }

template <int S>
struct Chunk {
    static constexpr int LS = S == 8 ? 3 : (S == 16 ? 4 : 5);
    static constexpr int P2 = S + 2;      // doubles per vertex slot (even)
    static constexpr int PP = P2 / 2;     // 16-byte pairs per vertex slot
    static constexpr int R = kLayers;     // layers per thread
    static constexpr int G = S / R;       // threads per cell
    static constexpr int CPP = kThreads / G;   // cells per pass
};

}  // namespace

// How vertices shared between tiles are summed (MODE):
//   kPlain  - one launch holds one colour of tiles: every vertex is
//             read-added-written;
//   kAtomic - shared vertices are added atomically, the others read-added-
//             written;
//   kOwner  - owner plan: the tile writes only the vertices it owns (the first
//             `owned` of its list), with read-add-write, and drops the
//             contributions of its cells to the other vertices.
constexpr int kPlain = 0, kAtomic = 1, kOwner = 2;

// Per-thread output items: item i of thread t is (vertex, level offset)
// (t + 256 i) / S, (t + 256 i) % S of the chunk.
constexpr int kItems = 4;

// The (input, output) pairs a tile walk computes, one pass each, over one set
// of tile tables: the single pair of a column-loop launch, or every field of
// a batch item.
struct OneField {
    const double* x;
    double* y;
    __device__ int count() const { return 1; }
    __device__ const double* src(int) const { return x; }
    __device__ double* dst(int) const { return y; }
};
struct ManyFields {
    const double* const* xs;
    double* const* ys;
    int n;
    __device__ int count() const { return n; }
    __device__ const double* src(int k) const { return xs[k]; }
    __device__ double* dst(int k) const { return ys[k]; }
};

// P1 x P1 mass action / RHS of one tile, y += M x (INC), or y = M x
// (OVERWRITE: owner tiles only, every vertex a tile writes is its own), for
// every (x, y) pair of F in turn; the tile tables, 2A and the output items are
// set up once.  LDS: Z[2] and X[2] of vstride * (S + 2) doubles (16-byte
// aligned vertex slots), the accumulator A (same slots, levels l0 .. l0 + S of
// the chunk, the top one carried into the next chunk), then tag and column
// start (ints) per tile vertex; (x, y) per vertex only during set-up, inside
// A.  The old output values of a chunk are loaded into registers while the
// chunk computes and added when it is written back, during the next chunk.
template <int S, int MODE, bool OVERWRITE, class Fields, int NT = kThreads>
__device__ __forceinline__ void pipe_p1_tile(const ColArgs& a, const TileArgs& t, const int32_t tile, const Fields& F)
{
    // OVERWRITE: owner tiles write their vertices once; shared tiles (kAtomic)
    // overwrite the vertices no other tile touches and add the shared ones
    // atomically, into outputs that hold zeros there
    static_assert(!OVERWRITE || MODE == kOwner || MODE == kAtomic, "overwriting needs one writer per vertex");
    constexpr bool ATOMIC = MODE == kAtomic;
    constexpr int P2 = S + 2, PP = P2 / 2, R = kLayers, G = S / R, CPP = NT / G;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int32_t no = MODE == kOwner ? t.owned[tile] : nv;   // vertices this tile writes
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Xs = lds + 2 * VS;
    double* const A = lds + 4 * VS;
    double* const Tx = A;                 // set-up only
    double* const Ty = A + t.vstride;
    int32_t* const Ttag = (int32_t*)(lds + 5 * VS);
    int32_t* const Txst = Ttag + t.vstride;
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* x = F.src(0);   // the pass's input and output
    double* y = F.dst(0);
    const int lam = a.n_layers;

    // this thread's cells (tile-local vertices), loaded before the tile's
    // vertex table so that the two loads overlap
    bool has[kPasses];
    int lvq[kPasses][3];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        const int c = tid / G + p * CPP;
        has[p] = tid < CPP * G && c < nc;
#pragma unroll
        for (int q = 0; q < 3; ++q) lvq[p][q] = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
    }
    // tile vertex table: tag, column start, (x, y) of the column
    for (int v = tid; v < nv; v += NT) {
        const int32_t tag = t.verts[vb0 + v];
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(tag));
        Ttag[v] = tag;
        Txst[v] = xs;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    // this thread's cells: LDS slot start of each vertex (with the parity
    // shift) and 2A, fixed for the whole column; layers r0 .. r0 + R - 1 of
    // every chunk
    const int r0 = (tid % G) * R;
    int vb[kPasses][3];
    double twoA[kPasses];
    int wmask[kPasses];   // bit q: vertex q of the cell is written by this tile
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        double xq[3], yq[3];
        wmask[p] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[p][q];
            vb[p][q] = lv * P2 + (Txst[lv] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
            wmask[p] |= (lv < no ? 1 : 0) << q;
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;

    // this thread's output items: accumulator slot, global index (without
    // the chunk's first level), kind
    // ipos: slot (low 30 bits) and kind (top 2 bits: 0 none, 1 read-add-write, 2 atomic)
    int32_t ipos[kItems], iglb[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int it = tid + NT * i;
        const int v = it / S, jj = it - (it / S) * S;
        const bool ok = v < no;
        const int32_t xs = ok ? Txst[v] : 0;
        const int kind = !ok ? 0 : ((ATOMIC && vshared(Ttag[v])) ? 2 : 1);
        ipos[i] = (v * P2 + (xs & 1) + jj) | (kind << 30);
        iglb[i] = xs + jj;
    }
    lds_barrier();   // (x, y) are no longer needed: the accumulator takes their place
    const int wave_e = tid & ~63;

    // copies: pair e of the tile's vertex slots (vertex e / PP), levels from
    // the even global index at or below the chunk's first level
    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += NT) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            const int eb = 2 * (e0 + wave_e);   // wave's first double in the slot array
            const int e2 = 2 * e;
            if (g + 1 < n) {
                copy16(z + g, Zs + b * VS + eb);
                copy16(x + g, Xs + b * VS + eb);
            } else {   // the array's last element: keep the read inside the array
                Zs[b * VS + e2] = z[g];
                Xs[b * VS + e2] = x[g];
            }
        }
    };
    // levels chunk k writes back: its nl layers' bottom levels, and on a
    // last chunk shorter than S its top level too (an item of the chunk's
    // level range, so its old value is loaded a step ahead like the others)
    const int nch = (lam + S - 1) / S;
    const int top_in_items = lam - (nch - 1) * S < S;
    auto levels_written = [&](int k) { return min(S, lam - k * S) + (k == nch - 1 ? top_in_items : 0); };
    // old output values of chunk k (the levels it writes), into registers
    auto load_old = [&](int k, double (&dst)[kItems]) {
        const int l0 = k * S;
        const int nw = levels_written(k);
#pragma unroll
        for (int i = 0; i < kItems; ++i)
            dst[i] = (((uint32_t)ipos[i] >> 30) == 1 && (tid + NT * i) % S < nw) ? y[(int64_t)iglb[i] + l0] : 0.0;
    };
    // write chunk k back (its levels_written levels from l0); with `carry`,
    // move its top level to level 0 for chunk k + 1
    auto write_back = [&](int k, const double (&old)[kItems], bool carry) {
        const int l0 = k * S;
        const int nw = levels_written(k);
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int jj = (tid + NT * i) % S;
            const int kind = (int)((uint32_t)ipos[i] >> 30);
            const int pos = ipos[i] & 0x3fffffff;
            if (kind == 0 || jj >= nw) continue;
            const double s = A[pos];
            const int64_t g = (int64_t)iglb[i] + l0;
            if (kind == 2)
                unsafeAtomicAdd(y + g, s);
            else
                y[g] = OVERWRITE ? s : old[i] + s;
            if (carry && jj == 0) {
                A[pos] = A[pos + S];
                A[pos + S] = 0.0;
            } else {
                A[pos] = 0.0;
            }
        }
    };

    for (int pass = 0; pass < F.count(); ++pass) {
        if (pass > 0) {   // the previous pass's last write-back has read A
            x = F.src(pass);
            y = F.dst(pass);
            lds_barrier();
        }
        for (int i = tid; i < VS; i += NT) A[i] = 0.0;
        // yA: old values of the next chunk to be written back (loading); yB: of
        // the chunk written back next
        double yA[kItems], yB[kItems];
        issue_copies(0);
        if (!OVERWRITE) load_old(0, yA);
        for (int k = 0; k < nch; ++k) {
            const int b = k & 1;
            const int l0 = k * S;
            const int nl = min(S, lam - l0);
            wait_copies();
            lds_barrier();
            // 1. write chunk k-1 back and carry its top level into chunk k
            if (k > 0) write_back(k - 1, yB, true);
            // 2. old output values of chunk k+1, then the copies of chunk k+1
#pragma unroll
            for (int i = 0; i < kItems; ++i) yB[i] = yA[i];
            if (!OVERWRITE && k + 1 < nch) load_old(k + 1, yA);
            lds_barrier();
            if (k + 1 < nch) issue_copies(k + 1);
            // 3. element kernels of chunk k: R consecutive layers of one cell per
            // thread; a level's sum over the thread's layers goes to LDS once
            const double* const Zb = Zs + b * VS;
            const double* const Xb = Xs + b * VS;
#pragma unroll
            for (int p = 0; p < kPasses; ++p) {
                if (p >= npass) break;
                if (!has[p] || r0 >= nl) continue;
                int o[3];
                double zc[3], xc[3], acc[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    o[q] = vb[p][q] + r0;
                    zc[q] = Zb[o[q]];
                    xc[q] = Xb[o[q]];
                    acc[q] = 0.0;
                }
                int r = 0;
#pragma unroll
                for (; r < R; ++r) {
                    if (r0 + r >= nl) break;
                    double zn[3], xn[3], h[3], yb[3], yt[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        zn[q] = Zb[o[q] + r + 1];
                        xn[q] = Xb[o[q] + r + 1];
                        h[q] = zn[q] - zc[q];
                    }
                    p1_mass(twoA[p], h, xc, xn, yb, yt);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        if (MODE != kOwner || (wmask[p] >> q & 1)) lds_add(A + o[q] + r, acc[q] + yb[q]);
                        acc[q] = yt[q];
                        zc[q] = zn[q];
                        xc[q] = xn[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if (MODE != kOwner || (wmask[p] >> q & 1)) lds_add(A + o[q] + r, acc[q]);
            }
        }
        // write back the last chunk, its top level included (by the items
        // when the chunk is shorter than S, else here)
        lds_barrier();
        {
            const int k = nch - 1;
            const int l0 = k * S, nl = lam - l0;
            write_back(k, yB, false);
            for (int v = top_in_items ? no : tid; v < no; v += NT) {
                const int32_t xs = Txst[v];
                const double s = A[v * P2 + (xs & 1) + nl];
                const int64_t g = (int64_t)xs + lam;
                if (ATOMIC && vshared(Ttag[v]))
                    unsafeAtomicAdd(y + g, s);
                else if (OVERWRITE)
                    y[g] = s;
                else
                    y[g] += s;
            }
        }
    }
}

// NT threads per workgroup: 256, or 384 and 512 for tiles of more cells
// (fewer halo columns and shared vertices per cell, fewer workgroups per CU).
template <int S, int MODE, int NT>
__global__ void __launch_bounds__(NT) k_pipe_p1(const ColArgs a, const TileArgs t)
{
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    pipe_p1_tile<S, MODE, false, OneField, NT>(a, t, tile, OneField{a.in0, a.out0});
}

// The P1 x P1 items of a batch, b = M f and g = M w for every field: one
// workgroup per (item, tile) unit, in list order (largest columns first),
// runs every field of its item through the tile walk.  On owner tiles
// (kOwner) it overwrites the outputs of the vertices the tile owns; on
// shared tiles (kAtomic) it overwrites those of the vertices only it touches
// and adds those of the shared vertices atomically (k_zero_columns has
// zeroed them).
template <int S, int MODE>
__global__ void __launch_bounds__(kThreads) k_batch_pipe_p1(const BatchPipeItem* __restrict__ items,
                                                            const int32_t* __restrict__ units)
{
    const int32_t u = (int32_t)blockIdx.x;
    const BatchPipeItem& I = items[units[2 * u]];
    pipe_p1_tile<S, MODE, true>(I.a, I.t, units[2 * u + 1], ManyFields{I.src, I.dst, I.n_pass});
}

// Zero the vertex columns a batch's shared P1 tiles add into: block
// (b, k) takes the columns of unit b (an item and a range of its shared
// vertices) in output k of the item, one wavefront per column at a time.
__global__ void __launch_bounds__(256) k_zero_columns(const ZeroUnit* __restrict__ units)
{
    const ZeroUnit U = units[blockIdx.x];
    const int32_t k = (int32_t)blockIdx.y;
    if (k >= U.n_out) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* const y = U.dst[k];
    for (int32_t i = wave; i < U.count; i += 4) {
        const int64_t c = U.starts[i];
        for (int32_t l = lane; l < U.len; l += 64) y[c + l] = 0.0;
    }
}

// P1 x P1 mass action / RHS (INC) on a mesh whose cell columns have layer
// ranges of their own (cell c: layers lo_c .. lo_c + lam_c - 1; vertex v:
// levels lo_v .. hi_v, the union of its cells' ranges, level L at column
// start + L - lo_v).  k_pipe_p1 on absolute levels: a tile walks the chunks
// of S levels that cover its own window (the lowest and highest level of its
// vertices, from an even level), copies of a vertex stay inside its column
// (a 16-byte pair half outside it is loaded element by element), a thread
// evaluates its layers of a cell only inside the cell's range, and a
// (vertex, level) outside the vertex's range is neither read nor written.
// Chunk indices are kept in 8 bits: the host allows at most 2000 layers.
// Four workgroups per CU as for k_pipe_p1 where S is a power of two (at most
// 128 VGPRs, which the range bookkeeping fits only with the item fields
// packed as below; unbounded it took 154 VGPRs, three workgroups, and 40 %
// more time on full columns).  Other chunk lengths need a few more
// registers for the level offsets and keep three workgroups rather than
// spill.
template <int S, int MODE>
__global__ void __launch_bounds__(kThreads, (S & (S - 1)) == 0 ? 4 : 3) k_pipe_p1_var(const ColArgs a,
                                                                                        const TileArgs t)
{
    static_assert(MODE != kOwner, "owner tiles need columns of one height");
    constexpr bool ATOMIC = MODE == kAtomic;
    constexpr int P2 = S + 2, PP = P2 / 2, R = kLayers, G = S / R, CPP = kThreads / G;
    extern __shared__ double lds[];
    __shared__ int32_t s_lo, s_hi;   // the tile's level window
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Xs = lds + 2 * VS;
    double* const A = lds + 4 * VS;
    double* const Tx = A;                 // set-up only
    double* const Ty = A + t.vstride;
    int32_t* const Ttag = (int32_t*)(lds + 5 * VS);
    int32_t* const Txst = Ttag + t.vstride;
    int32_t* const Tlo = Txst + t.vstride;
    int32_t* const Thi = Tlo + t.vstride;
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* const x = a.in0;
    double* const y = a.out0;

    // this thread's cells: tile-local vertices and layer range
    bool has[kPasses];
    int lvq[kPasses][3], crng[kPasses];   // crng: first layer | (last layer + 1) << 16
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        const int c = tid / G + p * CPP;
        has[p] = tid < CPP * G && c < nc;
        const int32_t cell = has[p] ? t.cells[cb + c] : 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) lvq[p][q] = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
        const int cl = has[p] ? t.clo[cell] : 0;
        crng[p] = has[p] ? cl | ((cl + a.cell_lam[cell]) << 16) : 0;
    }
    if (tid == 0) {
        s_lo = INT32_MAX;
        s_hi = -1;
    }
    lds_barrier();
    // tile vertex table: tag, column start, level range, (x, y) of the column
    int my_lo = INT32_MAX, my_hi = -1;
    for (int v = tid; v < nv; v += kThreads) {
        const int32_t tag = t.verts[vb0 + v];
        const int32_t xs = t.xstart[vid(tag)];
        const int32_t lo = t.vlo[vid(tag)], hi = t.vhi[vid(tag)];
        Ttag[v] = tag;
        Txst[v] = xs;
        Tlo[v] = lo;
        Thi[v] = hi;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
        my_lo = min(my_lo, lo);
        my_hi = max(my_hi, hi);
    }
    if (my_hi >= 0) {
        atomicMin(&s_lo, my_lo);
        atomicMax(&s_hi, my_hi);
    }
    lds_barrier();
    // first level of the first chunk (even, so that each vertex's parity is
    // fixed) and the tile's top level, the same in every lane
    const int L0b = __builtin_amdgcn_readfirstlane(s_lo & ~1);
    const int thi = __builtin_amdgcn_readfirstlane(s_hi);
    const int nch = (thi - L0b + S - 1) / S;

    // slot start of each vertex of this thread's cells (with the parity
    // shift of its column) and 2A; layers r0 .. r0 + R - 1 of every chunk
    const int r0 = (tid % G) * R;
    int vb[kPasses][3];
    double twoA[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[p][q];
            vb[p][q] = lv * P2 + ((Txst[lv] - Tlo[lv] + L0b) & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;

    // item i of this thread: (vertex, level L0b + k S + jj of chunk k),
    // (tid + 256 i) / S, (tid + 256 i) % S, fixed for the whole column.
    // ipos: accumulator slot (bits 0-13: LDS holds at most 4096 slots per
    // array), kind (bits 14-15: 0 no vertex, 1 read-add-write, 2 atomic) and
    // the first and last chunk at which the level is inside the vertex's
    // column (bits 16-23, 24-31: the host allows at most 2000 layers, 250
    // chunks of 8); iglb: global index at chunk 0 (used only inside).
    uint32_t ipos[kItems];
    int32_t iglb[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int it = tid + kThreads * i;
        const int v = it / S, jj = it - (it / S) * S;
        const bool ok = v < nv;
        const int32_t xs = ok ? Txst[v] : 0;
        const int lo = ok ? Tlo[v] : 0, hi = ok ? Thi[v] : 0;
        const int kind = !ok ? 0 : ((ATOMIC && vshared(Ttag[v])) ? 2 : 1);
        const int nlo = lo - L0b - jj, nhi = hi - L0b - jj;   // inside: nlo <= k S <= nhi
        const int klo = nlo > 0 ? (nlo + S - 1) / S : 0;
        const int khi = nhi >= 0 ? nhi / S : -1;
        const bool any = khi >= klo;
        ipos[i] = (uint32_t)(v * P2 + ((xs - lo + L0b) & 1) + jj) | ((uint32_t)kind << 14) |
                  ((uint32_t)(any ? klo : 1) << 16) | ((uint32_t)(any ? khi : 0) << 24);
        iglb[i] = xs - lo + L0b + jj;
    }
    auto kind_of = [&](int i) { return (int)((ipos[i] >> 14) & 3u); };
    auto slot_of = [&](int i) { return (int)(ipos[i] & 0x3fffu); };
    auto inside = [&](int i, int k) { return k >= (int)((ipos[i] >> 16) & 0xffu) && k <= (int)(ipos[i] >> 24); };
    const int wave_e = tid & ~63;
    auto issue_copies = [&](int k) {
        const int L0 = L0b + k * S;
        const int nl = min(S, thi - L0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += kThreads) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int lo = Tlo[v], hi = Thi[v];
            const int sv = (xs - lo + L0b) & 1;
            const int La = L0 - sv + 2 * w;   // the pair's levels La, La + 1
            if (2 * w - sv > nl || La + 1 < lo || La > hi) continue;
            const int64_t g = (int64_t)xs + (La - lo);
            const int e2 = 2 * e;
            if (La >= lo && La + 1 <= hi) {
                copy16(z + g, Zs + b * VS + 2 * (e0 + wave_e));
                copy16(x + g, Xs + b * VS + 2 * (e0 + wave_e));
            } else if (La >= lo) {   // only the pair's first level is in the column
                Zs[b * VS + e2] = z[g];
                Xs[b * VS + e2] = x[g];
            } else {                 // only its second
                Zs[b * VS + e2 + 1] = z[g + 1];
                Xs[b * VS + e2 + 1] = x[g + 1];
            }
        }
    };
    auto load_old = [&](int k, double (&dst)[kItems]) {
        const int nl = min(S, thi - (L0b + k * S));
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int jj = (tid + kThreads * i) % S;
            const bool rd = kind_of(i) == 1 && jj < nl && inside(i, k);
            dst[i] = rd ? y[(int64_t)iglb[i] + k * S] : 0.0;
        }
    };
    auto write_back = [&](int k, const double (&old)[kItems], bool carry) {
        const int nl = min(S, thi - (L0b + k * S));
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int jj = (tid + kThreads * i) % S;
            const int kind = kind_of(i);
            const int pos = slot_of(i);
            if (kind == 0 || jj >= nl) continue;
            if (inside(i, k)) {
                const double s = A[pos];
                const int64_t g = (int64_t)iglb[i] + k * S;
                if (kind == 2)
                    unsafeAtomicAdd(y + g, s);
                else
                    y[g] = old[i] + s;
            }
            // the chunk's top level moves to level 0 of the next chunk even
            // where the old level 0 lies below the column
            if (carry && jj == 0) {
                A[pos] = A[pos + S];
                A[pos + S] = 0.0;
            } else {
                A[pos] = 0.0;
            }
        }
    };

    lds_barrier();   // (x, y) are no longer needed: the accumulator takes their place
    for (int i = tid; i < VS; i += kThreads) A[i] = 0.0;
    double yA[kItems], yB[kItems];
    issue_copies(0);
    load_old(0, yA);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int L0 = L0b + k * S;
        const int nl = min(S, thi - L0);
        wait_copies();
        lds_barrier();
        if (k > 0) write_back(k - 1, yB, true);
#pragma unroll
        for (int i = 0; i < kItems; ++i) yB[i] = yA[i];
        if (k + 1 < nch) load_old(k + 1, yA);
        lds_barrier();
        if (k + 1 < nch) issue_copies(k + 1);
        const double* const Zb = Zs + b * VS;
        const double* const Xb = Xs + b * VS;
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            if (p >= npass) break;
            const int clo = crng[p] & 0xffff, chi = crng[p] >> 16;
            if (!has[p] || r0 >= nl || L0 + r0 >= chi || L0 + r0 + R <= clo) continue;
            int o[3];
            double zc[3], xc[3], acc[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                o[q] = vb[p][q] + r0;
                zc[q] = Zb[o[q]];
                xc[q] = Xb[o[q]];
                acc[q] = 0.0;
            }
            int r = 0;
#pragma unroll
            for (; r < R; ++r) {
                if (r0 + r >= nl) break;
                const int L = L0 + r0 + r;
                const bool in = L >= clo && L < chi;   // a prism of this cell
                double zn[3], xn[3], h[3], yb[3] = {0.0, 0.0, 0.0}, yt[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    zn[q] = Zb[o[q] + r + 1];
                    xn[q] = Xb[o[q] + r + 1];
                    h[q] = zn[q] - zc[q];
                }
                if (in) p1_mass(twoA[p], h, xc, xn, yb, yt);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (in || acc[q] != 0.0) lds_add(A + o[q] + r, acc[q] + yb[q]);
                    acc[q] = yt[q];
                    zc[q] = zn[q];
                    xc[q] = xn[q];
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (acc[q] != 0.0) lds_add(A + o[q] + r, acc[q]);
        }
    }
    // write back the last chunk, and the tile's top level for the vertices that reach it
    lds_barrier();
    {
        const int k = nch - 1;
        const int L0 = L0b + k * S, nl = thi - L0;
        write_back(k, yB, false);
        for (int v = tid; v < nv; v += kThreads) {
            if (Thi[v] != thi) continue;
            const int32_t xs = Txst[v];
            const int lo = Tlo[v];
            const double s = A[v * P2 + ((xs - lo + L0b) & 1) + nl];
            const int64_t g = (int64_t)xs + (thi - lo);
            if (ATOMIC && vshared(Ttag[v]))
                unsafeAtomicAdd(y + g, s);
            else
                y[g] += s;
        }
    }
}

// Mass action / RHS on the spaces discontinuous horizontally and vertically:
// NH horizontal by NV vertical nodes per layer (DG0 x DG0 1 x 1, DG1 x DG1
// 3 x 2, DG0 x DG1 1 x 2, DG1 x DG0 3 x 1; node (a, b) at NV a + b of the
// layer, NDOF = NH NV values).  Only z
// is shared between the cells of a tile, so only z goes through LDS (S + 1
// levels per tile vertex and chunk, copied one chunk ahead).  A cell's DoFs
// form one contiguous column of NDOF * lambda values that no other cell
// touches: each thread takes one layer of a few cells, loads that layer's
// field values into registers one chunk ahead (coalesced along the column),
// and stores its results while the next chunk computes.  Every (x, y) pair
// of F runs in turn over one set-up of the tile.  LDS: Z[2] of
// vstride * (S + 2) doubles, then x, y (doubles) and the column start (int)
// per tile vertex.
template <int NH, int NV, int S, int NP, int NT, class Fields>
__device__ __forceinline__ void pipe_dg_tile(const ColArgs& a, const TileArgs& t, const int32_t tile, const Fields& F)
{
    constexpr int NDOF = NH * NV;
    using C = Chunk<S>;
    constexpr int P2 = C::P2, PP = C::PP;
    constexpr int CPP = NT / S;   // one layer per thread (S need not be a power of two)
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Tx = Zs + 2 * VS;
    double* const Ty = Tx + t.vstride;
    int32_t* const Txst = (int32_t*)(Ty + t.vstride);
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* f = F.src(0);   // the pass's input and output
    double* out = F.dst(0);
    const int lam = a.n_layers;

    // this thread's cells (tile-local vertices, field column), loaded before
    // the tile's vertex table so that the loads overlap
    bool has[NP];
    int lvq[NP][3];
    int32_t d0[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int c = tid / S + p * CPP;
        has[p] = tid < CPP * S && c < nc;
#pragma unroll
        for (int q = 0; q < 3; ++q) lvq[p][q] = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
        d0[p] = has[p] ? a.fmap[(int64_t)t.cells[cb + c] * NDOF] : 0;
    }
    for (int v = tid; v < nv; v += NT) {
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(t.verts[vb0 + v]));
        Txst[v] = xs;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    const int j = tid % S;
    int vb[NP][3];
    double twoA[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[p][q];
            vb[p][q] = lv * P2 + (Txst[lv] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;
    const int wave_e = tid & ~63;

    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += NT) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            if (g + 1 < n)
                copy16(z + g, Zs + b * VS + 2 * (e0 + wave_e));
            else
                Zs[b * VS + 2 * e] = z[g];
        }
    };
    auto load_field = [&](int k, double (&fv)[NP][NDOF]) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass) break;
            if (!has[p] || j >= nl) continue;
            const double* src = f + (int64_t)d0[p] + (int64_t)(l0 + j) * NDOF;
            if constexpr (NDOF % 2 == 0) {
                // even column starts and an even stride: 16-byte aligned pairs
#pragma unroll
                for (int q = 0; q < NDOF / 2; ++q) {
                    const double2 v2 = reinterpret_cast<const double2*>(src)[q];
                    fv[p][2 * q] = v2.x;
                    fv[p][2 * q + 1] = v2.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < NDOF; ++q) fv[p][q] = src[q];
            }
        }
    };

    double fcur[NP][NDOF], fnext[NP][NDOF], res[NP][NDOF];
    int prev_l0 = -1, prev_nl = 0;
    auto store_results = [&]() {
        if (prev_l0 < 0) return;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass) break;
            if (!has[p] || j >= prev_nl) continue;
            double* dst = out + (int64_t)d0[p] + (int64_t)(prev_l0 + j) * NDOF;
            if (a.write) {
                if constexpr (NDOF % 2 == 0) {
#pragma unroll
                    for (int q = 0; q < NDOF / 2; ++q)
                        reinterpret_cast<double2*>(dst)[q] = make_double2(res[p][2 * q], res[p][2 * q + 1]);
                } else {
#pragma unroll
                    for (int q = 0; q < NDOF; ++q) dst[q] = res[p][q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < NDOF; ++q) dst[q] += res[p][q];
            }
        }
    };

    const int nch = (lam + S - 1) / S;
    for (int pass = 0; pass < F.count(); ++pass) {
        if (pass > 0) {   // every thread is done with the previous pass's buffers
            f = F.src(pass);
            out = F.dst(pass);
            prev_l0 = -1;
            lds_barrier();
        }
        issue_copies(0);
        load_field(0, fcur);
        for (int k = 0; k < nch; ++k) {
            const int b = k & 1;
            const int l0 = k * S;
            const int nl = min(S, lam - l0);
            wait_copies();
            lds_barrier();
            if (k + 1 < nch) {
                issue_copies(k + 1);
                load_field(k + 1, fnext);
            }
            store_results();
            const double* const Zb = Zs + b * VS;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                if (p >= npass) break;
                if (!has[p] || j >= nl) continue;
                double h[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) h[q] = Zb[vb[p][q] + j + 1] - Zb[vb[p][q] + j];
                if constexpr (NDOF == 1) {
                    res[p][0] = dg0_mass(twoA[p], h, fcur[p][0]);
                } else if constexpr (NH != 3 || NV != 2) {   // DG0 x DG1, DG1 x DG0: node (a, b) at NV a + b
                    double x[NH][NV], y[NH][NV];
#pragma unroll
                    for (int q = 0; q < NDOF; ++q) x[q / NV][q % NV] = fcur[p][q];
                    tp_mass<NH, NV>(twoA[p], h, x, y);
#pragma unroll
                    for (int q = 0; q < NDOF; ++q) res[p][q] = y[q / NV][q % NV];
                } else {
                    double xb[3], xt[3], yb[3], yt[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        xb[q] = fcur[p][2 * q];
                        xt[q] = fcur[p][2 * q + 1];
                    }
                    p1_mass(twoA[p], h, xb, xt, yb, yt);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        res[p][2 * q] = yb[q];
                        res[p][2 * q + 1] = yt[q];
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int q = 0; q < NDOF; ++q) fcur[p][q] = fnext[p][q];
            prev_l0 = l0;
            prev_nl = nl;
        }
        store_results();
    }
}

// DG0 x DG0 mass action / RHS on a mesh whose cell columns have layer ranges
// of their own (cell c: layers lo_c .. lo_c + lam_c - 1, its list entry the
// DoF of layer lo_c; vertex v: levels lo_v .. hi_v).  The DG0 walk of
// pipe_dg_tile on absolute levels, with the level window and the clipped z
// copies of k_pipe_p1_var: a tile walks the chunks of S layers from an even
// level at or below its lowest vertex level up to its top level, and a
// thread's layer of a cell is loaded, evaluated and stored only inside the
// cell's range.  LDS as pipe_dg_tile, plus the level range (ints) per tile
// vertex.
template <int S, int NP, int NT>
__global__ void __launch_bounds__(NT, 7) k_pipe_dg0_var(const ColArgs a, const TileArgs t)
{
    using C = Chunk<S>;
    constexpr int P2 = C::P2, PP = C::PP, LS = C::LS;
    constexpr int CPP = NT >> LS;   // one layer per thread
    extern __shared__ double lds[];
    __shared__ int32_t s_lo, s_hi;   // the tile's level window
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Tx = Zs + 2 * VS;
    double* const Ty = Tx + t.vstride;
    int32_t* const Txst = (int32_t*)(Ty + t.vstride);
    int32_t* const Tlo = Txst + t.vstride;
    int32_t* const Thi = Tlo + t.vstride;
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* const f = a.in0;
    double* const out = a.out0;

    // this thread's cells: tile-local vertices, list entry, layer range
    bool has[NP];
    int lvq[NP][3];
    int32_t d0[NP];
    int crng[NP];   // first layer | (last layer + 1) << 16
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int c = (tid >> LS) + p * CPP;
        has[p] = c < nc;
        const int32_t cell = has[p] ? t.cells[cb + c] : 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) lvq[p][q] = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
        d0[p] = has[p] ? a.fmap[cell] : 0;
        const int cl = has[p] ? t.clo[cell] : 0;
        crng[p] = has[p] ? cl | ((cl + a.cell_lam[cell]) << 16) : 0;
    }
    if (tid == 0) {
        s_lo = INT32_MAX;
        s_hi = -1;
    }
    lds_barrier();
    int my_lo = INT32_MAX, my_hi = -1;
    for (int v = tid; v < nv; v += NT) {
        const int32_t id = vid(t.verts[vb0 + v]);
        const int32_t xs = t.xstart[id];
        const int32_t lo = t.vlo[id], hi = t.vhi[id];
        Txst[v] = xs;
        Tlo[v] = lo;
        Thi[v] = hi;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
        my_lo = min(my_lo, lo);
        my_hi = max(my_hi, hi);
    }
    if (my_hi >= 0) {
        atomicMin(&s_lo, my_lo);
        atomicMax(&s_hi, my_hi);
    }
    lds_barrier();
    const int L0b = __builtin_amdgcn_readfirstlane(s_lo & ~1);   // even: each vertex's parity is fixed
    const int thi = __builtin_amdgcn_readfirstlane(s_hi);        // the tile's top level

    const int j = tid & (S - 1);
    int vb[NP][3];
    double twoA[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[p][q];
            vb[p][q] = lv * P2 + ((Txst[lv] - Tlo[lv] + L0b) & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;
    const int wave_e = tid & ~63;

    // z of chunk k: levels L0 .. L0 + nl of every tile vertex, inside its column
    auto issue_copies = [&](int k) {
        const int L0 = L0b + k * S;
        const int nl = min(S, thi - L0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += NT) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int lo = Tlo[v], hi = Thi[v];
            const int sv = (xs - lo + L0b) & 1;
            const int La = L0 - sv + 2 * w;   // the pair's levels La, La + 1
            if (2 * w - sv > nl || La + 1 < lo || La > hi) continue;
            const int64_t g = (int64_t)xs + (La - lo);
            if (La >= lo && La + 1 <= hi)
                copy16(z + g, Zs + b * VS + 2 * (e0 + wave_e));
            else if (La >= lo)   // only the pair's first level is in the column
                Zs[b * VS + 2 * e] = z[g];
            else                 // only its second
                Zs[b * VS + 2 * e + 1] = z[g + 1];
        }
    };
    // this thread's layer L0 + j of cell p, if the cell has it
    auto inside = [&](int p, int L) { return L >= (crng[p] & 0xffff) && L < (crng[p] >> 16); };
    auto load_field = [&](int k, double (&fv)[NP]) {
        const int L0 = L0b + k * S;
        const int nl = min(S, thi - L0);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            fv[p] = 0.0;
            if (p >= npass || !has[p] || j >= nl || !inside(p, L0 + j)) continue;
            fv[p] = f[(int64_t)d0[p] + (L0 + j - (crng[p] & 0xffff))];
        }
    };

    double fcur[NP], fnext[NP], res[NP];
    int prev_L0 = -1, prev_nl = 0;
    auto store_results = [&]() {
        if (prev_L0 < 0) return;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass || !has[p] || j >= prev_nl || !inside(p, prev_L0 + j)) continue;
            double* dst = out + (int64_t)d0[p] + (prev_L0 + j - (crng[p] & 0xffff));
            if (a.write)
                *dst = res[p];
            else
                *dst += res[p];
        }
    };

    const int nch = (thi - L0b + S - 1) / S;
    issue_copies(0);
    load_field(0, fcur);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int L0 = L0b + k * S;
        const int nl = min(S, thi - L0);
        wait_copies();
        lds_barrier();
        if (k + 1 < nch) {
            issue_copies(k + 1);
            load_field(k + 1, fnext);
        }
        store_results();
        const double* const Zb = Zs + b * VS;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass || !has[p] || j >= nl || !inside(p, L0 + j)) continue;
            double h[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) h[q] = Zb[vb[p][q] + j + 1] - Zb[vb[p][q] + j];
            res[p] = dg0_mass(twoA[p], h, fcur[p]);
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) fcur[p] = fnext[p];
        prev_L0 = L0;
        prev_nl = nl;
    }
    store_results();
}

template <int NH, int NV, int S, int NP, int NT>
__global__ void __launch_bounds__(NT, NH * NV == 1 ? 8 : 4) k_pipe_dg(const ColArgs a, const TileArgs t)
{
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    pipe_dg_tile<NH, NV, S, NP, NT>(a, t, tile, OneField{a.in0, a.out0});
}

// The DG0 x DG0 items of a batch: one workgroup per (item, tile) unit, in
// list order, runs every field of its item through the DG tile walk (outputs
// written).
template <int S, int NP, int NT>
__global__ void __launch_bounds__(NT, 7) k_batch_pipe_dg0(const BatchPipeItem* __restrict__ items,
                                                          const int32_t* __restrict__ units)
{
    const int32_t u = (int32_t)blockIdx.x;
    const BatchPipeItem& I = items[units[2 * u]];
    pipe_dg_tile<1, 1, S, NP, NT>(I.a, I.t, units[2 * u + 1], ManyFields{I.src, I.dst, I.n_pass});
}

// Mass action / RHS on the spaces discontinuous horizontally and continuous
// vertically (DG0 x CG1: NH = 1, DG1 x CG1: NH = 3 values per level): a
// cell's column holds NH values on each of its lambda + 1 levels, level l at
// column start + NH l, and no other cell touches it.  As k_pipe_dg (z
// through LDS, the cell's own column through registers, one layer per
// thread), and, as in the DIRECT schedule, the layers of a cell sit on
// consecutive lanes: a lane takes the top values of its layer from the lane
// above (or loads them at the chunk's last layer), and adds the top row of
// the layer below (the lane below, or the carry from the previous chunk) to
// its bottom row, so every level is written once (INC, no atomics).
template <int NH, int S, int NP, int NT>
__global__ void __launch_bounds__(NT) k_pipe_dgv(const ColArgs a, const TileArgs t)
{
    using C = Chunk<S>;
    constexpr int P2 = C::P2, PP = C::PP, LS = C::LS;
    constexpr int CPP = NT >> LS;   // one layer per thread
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Tx = Zs + 2 * VS;
    double* const Ty = Tx + t.vstride;
    int32_t* const Txst = (int32_t*)(Ty + t.vstride);
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* const f = a.in0;
    double* const out = a.out0;
    const int lam = a.n_layers;

    // this thread's cells (tile-local vertices, field column), loaded before
    // the tile's vertex table so that the loads overlap
    bool has[NP];
    int lvq[NP][3];
    int32_t d0[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const int c = (tid >> LS) + p * CPP;
        has[p] = c < nc;
#pragma unroll
        for (int q = 0; q < 3; ++q) lvq[p][q] = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
        d0[p] = has[p] ? a.fmap[(int64_t)t.cells[cb + c] * (2 * NH)] : 0;
    }
    for (int v = tid; v < nv; v += NT) {
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(t.verts[vb0 + v]));
        Txst[v] = xs;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    const int j = tid & (S - 1);
    const int top_lane = (lane & ~(S - 1)) + S - 1;   // the lane of this cell's last layer in the chunk
    int vb[NP][3];
    double twoA[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[p][q];
            vb[p][q] = lv * P2 + (Txst[lv] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;
    const int wave_e = tid & ~63;

    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += NT) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            if (g + 1 < n)
                copy16(z + g, Zs + b * VS + 2 * (e0 + wave_e));
            else
                Zs[b * VS + 2 * e] = z[g];
        }
    };
    // the values of level l0 + j and, at the chunk's (or column's) last
    // layer, of level l0 + j + 1
    auto load_field = [&](int k, double (&fv)[NP][NH], double (&ft)[NP][NH]) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass) break;
            const bool act = has[p] && j < nl;
            const bool edge = act && j == nl - 1;
            const double* src = f + (int64_t)d0[p] + (int64_t)(l0 + j) * NH;
#pragma unroll
            for (int q = 0; q < NH; ++q) {
                fv[p][q] = act ? src[q] : 0.0;
                ft[p][q] = edge ? src[NH + q] : 0.0;
            }
        }
    };

    double fcur[NP][NH], tcur[NP][NH], fnext[NP][NH], tnext[NP][NH], res[NP][NH], carry[NP][NH];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int q = 0; q < NH; ++q) carry[p][q] = 0.0;
    int prev_l0 = -1, prev_nl = 0;
    auto store_results = [&]() {
        if (prev_l0 < 0) return;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass) break;
            if (!has[p] || j >= prev_nl) continue;
            double* dst = out + (int64_t)d0[p] + (int64_t)(prev_l0 + j) * NH;
#pragma unroll
            for (int q = 0; q < NH; ++q) dst[q] += res[p][q];
        }
    };

    const int nch = (lam + S - 1) / S;
    issue_copies(0);
    load_field(0, fcur, tcur);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        wait_copies();
        lds_barrier();
        if (k + 1 < nch) {
            issue_copies(k + 1);
            load_field(k + 1, fnext, tnext);
        }
        store_results();
        const double* const Zb = Zs + b * VS;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= npass) break;   // uniform: every lane takes part in the shuffles below
            const bool act = has[p] && j < nl;
            double h[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) h[q] = act ? Zb[vb[p][q] + j + 1] - Zb[vb[p][q] + j] : 0.0;
            double x[NH][2], y[NH][2];
#pragma unroll
            for (int q = 0; q < NH; ++q) {
                const double above = __shfl_down(fcur[p][q], 1, 64);   // level l0 + j + 1 from the lane above
                x[q][0] = fcur[p][q];
                x[q][1] = j == nl - 1 ? tcur[p][q] : above;
            }
            if (act) {
                tp_mass<NH, 2>(twoA[p], h, x, y);
            } else {
#pragma unroll
                for (int q = 0; q < NH; ++q) y[q][0] = y[q][1] = 0.0;
            }
#pragma unroll
            for (int q = 0; q < NH; ++q) {
                const double below = __shfl_up(y[q][1], 1, 64);   // top row of the layer below
                res[p][q] = y[q][0] + (j == 0 ? carry[p][q] : below);
                carry[p][q] = __shfl(y[q][1], top_lane, 64);      // into level 0 of the next chunk
            }
            // the column's top level: the top row of its last layer
            if (act && l0 + j == lam - 1) {
                double* dst = out + (int64_t)d0[p] + (int64_t)lam * NH;
#pragma unroll
                for (int q = 0; q < NH; ++q) dst[q] += y[q][1];
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int q = 0; q < NH; ++q) {
                fcur[p][q] = fnext[p][q];
                tcur[p][q] = tnext[p][q];
            }
        prev_l0 = l0;
        prev_nl = nl;
    }
    store_results();
}

// Mass action / RHS (INC) on the spaces continuous horizontally and
// discontinuous vertically (CG1 x DG0: NV = 1, CG1 x DG1: NV = 2 values per
// layer of a vertex column, layer l at column start + NV l).  The tile walk
// of k_pipe_p1 without the vertical carry: per chunk of S layers the NV S
// values of every tile vertex land in LDS beside z, one thread takes one
// layer of one cell and adds its element rows to the LDS accumulator, and
// chunk k - 1 is written back while chunk k computes (shared vertices
// atomically).  LDS: Z[2] of vstride * (S + 2) doubles, X[2] and A of
// vstride * (NV S + 2) doubles, then tag, coordinate and field column start
// per tile vertex (ints); (x, y) only during set-up, inside A.
constexpr int kItemsD = 8;   // output items per thread: vertices * NV * S <= 256 * kItemsD

template <int NV, int S, int MODE>
__global__ void __launch_bounds__(kThreads) k_pipe_cgdg(const ColArgs a, const TileArgs t)
{
    static_assert(MODE != kOwner, "owner-computes is for the P1 x P1 mass action");
    constexpr bool ATOMIC = MODE == kAtomic;
    constexpr int PZ = S + 2, PZP = PZ / 2;          // z slot
    constexpr int W = NV * S;                        // field values of a vertex per chunk
    constexpr int PX = W + 2, PXP = PX / 2;          // field / accumulator slot (parity shift, even)
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VZ = t.vstride * PZ;
    const int VX = t.vstride * PX;
    double* const Zs = lds;                          // [2][VZ]
    double* const Xs = lds + 2 * VZ;                 // [2][VX]
    double* const A = Xs + 2 * VX;                   // [VX]
    double* const Tx = A;                            // set-up only
    double* const Ty = A + t.vstride;
    int32_t* const Ttag = (int32_t*)(A + VX);
    int32_t* const Txst = Ttag + t.vstride;
    int32_t* const Tfst = Txst + t.vstride;
    const int64_t n = a.xn, fn = a.fn;
    const double* const z = a.X + 2 * n;
    const double* const x = a.in0;
    double* const y = a.out0;
    const int lam = a.n_layers;

    // this thread's cell (tile-local vertices) and its layer r of every
    // chunk, loaded before the vertex table so that the loads overlap
    const int r = tid % S;
    const int c = tid / S;
    const bool has = c < nc;
    int lvq[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) lvq[q] = has ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
    for (int v = tid; v < nv; v += kThreads) {
        const int32_t tag = t.verts[vb0 + v];
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(tag));
        Ttag[v] = tag;
        Txst[v] = xs;
        Tfst[v] = column_start(t.fstart0, t.fbase0, t.fstep0, vid(tag));
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    int zb[3], xb[3];
    double twoA;
    {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[q];
            zb[q] = lv * PZ + (Txst[lv] & 1);
            xb[q] = lv * PX + (Tfst[lv] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA = has ? twice_area(xq, yq) : 0.0;
    }
    lds_barrier();   // (x, y) are no longer needed: the accumulator takes their place
    for (int i = tid; i < VX; i += kThreads) A[i] = 0.0;
    const int wave_e = tid & ~63;

    // copies of chunk k: z levels l0 .. l0 + nl and field values
    // NV l0 .. NV (l0 + nl) - 1 of every tile vertex, in 16-byte pairs from the
    // even global index at or below the first
    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PZP; e0 += kThreads) {
            const int e = e0 + tid;
            const int v = e / PZP, w = e - (e / PZP) * PZP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            if (g + 1 < n)
                copy16(z + g, Zs + b * VZ + 2 * (e0 + wave_e));
            else   // the array's last element: keep the read inside the array
                Zs[b * VZ + 2 * e] = z[g];
        }
        for (int e0 = 0; e0 < nv * PXP; e0 += kThreads) {
            const int e = e0 + tid;
            const int v = e / PXP, w = e - (e / PXP) * PXP;
            if (v >= nv) continue;
            const int32_t fs = Tfst[v];
            const int sv = fs & 1;
            if (2 * w - sv >= NV * nl) continue;
            const int64_t g = (int64_t)fs - sv + (int64_t)NV * l0 + 2 * w;
            if (g + 1 < fn)
                copy16(x + g, Xs + b * VX + 2 * (e0 + wave_e));
            else
                Xs[b * VX + 2 * e] = x[g];
        }
    };
    // item i of this thread: (vertex, value of the chunk) (tid + 256 i) / W,
    // (tid + 256 i) % W; kind 0 none, 1 read-add-write, 2 atomic
    auto item_kind = [&](int i) {
        const int v = (tid + kThreads * i) / W;
        return v >= nv ? 0 : ((ATOMIC && vshared(Ttag[v])) ? 2 : 1);
    };
    auto load_old = [&](int k, double (&dst)[kItemsD]) {
        const int nl = min(S, lam - k * S);
#pragma unroll
        for (int i = 0; i < kItemsD; ++i) {
            const int it = tid + kThreads * i;
            const int v = it / W, jj = it % W;
            dst[i] = (item_kind(i) == 1 && jj < NV * nl) ? y[(int64_t)Tfst[v] + (int64_t)NV * k * S + jj] : 0.0;
        }
    };
    auto write_back = [&](int k, const double (&old)[kItemsD]) {
        const int nl = min(S, lam - k * S);
#pragma unroll
        for (int i = 0; i < kItemsD; ++i) {
            const int it = tid + kThreads * i;
            const int v = it / W, jj = it % W;
            const int kind = item_kind(i);
            if (kind == 0 || jj >= NV * nl) continue;
            const int32_t fs = Tfst[v];
            const int pos = v * PX + (fs & 1) + jj;
            const double s = A[pos];
            const int64_t g = (int64_t)fs + (int64_t)NV * k * S + jj;
            if (kind == 2)
                unsafeAtomicAdd(y + g, s);
            else
                y[g] = old[i] + s;
            A[pos] = 0.0;
        }
    };

    double yO[kItemsD];   // old output values of the chunk written back next
    const int nch = (lam + S - 1) / S;
    issue_copies(0);
    load_old(0, yO);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int nl = min(S, lam - k * S);
        wait_copies();
        lds_barrier();
        if (k > 0) {
            write_back(k - 1, yO);
            load_old(k, yO);
        }
        lds_barrier();
        if (k + 1 < nch) issue_copies(k + 1);
        if (!has || r >= nl) continue;
        const double* const Zb = Zs + b * VZ;
        const double* const Xb = Xs + b * VX;
        double h[3], xv[3][NV], yv[3][NV];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            h[q] = Zb[zb[q] + r + 1] - Zb[zb[q] + r];
#pragma unroll
            for (int be = 0; be < NV; ++be) xv[q][be] = Xb[xb[q] + NV * r + be];
        }
        tp_mass<3, NV>(twoA, h, xv, yv);
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int be = 0; be < NV; ++be) lds_add(A + xb[q] + NV * r + be, yv[q][be]);
    }
    lds_barrier();
    write_back(nch - 1, yO);
}

// P2 x P2 mass action, y += M x (INC).  The tile walk of k_pipe_p1 with the
// P2 columns: every base vertex and edge of the tile owns a field column of
// 2 lambda + 1 nodes (level l at 2 l, the middle of layer l at 2 l + 1), and
// per chunk of S layers its 2 S + 1 nodes land in LDS next to the S + 1 levels
// of z of every tile vertex.  Entity slots: the tile's vertices first, then
// its edges.  LDS: Z[2] of vstride * (S + 2) doubles, X[2] and the
// accumulator A of estride2 * (2 S + 2) doubles (estride2 = vstride +
// estride), then tag and field column start per entity and the coordinate
// column start per vertex (ints); (x, y) per vertex only during set-up,
// inside A.  Each thread takes one layer of one cell and adds each row of
// the element to LDS as soon as it is computed (one layer per thread keeps
// the element's registers within three wavefronts per SIMD).  Old output
// values of a chunk are loaded into registers right after the previous chunk
// is written back and added when this one is, one step later.
constexpr int kLayers2 = 1;   // consecutive layers of one cell per thread: tile_cells <= 256 * kLayers2 / S
constexpr int kItems2 = 8;    // output items per thread: (vertices + edges) * 2 S <= 256 * kItems2

template <int S, int MODE>
__global__ void __launch_bounds__(kThreads) k_pipe_p2(const ColArgs a, const TileArgs t)
{
    static_assert(MODE != kOwner, "no owner plan for edges");
    constexpr bool ATOMIC = MODE == kAtomic;
    constexpr int PZ = S + 2, PZP = PZ / 2;        // z slot (doubles, 16-byte pairs)
    constexpr int PX = 2 * S + 2, PXP = PX / 2;    // field / accumulator slot
    constexpr int W = 2 * S;                       // nodes a chunk writes per entity (the top one carries)
    constexpr int R = kLayers2, G = S / R;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int32_t eb0 = t.edge_off[tile], ne = t.edge_off[tile + 1] - eb0;
    const int32_t nent = nv + ne;
    const int ES = t.vstride + t.estride;
    const int VZ = t.vstride * PZ;
    const int VX = ES * PX;
    double* const Zs = lds;
    double* const Xs = lds + 2 * VZ;
    double* const A = Xs + 2 * VX;
    double* const Tx = A;                 // set-up only
    double* const Ty = A + t.vstride;
    int32_t* const Ttag = (int32_t*)(A + VX);
    int32_t* const Tfst = Ttag + ES;
    int32_t* const Txst = Tfst + ES;
    const int64_t n = a.xn, fn = a.fn;
    const double* const z = a.X + 2 * n;
    const double* const x = a.in0;
    double* const y = a.out0;
    const int lam = a.n_layers;

    // this thread's cell (tile-local vertices and edges), loaded before the
    // entity table so that the loads overlap
    const bool has = tid / G < nc;
    int lvq[3], leq[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        lvq[q] = has ? (int)t.lcv[(int64_t)(cb + tid / G) * 3 + q] : 0;
        leq[q] = has ? nv + (int)t.lce[(int64_t)(cb + tid / G) * 3 + q] : 0;
    }
    // entity table: tag, field column start; per vertex the coordinate column
    // start and (x, y) of the column
    for (int e = tid; e < nent; e += kThreads) {
        const bool vert = e < nv;
        const int32_t tag = vert ? t.verts[vb0 + e] : t.edges[eb0 + e - nv];
        Ttag[e] = tag;
        Tfst[e] = vert ? column_start(t.fstart0, t.fbase0, t.fstep0, vid(tag))
                       : column_start(t.fstart1, t.fbase1, t.fstep1, vid(tag));
        if (vert) {
            const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(tag));
            Txst[e] = xs;
            Tx[e] = a.X[xs];
            Ty[e] = a.X[n + xs];
        }
    }
    lds_barrier();

    // this thread's cell: z slot of each vertex, field slot of each of the
    // six horizontal nodes (vertices 0, 1, 2, then the edges opposite them),
    // with the parity shifts, and 2A; layers r0 .. r0 + R - 1 of every chunk
    const int r0 = (tid % G) * R;
    int zb[3], xb[6];
    double twoA;
    {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[q];
            const int le = leq[q];
            zb[q] = lv * PZ + (Txst[lv] & 1);
            xb[q] = lv * PX + (Tfst[lv] & 1);
            xb[3 + q] = le * PX + (Tfst[le] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA = has ? twice_area(xq, yq) : 0.0;
    }

    lds_barrier();   // (x, y) are no longer needed: the accumulator takes their place
    for (int i = tid; i < VX; i += kThreads) A[i] = 0.0;
    const int wave_e = tid & ~63;

    // copies of chunk k: z pairs of every vertex (levels from the even global
    // index at or below l0), field pairs of every entity (nodes from the even
    // global index at or below 2 l0)
    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PZP; e0 += kThreads) {
            const int e = e0 + tid;
            const int v = e / PZP, w = e - (e / PZP) * PZP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            if (g + 1 < n)
                copy16(z + g, Zs + b * VZ + 2 * (e0 + wave_e));
            else   // the array's last element: keep the read inside the array
                Zs[b * VZ + 2 * e] = z[g];
        }
        for (int e0 = 0; e0 < nent * PXP; e0 += kThreads) {
            const int e = e0 + tid;
            const int s = e / PXP, w = e - (e / PXP) * PXP;
            if (s >= nent) continue;
            const int32_t fs = Tfst[s];
            const int sv = fs & 1;
            if (2 * w - sv > 2 * nl) continue;
            const int64_t g = (int64_t)fs - sv + 2 * l0 + 2 * w;
            if (g + 1 < fn)
                copy16(x + g, Xs + b * VX + 2 * (e0 + wave_e));
            else
                Xs[b * VX + 2 * e] = x[g];
        }
    };
    // output items: item i of this thread is (entity, node) (tid + 256 i) / W,
    // (tid + 256 i) % W of the chunk; its kind is 0 (none), 1 (read-add-write)
    // or 2 (atomic)
    auto item_kind = [&](int i) {
        const int e = (tid + kThreads * i) / W;
        return e >= nent ? 0 : ((ATOMIC && vshared(Ttag[e])) ? 2 : 1);
    };
    auto load_old = [&](int k, double (&dst)[kItems2]) {
        const int nl = min(S, lam - k * S);
#pragma unroll
        for (int i = 0; i < kItems2; ++i) {
            const int it = tid + kThreads * i;
            const int e = it / W, jj = it % W;
            dst[i] = (item_kind(i) == 1 && jj < 2 * nl) ? y[(int64_t)Tfst[e] + 2 * k * S + jj] : 0.0;
        }
    };
    auto write_back = [&](int k, const double (&old)[kItems2], bool carry) {
        const int nl = min(S, lam - k * S);
#pragma unroll
        for (int i = 0; i < kItems2; ++i) {
            const int it = tid + kThreads * i;
            const int e = it / W, jj = it % W;
            const int kind = item_kind(i);
            if (kind == 0 || jj >= 2 * nl) continue;
            const int32_t fs = Tfst[e];
            const int pos = e * PX + (fs & 1) + jj;
            const double s = A[pos];
            const int64_t g = (int64_t)fs + 2 * k * S + jj;
            if (kind == 2)
                unsafeAtomicAdd(y + g, s);
            else
                y[g] = old[i] + s;
            if (carry && jj == 0) {
                A[pos] = A[pos + W];
                A[pos + W] = 0.0;
            } else {
                A[pos] = 0.0;
            }
        }
    };

    // yO: old output values of the chunk written back next
    double yO[kItems2];
    const int nch = (lam + S - 1) / S;
    issue_copies(0);
    load_old(0, yO);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int nl = min(S, lam - k * S);
        wait_copies();
        lds_barrier();
        if (k > 0) {
            write_back(k - 1, yO, true);
            load_old(k, yO);
        }
        lds_barrier();
        if (k + 1 < nch) issue_copies(k + 1);
        if (!has || r0 >= nl) continue;
        const double* const Zb = Zs + b * VZ;
        const double* const Xb = Xs + b * VX;
        double zc[3], xv[6][3], acc[6];
#pragma unroll
        for (int q = 0; q < 3; ++q) zc[q] = Zb[zb[q] + r0];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            xv[e][0] = Xb[xb[e] + 2 * r0];
            acc[e] = 0.0;
        }
        int r = 0;
#pragma unroll
        for (; r < R; ++r) {
            if (r0 + r >= nl) break;
            const int o = 2 * (r0 + r);
            double h[3], g[6][3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double zn = Zb[zb[q] + r0 + r + 1];
                h[q] = zn - zc[q];
                zc[q] = zn;
            }
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                xv[e][2] = Xb[xb[e] + o + 1];
                xv[e][1] = Xb[xb[e] + o + 2];
            }
            p2_vertical(xv, g);
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                double yi[3];
                p2_mass_row(twoA, h, g, e, yi);
                lds_add(A + xb[e] + o, acc[e] + yi[0]);
                lds_add(A + xb[e] + o + 1, yi[2]);
                acc[e] = yi[1];
                xv[e][0] = xv[e][1];
            }
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) lds_add(A + xb[e] + 2 * (r0 + r), acc[e]);
    }
    // write back the last chunk, its top node included
    lds_barrier();
    {
        const int k = nch - 1;
        const int nl = lam - k * S;
        write_back(k, yO, false);
        for (int e = tid; e < nent; e += kThreads) {
            const int32_t fs = Tfst[e];
            const double s = A[e * PX + (fs & 1) + 2 * nl];
            const int64_t g = (int64_t)fs + 2 * lam;
            if (ATOMIC && vshared(Ttag[e]))
                unsafeAtomicAdd(y + g, s);
            else
                y[g] += s;
        }
    }
}

// Cubic forms of P1 x P1 (FORM 1: F = integral (u^3 - f) v; 2: its adjoint
// g_u, g_f; 3: both in one sweep; inputs and outputs as in cubic_element),
// all INC.  The tile walk of k_pipe_p1 with NIN input columns and NOUT
// accumulators per tile vertex: z and every input land in LDS one chunk
// ahead, one thread takes one layer of one cell and adds the bottom and top
// rows of every output to LDS, and chunk k - 1 is written back while chunk k
// computes.  LDS: Z[2], X[2][NIN], A[NOUT] of vstride * (S + 2) doubles, then
// tag and column start per tile vertex (ints); (x, y) per vertex only during
// set-up, inside A.  Old output values of a chunk are loaded into registers
// right after the previous chunk is written back (item indices come from the
// LDS tables, not from registers).  Tiles of up to 256 / S cells: larger
// tiles in 512-thread workgroups measured slower.  NI output items per
// thread (vertices * S <= 256 NI): the launch takes the fewest that cover its
// tiles, since each item holds NOUT old values in registers; the forward and
// adjoint forms then fit four waves per SIMD, the fused form three.
constexpr int kItemsC = 4;   // the most output items per thread

template <int FORM>
struct CubicIO {
    static constexpr int NIN = FORM == 3 ? 3 : 2;
    static constexpr int NOUT = FORM == 1 ? 1 : (FORM == 2 ? 2 : 3);
};

template <int FORM, int S, int MODE, int NI>
__global__ void __launch_bounds__(kThreads, FORM == 3 && NI > 1 ? 3 : 4) k_pipe_cubic(const ColArgs a,
                                                                                       const TileArgs t)
{
    static_assert(MODE != kOwner, "owner-computes is for the mass action");
    constexpr int NIN = CubicIO<FORM>::NIN, NOUT = CubicIO<FORM>::NOUT;
    constexpr bool ATOMIC = MODE == kAtomic;
    constexpr int P2 = S + 2, PP = P2 / 2;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + blk] : t.tile_begin + blk;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int VS = t.vstride * P2;
    double* const Zs = lds;                        // [2][VS]
    double* const Xs = lds + 2 * VS;               // [2][NIN][VS]
    double* const A = lds + (2 + 2 * NIN) * VS;    // [NOUT][VS]
    double* const Tx = A;                          // set-up only
    double* const Ty = A + t.vstride;
    int32_t* const Ttag = (int32_t*)(lds + (2 + 2 * NIN + NOUT) * VS);
    int32_t* const Txst = Ttag + t.vstride;
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* const in[3] = {a.in0, a.in1, a.in2};
    double* const out[3] = {a.out0, a.out1, a.out2};
    const int lam = a.n_layers;

    // this thread's cell and its layer r of every chunk; the cell's tile-local
    // vertices are loaded before the vertex table so that the loads overlap
    const int r = tid % S;
    const int c = tid / S;
    const bool has = c < nc;
    int lvq[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) lvq[q] = has ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
    for (int v = tid; v < nv; v += kThreads) {
        const int32_t tag = t.verts[vb0 + v];
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(tag));
        Ttag[v] = tag;
        Txst[v] = xs;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    int vb[3];
    double twoA;
    {
        double xq[3], yq[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = lvq[q];
            vb[q] = lv * P2 + (Txst[lv] & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
        }
        twoA = has ? twice_area(xq, yq) : 0.0;
    }
    lds_barrier();   // (x, y) are no longer needed: the accumulators take their place
    for (int i = tid; i < NOUT * VS; i += kThreads) A[i] = 0.0;
    const int wave_e = tid & ~63;

    auto issue_copies = [&](int k) {
        const int l0 = k * S;
        const int nl = min(S, lam - l0);
        const int b = k & 1;
        for (int e0 = 0; e0 < nv * PP; e0 += kThreads) {
            const int e = e0 + tid;
            const int v = e / PP, w = e - (e / PP) * PP;
            if (v >= nv) continue;
            const int32_t xs = Txst[v];
            const int sv = xs & 1;
            if (2 * w - sv > nl) continue;
            const int64_t g = (int64_t)xs - sv + l0 + 2 * w;
            if (g + 1 < n) {
                copy16(z + g, Zs + b * VS + 2 * (e0 + wave_e));
#pragma unroll
                for (int i = 0; i < NIN; ++i) copy16(in[i] + g, Xs + (b * NIN + i) * VS + 2 * (e0 + wave_e));
            } else {   // the array's last element: keep the read inside the array
                Zs[b * VS + 2 * e] = z[g];
#pragma unroll
                for (int i = 0; i < NIN; ++i) Xs[(b * NIN + i) * VS + 2 * e] = in[i][g];
            }
        }
    };
    // item i of this thread: (vertex, level of the chunk) (tid + 256 i) / S,
    // (tid + 256 i) % S; kind 0 none, 1 read-add-write, 2 atomic
    auto item_kind = [&](int i) {
        const int v = (tid + kThreads * i) / S;
        return v >= nv ? 0 : ((ATOMIC && vshared(Ttag[v])) ? 2 : 1);
    };
    // levels chunk k writes back: its layers' bottom levels, and on a last
    // chunk shorter than S its top level too (so that its old value is
    // loaded a step ahead like the others)
    const int nch = (lam + S - 1) / S;
    const int top_in_items = lam - (nch - 1) * S < S;
    auto levels_written = [&](int k) { return min(S, lam - k * S) + (k == nch - 1 ? top_in_items : 0); };
    auto load_old = [&](int k, double (&dst)[NOUT][NI]) {
        const int nw = levels_written(k);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int it = tid + kThreads * i;
            const int v = it / S, jj = it % S;
            const bool ld = item_kind(i) == 1 && jj < nw;
            const int64_t g = ld ? (int64_t)Txst[v] + k * S + jj : 0;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) dst[o][i] = ld ? out[o][g] : 0.0;
        }
    };
    auto write_back = [&](int k, const double (&old)[NOUT][NI], bool carry) {
        const int nw = levels_written(k);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int it = tid + kThreads * i;
            const int v = it / S, jj = it % S;
            const int kind = item_kind(i);
            if (kind == 0 || jj >= nw) continue;
            const int32_t xs = Txst[v];
            const int pos = v * P2 + (xs & 1) + jj;
            const int64_t g = (int64_t)xs + k * S + jj;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                double* const Ao = A + o * VS;
                const double s = Ao[pos];
                if (kind == 2)
                    unsafeAtomicAdd(out[o] + g, s);
                else
                    out[o][g] = old[o][i] + s;
                if (carry && jj == 0) {
                    Ao[pos] = Ao[pos + S];
                    Ao[pos + S] = 0.0;
                } else {
                    Ao[pos] = 0.0;
                }
            }
        }
    };

    double yO[NOUT][NI];   // old output values of the chunk written back next
    issue_copies(0);
    load_old(0, yO);
    for (int k = 0; k < nch; ++k) {
        const int b = k & 1;
        const int nl = min(S, lam - k * S);
        wait_copies();
        lds_barrier();
        if (k > 0) {
            write_back(k - 1, yO, true);
            load_old(k, yO);
        }
        lds_barrier();
        if (k + 1 < nch) issue_copies(k + 1);
        if (!has || r >= nl) continue;
        const double* const Zb = Zs + b * VS;
        double h[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) h[q] = Zb[vb[q] + r + 1] - Zb[vb[q] + r];
        // the element of inputs i0, i1 (u and f, or u and w) into outputs o0 ..
        auto element = [&](auto form, int i1, int o0) {
            constexpr int EF = decltype(form)::value;
            constexpr int NO = EF == 1 ? 1 : 2;
            double vbot[2][3], vtop[2][3], yb[NO][3], yt[NO][3];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const double* const Xb = Xs + (b * NIN + (i == 0 ? 0 : i1)) * VS;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    vbot[i][q] = Xb[vb[q] + r];
                    vtop[i][q] = Xb[vb[q] + r + 1];
                }
            }
            cubic_element<EF>(twoA, h, vbot, vtop, yb, yt);
#pragma unroll
            for (int o = 0; o < NO; ++o)
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    lds_add(A + (o0 + o) * VS + vb[q] + r, yb[o][q]);
                    lds_add(A + (o0 + o) * VS + vb[q] + r + 1, yt[o][q]);
                }
        };
        if constexpr (FORM == 1) element(std::integral_constant<int, 1>{}, 1, 0);
        if constexpr (FORM == 2) element(std::integral_constant<int, 2>{}, 1, 0);
        if constexpr (FORM == 3) {
            // both forms on one prism, sharing u at the triangle points; the
            // linear terms first, so that f and the rows of g_f are done with
            // before the points' loop: F from -M f, g_f = -M w into LDS, then
            // the terms in u^3 and 3 u^2 w
            auto load = [&](int i, double (&vb_)[3], double (&vt_)[3]) {
                const double* const Xb = Xs + (b * NIN + i) * VS;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    vb_[q] = Xb[vb[q] + r];
                    vt_[q] = Xb[vb[q] + r + 1];
                }
            };
            double fb[3], ft[3], gb[3] = {0.0, 0.0, 0.0}, gt[3] = {0.0, 0.0, 0.0};
            {
                double xb[3], xt[3];
                load(1, xb, xt);
                p1_mass(twoA, h, xb, xt, fb, ft);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    fb[q] = -fb[q];
                    ft[q] = -ft[q];
                }
            }
            double wb[3], wt[3];
            load(2, wb, wt);
            {
                double mb[3], mt[3];
                p1_mass(twoA, h, wb, wt, mb, mt);
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    lds_add(A + 2 * VS + vb[q] + r, -mb[q]);
                    lds_add(A + 2 * VS + vb[q] + r + 1, -mt[q]);
                }
            }
            double ub[3], ut[3];
            load(0, ub, ut);
            cubic_points<true, true>(twoA, h, ub, ut, wb, wt, fb, ft, gb, gt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                lds_add(A + vb[q] + r, fb[q]);
                lds_add(A + vb[q] + r + 1, ft[q]);
                lds_add(A + VS + vb[q] + r, gb[q]);
                lds_add(A + VS + vb[q] + r + 1, gt[q]);
            }
        }
    }
    // write back the last chunk, its top level included (by the items when
    // the chunk is shorter than S, else here)
    lds_barrier();
    {
        const int k = nch - 1;
        const int nl = lam - k * S;
        write_back(k, yO, false);
        for (int v = top_in_items ? nv : tid; v < nv; v += kThreads) {
            const int32_t xs = Txst[v];
            const int64_t g = (int64_t)xs + lam;
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                const double s = A[o * VS + v * P2 + (xs & 1) + nl];
                if (ATOMIC && vshared(Ttag[v]))
                    unsafeAtomicAdd(out[o] + g, s);
                else
                    out[o][g] += s;
            }
        }
    }
}

// CHUNKED schedule, P1 x P1 mass action / RHS (INC): one workgroup per
// (tile, chunk).  Chunk c computes the layers c (S - 1) .. c (S - 1) + S - 1
// and writes the levels whose two neighbouring layers it computed (the
// chunk's inner levels, plus level 0 in the first chunk and level lambda in
// the last): consecutive chunks overlap by one layer, so no partial sum
// crosses a workgroup and every (vertex, level) is written by one workgroup
// per tile.  Workgroups are independent: each copies its column segments
// into LDS (asynchronous 16-byte copies), waits once, computes, and writes.
// The grid is chunk-major, so the workgroups that run together hold
// neighbouring tiles at the same levels and share their boundary columns in
// L2.  MODE as for k_pipe_p1 (kOwner with an owner plan, kAtomic, or kPlain
// for one colour of tiles).  LDS: Z, X, Y of vstride * (S + 2) doubles, then
// x, y (doubles) and tag, column start (ints) per tile vertex.
template <int S, int MODE>
__global__ void __launch_bounds__(kThreads) k_chunk_p1(const ColArgs a, const TileArgs t, int32_t n_chunks)
{
    constexpr bool ATOMIC = MODE == kAtomic;
    using C = Chunk<S>;
    constexpr int P2 = C::P2, PP = C::PP, R = C::R, G = C::G, CPP = C::CPP;
    extern __shared__ double lds[];
    const int tid = threadIdx.x;
    const int32_t blk = (int32_t)xcd_block_p(blockIdx.x, gridDim.x);
    const int32_t chunk = blk / t.tile_count;
    const int32_t tl = blk - chunk * t.tile_count;
    const int32_t tile = t.tiles ? t.tiles[t.tile_begin + tl] : t.tile_begin + tl;
    const int32_t cb = t.cell_off[tile], nc = t.cell_off[tile + 1] - cb;
    const int32_t vb0 = t.vert_off[tile], nv = t.vert_off[tile + 1] - vb0;
    const int32_t no = MODE == kOwner ? t.owned[tile] : nv;
    const int VS = t.vstride * P2;
    double* const Zs = lds;
    double* const Xs = lds + VS;
    double* const Ys = lds + 2 * VS;
    double* const Tx = lds + 3 * VS;
    double* const Ty = Tx + t.vstride;
    int32_t* const Ttag = (int32_t*)(Ty + t.vstride);
    int32_t* const Txst = Ttag + t.vstride;
    const int64_t n = a.xn;
    const double* const z = a.X + 2 * n;
    const double* const x = a.in0;
    double* const y = a.out0;
    const int lam = a.n_layers;
    const int la = chunk * (S - 1);                // first layer computed
    const int nlay = min(S, lam - la);             // layers computed
    const int lw0 = chunk == 0 ? 0 : 1;            // written levels: la + lw0 .. la + lw1
    const int lw1 = la + nlay == lam ? nlay : nlay - 1;
    (void)n_chunks;

    for (int v = tid; v < nv; v += kThreads) {
        const int32_t tag = t.verts[vb0 + v];
        const int32_t xs = column_start(t.xstart, t.xbase, t.xstep, vid(tag));
        Ttag[v] = tag;
        Txst[v] = xs;
        Tx[v] = a.X[xs];
        Ty[v] = a.X[n + xs];
    }
    lds_barrier();

    // copies: slot of vertex v holds levels la - s_v .. la - s_v + S + 1, s_v
    // the parity of its first level (16-byte aligned pairs)
    const int wave_e = tid & ~63;
    for (int e0 = 0; e0 < nv * PP; e0 += kThreads) {
        const int e = e0 + tid;
        const int v = e / PP, w = e - (e / PP) * PP;
        if (v >= nv) continue;
        const int32_t xs = Txst[v];
        const int sv = (xs + la) & 1;
        if (2 * w - sv > nlay) continue;           // levels la .. la + nlay
        const int64_t g = (int64_t)xs + la - sv + 2 * w;
        const bool wr = v < no;                    // a written vertex: its old output values too
        const bool zero = ATOMIC && vshared(Ttag[v]);
        if (g + 1 < n) {
            copy16(z + g, Zs + 2 * (e0 + wave_e));
            copy16(x + g, Xs + 2 * (e0 + wave_e));
            if (wr && !zero) copy16(y + g, Ys + 2 * (e0 + wave_e));
        } else {
            Zs[2 * e] = z[g];
            Xs[2 * e] = x[g];
            if (wr && !zero) Ys[2 * e] = y[g];
        }
        if (zero) {
            Ys[2 * e] = 0.0;
            Ys[2 * e + 1] = 0.0;
        }
    }

    // this thread's cells, layers r0 .. r0 + R - 1 of the chunk
    const int r0 = (tid & (G - 1)) * R;
    int vb[kPasses][3];
    double twoA[kPasses];
    bool has[kPasses];
    int wmask[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        const int c = tid / G + p * CPP;
        has[p] = c < nc;
        double xq[3], yq[3];
        wmask[p] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int lv = has[p] ? (int)t.lcv[(int64_t)(cb + c) * 3 + q] : 0;
            vb[p][q] = lv * P2 + ((Txst[lv] + la) & 1);
            xq[q] = Tx[lv];
            yq[q] = Ty[lv];
            wmask[p] |= (lv < no ? 1 : 0) << q;
        }
        twoA[p] = has[p] ? twice_area(xq, yq) : 0.0;
    }
    const int npass = (nc + CPP - 1) / CPP;
    wait_copies();
    lds_barrier();

#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
        if (p >= npass) break;
        if (!has[p] || r0 >= nlay) continue;
        int o[3];
        double zc[3], xc[3], acc[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            o[q] = vb[p][q] + r0;
            zc[q] = Zs[o[q]];
            xc[q] = Xs[o[q]];
            acc[q] = 0.0;
        }
        int r = 0;
#pragma unroll
        for (; r < R; ++r) {
            if (r0 + r >= nlay) break;
            double zn[3], xn[3], h[3], yb[3], yt[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                zn[q] = Zs[o[q] + r + 1];
                xn[q] = Xs[o[q] + r + 1];
                h[q] = zn[q] - zc[q];
            }
            p1_mass(twoA[p], h, xc, xn, yb, yt);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (MODE != kOwner || (wmask[p] >> q & 1)) lds_add(Ys + o[q] + r, acc[q] + yb[q]);
                acc[q] = yt[q];
                zc[q] = zn[q];
                xc[q] = xn[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (MODE != kOwner || (wmask[p] >> q & 1)) lds_add(Ys + o[q] + r, acc[q]);
    }
    lds_barrier();

    // write the chunk's levels la + lw0 .. la + lw1 of every written vertex
    const int nw = lw1 - lw0 + 1;
    for (int it = tid; it < no * nw; it += kThreads) {
        const int v = it / nw, jj = lw0 + (it - (it / nw) * nw);
        const int32_t xs = Txst[v];
        const double s = Ys[v * P2 + ((xs + la) & 1) + jj];
        const int64_t g = (int64_t)xs + la + jj;
        if (ATOMIC && vshared(Ttag[v]))
            unsafeAtomicAdd(y + g, s);
        else
            y[g] = s;
    }
}

size_t chunk_lds_bytes(int32_t vstride, int32_t S)
{
    return sizeof(double) * (3 * (size_t)vstride * (S + 2) + 2 * (size_t)vstride) + 2 * sizeof(int32_t) * vstride;
}

int32_t chunk_count(int32_t n_layers, int32_t S) { return n_layers <= S ? 1 : 1 + (n_layers - 2) / (S - 1); }

template <int S>
static void launch_chunk_s(int32_t race, const ColArgs& a, const TileArgs& t, int32_t nch, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)((int64_t)t.tile_count * nch)), block(kThreads);
    if (race == EXM_RACE_OWNER)
        hipLaunchKernelGGL((k_chunk_p1<S, kOwner>), grid, block, lds, s, a, t, nch);
    else if (race == EXM_RACE_COLOUR)
        hipLaunchKernelGGL((k_chunk_p1<S, kPlain>), grid, block, lds, s, a, t, nch);
    else
        hipLaunchKernelGGL((k_chunk_p1<S, kAtomic>), grid, block, lds, s, a, t, nch);
}

int32_t launch_chunked(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t S, size_t lds, hipStream_t s)
{
    if (t.tile_count <= 0) return EXM_OK;
    EXM_CHECK(P.kernel == EXM_K_MASS && P.element == EXM_ELEMENT_P1P1, EXM_EUNSUPPORTED,
              "the CHUNKED schedule runs the P1xP1 mass action only");
    const uintptr_t al = (uintptr_t)a.X | (uintptr_t)a.in0 | (uintptr_t)a.out0;
    EXM_CHECK((al & 15) == 0, EXM_EUNSUPPORTED, "the CHUNKED schedule needs 16-byte aligned field pointers");
    EXM_CHECK(P.race != EXM_RACE_OWNER || t.owned != nullptr, EXM_EINVAL, "owner-computes needs an owner plan");
    const int32_t nch = chunk_count(a.n_layers, S);
    EXM_CHECK((int64_t)t.tile_count * nch < INT32_MAX, EXM_EOVERFLOW, "too many workgroups");
    switch (S) {
    case 8: launch_chunk_s<8>(P.race, a, t, nch, lds, s); break;
    case 16: launch_chunk_s<16>(P.race, a, t, nch, lds, s); break;
    case 32: launch_chunk_s<32>(P.race, a, t, nch, lds, s); break;
    default: return fail(EXM_ERANGE, "chunk_layers = %d: the CHUNKED schedule takes 8, 16 or 32", S);
    }
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

// ---------------------------------------------------------------------------

static bool cubic_kernel(int32_t kernel)
{
    return kernel == EXM_K_CUBIC || kernel == EXM_K_CUBIC_VJP || kernel == EXM_K_CUBIC_FUSED;
}

// Spaces discontinuous horizontally: a cell's column belongs to that cell
// alone, so only z goes through LDS (the first four are discontinuous
// vertically too, the last two continuous).
static bool dg_element(int32_t element)
{
    return element == EXM_ELEMENT_DG0DG0 || element == EXM_ELEMENT_DG1DG1 || element == EXM_ELEMENT_DG0DG1 ||
           element == EXM_ELEMENT_DG1DG0 || element == EXM_ELEMENT_DG0P1 || element == EXM_ELEMENT_DG1P1;
}

static bool cgdg_element(int32_t element) { return element == EXM_ELEMENT_P1DG0 || element == EXM_ELEMENT_P1DG1; }

size_t pipe_lds_bytes(int32_t kernel, int32_t element, int32_t vstride, int32_t estride, int32_t cstride, int32_t S)
{
    if (kernel == EXM_K_MASS && cgdg_element(element)) {
        const int nv = element == EXM_ELEMENT_P1DG0 ? 1 : 2;
        return sizeof(double) * (2 * (size_t)vstride * (S + 2) + 3 * (size_t)vstride * (nv * S + 2)) +
               3 * sizeof(int32_t) * vstride;
    }
    if (cubic_kernel(kernel) && element == EXM_ELEMENT_P1P1) {
        const int nin = kernel == EXM_K_CUBIC_FUSED ? 3 : 2;
        const int nout = kernel == EXM_K_CUBIC ? 1 : (kernel == EXM_K_CUBIC_VJP ? 2 : 3);
        return sizeof(double) * (size_t)(2 + 2 * nin + nout) * (size_t)vstride * (S + 2) +
               2 * sizeof(int32_t) * vstride;
    }
    if (kernel != EXM_K_MASS) return 0;
    if (element == EXM_ELEMENT_P1P1)   // tag, column start, and a level range for columns of different heights
        return sizeof(double) * 5 * (size_t)vstride * (S + 2) + 4 * sizeof(int32_t) * vstride;
    if (element == EXM_ELEMENT_P2P2) {
        const size_t es = (size_t)vstride + (size_t)estride;
        return sizeof(double) * (2 * (size_t)vstride * (S + 2) + 3 * es * (2 * S + 2)) +
               sizeof(int32_t) * (2 * es + (size_t)vstride);
    }
    if (dg_element(element))   // column start, and a level range for columns of different heights
        return sizeof(double) * (2 * (size_t)vstride * (S + 2) + 2 * (size_t)vstride) + 3 * sizeof(int32_t) * vstride;
    return 0;
}

bool pipe_supported(int32_t kernel, int32_t element)
{
    if (cubic_kernel(kernel)) return element == EXM_ELEMENT_P1P1;
    return kernel == EXM_K_MASS && (element == EXM_ELEMENT_P1P1 || element == EXM_ELEMENT_P2P2 ||
                                    cgdg_element(element) || dg_element(element));
}

int32_t pipe_max_tile_cells(int32_t kernel, int32_t element, int32_t S)
{
    if (cubic_kernel(kernel) || cgdg_element(element)) return kThreads / S;   // one layer of one cell per thread
    if (dg_element(element)) return 2 * (512 / S);   // two passes of a 512-thread workgroup
    if (element == EXM_ELEMENT_P2P2) return kThreads / (S / kLayers2);
    return kPasses * (kThreads / (S / kLayers));
}

bool pipe_chunk_ok(int32_t kernel, int32_t element, int32_t S)
{
    if (cubic_kernel(kernel) || cgdg_element(element)) return S == 8 || S == 16;
    if (element == EXM_ELEMENT_P1P1) return S == 8 || S == 12 || S == 16 || S == 20 || S == 24 || S == 32;
    if (element == EXM_ELEMENT_P2P2) return S == 8 || S == 16;
    if (element == EXM_ELEMENT_DG0DG0 && dg0_long_chunk(S)) return true;
    return S == 8 || S == 16 || S == 32;
}

int32_t pipe_max_tile_verts(int32_t kernel, int32_t element, int32_t S)
{
    if (cgdg_element(element)) return kThreads * kItemsD / ((element == EXM_ELEMENT_P1DG0 ? 1 : 2) * S);
    return kThreads * (cubic_kernel(kernel) ? kItemsC : kItems) / S;
}

// The fixed-height P1 x P1 tile walk also runs in workgroups of 384 and 512
// threads (chunks of 8, 16 or 32 layers): its limits then, 0 where it does not.
int32_t pipe_p1_wide_max_cells(int32_t S) { return S == 8 || S == 16 || S == 32 ? kPasses * (512 / (S / kLayers)) : 0; }
int32_t pipe_p1_wide_max_verts(int32_t S) { return S == 8 || S == 16 || S == 32 ? 512 * kItems / S : 0; }

int32_t pipe_max_tile_entities(int32_t S) { return kThreads * kItems2 / (2 * S); }

template <int S, int NT>
static void launch_pipe_p1_nt(int32_t race, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count), block(NT);
    if (race == EXM_RACE_OWNER)
        hipLaunchKernelGGL((k_pipe_p1<S, kOwner, NT>), grid, block, lds, s, a, t);
    else if (race == EXM_RACE_COLOUR)
        hipLaunchKernelGGL((k_pipe_p1<S, kPlain, NT>), grid, block, lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_p1<S, kAtomic, NT>), grid, block, lds, s, a, t);
}

// Workgroup size of the fixed-height P1 tile walk: the smallest of 256, 384
// and 512 threads that takes every cell of the largest tile in one pass and
// its vertices x S levels in kItems items per thread; otherwise two passes
// of 256 (or 512) threads.
int32_t pipe_p1_threads(int32_t S, int32_t cells, int32_t verts)
{
    const int G = S / kLayers;
    const bool wide_ok = S == 8 || S == 16 || S == 32;
    for (int nt : {128, 192, 256, 384, 512}) {
        if (nt != 256 && !wide_ok) continue;
        if (cells * G <= nt && verts * S <= nt * kItems) return nt;
    }
    if (cells * G <= kPasses * 256 && verts * S <= 256 * kItems) return 256;
    return wide_ok ? 512 : 256;
}

template <int S>
static void launch_pipe_s(int32_t race, const ColArgs& a, const TileArgs& t, int32_t cstride, size_t lds,
                          hipStream_t s)
{
    if (t.vlo) {   // columns of different heights
        const dim3 grid((unsigned)t.tile_count), block(kThreads);
        if (race == EXM_RACE_COLOUR)
            hipLaunchKernelGGL((k_pipe_p1_var<S, kPlain>), grid, block, lds, s, a, t);
        else
            hipLaunchKernelGGL((k_pipe_p1_var<S, kAtomic>), grid, block, lds, s, a, t);
        return;
    }
    if constexpr (S == 8 || S == 16 || S == 32) {
        const int nt = pipe_p1_threads(S, cstride, t.vstride);
        if (nt == 512) return launch_pipe_p1_nt<S, 512>(race, a, t, lds, s);
        if (nt == 384) return launch_pipe_p1_nt<S, 384>(race, a, t, lds, s);
        if (nt == 192) return launch_pipe_p1_nt<S, 192>(race, a, t, lds, s);
        if (nt == 128) return launch_pipe_p1_nt<S, 128>(race, a, t, lds, s);
    }
    launch_pipe_p1_nt<S, kThreads>(race, a, t, lds, s);
}

int32_t launch_batch_pipe_dg0(const BatchPipeItem* items, const int32_t* units, int32_t n_units, int32_t S,
                              int32_t cstride, size_t lds, hipStream_t s)
{
    if (n_units <= 0) return EXM_OK;
    const dim3 grid((unsigned)n_units);
    // tiles beyond two cells per thread of a 256-thread workgroup take 512 threads
    const bool wide = cstride > 2 * (kThreads / S);
    switch (S) {
    case 8:
        if (wide)
            hipLaunchKernelGGL((k_batch_pipe_dg0<8, 2, 512>), grid, dim3(512), lds, s, items, units);
        else
            hipLaunchKernelGGL((k_batch_pipe_dg0<8, 2, 256>), grid, dim3(256), lds, s, items, units);
        break;
    case 16:
        if (wide)
            hipLaunchKernelGGL((k_batch_pipe_dg0<16, 2, 512>), grid, dim3(512), lds, s, items, units);
        else
            hipLaunchKernelGGL((k_batch_pipe_dg0<16, 2, 256>), grid, dim3(256), lds, s, items, units);
        break;
    case 32:
        if (wide)
            hipLaunchKernelGGL((k_batch_pipe_dg0<32, 2, 512>), grid, dim3(512), lds, s, items, units);
        else
            hipLaunchKernelGGL((k_batch_pipe_dg0<32, 2, 256>), grid, dim3(256), lds, s, items, units);
        break;
    case 34:   // 100 layers in three chunk steps
        if (wide)
            hipLaunchKernelGGL((k_batch_pipe_dg0<34, 2, 512>), grid, dim3(512), lds, s, items, units);
        else
            hipLaunchKernelGGL((k_batch_pipe_dg0<34, 2, 256>), grid, dim3(256), lds, s, items, units);
        break;
    default: return fail(EXM_ERANGE, "chunk_layers = %d: batched DG0 tiles take 8, 16, 32 or 34", S);
    }
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t launch_batch_pipe_p1(const BatchPipeItem* items, const int32_t* units, int32_t n_units, int32_t S,
                             bool shared, size_t lds, hipStream_t s)
{
    if (n_units <= 0) return EXM_OK;
    const dim3 grid((unsigned)n_units), block(kThreads);
    switch (S * 2 + (shared ? 1 : 0)) {
    case 16: hipLaunchKernelGGL((k_batch_pipe_p1<8, kOwner>), grid, block, lds, s, items, units); break;
    case 17: hipLaunchKernelGGL((k_batch_pipe_p1<8, kAtomic>), grid, block, lds, s, items, units); break;
    case 32: hipLaunchKernelGGL((k_batch_pipe_p1<16, kOwner>), grid, block, lds, s, items, units); break;
    case 33: hipLaunchKernelGGL((k_batch_pipe_p1<16, kAtomic>), grid, block, lds, s, items, units); break;
    default: return fail(EXM_ERANGE, "chunk_layers = %d: batched P1 tiles take 8 or 16", S);
    }
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

int32_t launch_zero_columns(const ZeroUnit* units, int32_t n_units, int32_t max_out, hipStream_t s)
{
    if (n_units <= 0 || max_out <= 0) return EXM_OK;
    EXM_CHECK(max_out <= 65535, EXM_ERANGE, "%d outputs per batch item exceed the grid", max_out);
    hipLaunchKernelGGL(k_zero_columns, dim3((unsigned)n_units, (unsigned)max_out), dim3(256), 0, s, units);
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

template <int FORM, int S, int NI>
static void launch_pipe_cubic_n(int32_t race, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count), block(kThreads);
    if (race == EXM_RACE_COLOUR)
        hipLaunchKernelGGL((k_pipe_cubic<FORM, S, kPlain, NI>), grid, block, lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_cubic<FORM, S, kAtomic, NI>), grid, block, lds, s, a, t);
}

// output items per thread: the fewest that cover the tiles' vertices x S
// levels (fewer items hold fewer old output values in registers)
template <int FORM, int S>
static void launch_pipe_cubic_f(int32_t race, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    if (t.vstride * S <= kThreads)
        launch_pipe_cubic_n<FORM, S, 1>(race, a, t, lds, s);
    else if (t.vstride * S <= 2 * kThreads)
        launch_pipe_cubic_n<FORM, S, 2>(race, a, t, lds, s);
    else
        launch_pipe_cubic_n<FORM, S, kItemsC>(race, a, t, lds, s);
}

template <int S>
static void launch_pipe_cubic(int32_t kernel, int32_t race, const ColArgs& a, const TileArgs& t, size_t lds,
                              hipStream_t s)
{
    if (kernel == EXM_K_CUBIC)
        launch_pipe_cubic_f<1, S>(race, a, t, lds, s);
    else if (kernel == EXM_K_CUBIC_VJP)
        launch_pipe_cubic_f<2, S>(race, a, t, lds, s);
    else
        launch_pipe_cubic_f<3, S>(race, a, t, lds, s);
}

template <int NV, int S>
static void launch_pipe_cgdg(int32_t race, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count), block(kThreads);
    if (race == EXM_RACE_COLOUR)
        hipLaunchKernelGGL((k_pipe_cgdg<NV, S, kPlain>), grid, block, lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_cgdg<NV, S, kAtomic>), grid, block, lds, s, a, t);
}

template <int S>
static void launch_pipe_p2(int32_t race, const ColArgs& a, const TileArgs& t, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count), block(kThreads);
    if (race == EXM_RACE_COLOUR)
        hipLaunchKernelGGL((k_pipe_p2<S, kPlain>), grid, block, lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_p2<S, kAtomic>), grid, block, lds, s, a, t);
}

template <int NH, int NV, int S>
static void launch_pipe_dg_e(const ColArgs& a, const TileArgs& t, int32_t cstride, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count);
    // tiles beyond two cells per thread of a 256-thread workgroup take 512 threads
    if (cstride > 2 * (kThreads / S))
        hipLaunchKernelGGL((k_pipe_dg<NH, NV, S, 2, 512>), grid, dim3(512), lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_dg<NH, NV, S, 2, 256>), grid, dim3(kThreads), lds, s, a, t);
}

template <int NH, int S>
static void launch_pipe_dgv_e(const ColArgs& a, const TileArgs& t, int32_t cstride, size_t lds, hipStream_t s)
{
    const dim3 grid((unsigned)t.tile_count);
    if (cstride > 2 * (kThreads / S))
        hipLaunchKernelGGL((k_pipe_dgv<NH, S, 2, 512>), grid, dim3(512), lds, s, a, t);
    else
        hipLaunchKernelGGL((k_pipe_dgv<NH, S, 2, 256>), grid, dim3(kThreads), lds, s, a, t);
}

template <int S>
static void launch_pipe_dg(int32_t element, const ColArgs& a, const TileArgs& t, int32_t cstride, size_t lds,
                           hipStream_t s)
{
    if constexpr (S == 20 || S == 26 || S == 34) {   // DG0 x DG0 on columns of one height only (checked by the caller)
        launch_pipe_dg_e<1, 1, S>(a, t, cstride, lds, s);
        return;
    }
    if (t.vlo) {   // columns of different heights (DG0 x DG0 only)
        const dim3 grid((unsigned)t.tile_count);
        if (cstride > 2 * (kThreads / S))
            hipLaunchKernelGGL((k_pipe_dg0_var<S, 2, 512>), grid, dim3(512), lds, s, a, t);
        else
            hipLaunchKernelGGL((k_pipe_dg0_var<S, 2, 256>), grid, dim3(kThreads), lds, s, a, t);
        return;
    }
    switch (element) {
    case EXM_ELEMENT_DG0P1: launch_pipe_dgv_e<1, S>(a, t, cstride, lds, s); break;
    case EXM_ELEMENT_DG1P1: launch_pipe_dgv_e<3, S>(a, t, cstride, lds, s); break;
    case EXM_ELEMENT_DG0DG0: launch_pipe_dg_e<1, 1, S>(a, t, cstride, lds, s); break;
    case EXM_ELEMENT_DG0DG1: launch_pipe_dg_e<1, 2, S>(a, t, cstride, lds, s); break;
    case EXM_ELEMENT_DG1DG0: launch_pipe_dg_e<3, 1, S>(a, t, cstride, lds, s); break;
    default: launch_pipe_dg_e<3, 2, S>(a, t, cstride, lds, s); break;   // DG1 x DG1
    }
}

int32_t launch_pipe(const LoopLaunch& P, const ColArgs& a, const TileArgs& t, int32_t cstride, int32_t S, size_t lds,
                    hipStream_t s)
{
    if (t.tile_count <= 0) return EXM_OK;
    EXM_CHECK(pipe_supported(P.kernel, P.element), EXM_EUNSUPPORTED,
              "the PIPELINED schedule runs the mass action on every space but the mixed-degree one, and the "
              "cubic forms on P1xP1");
    const uintptr_t al = (uintptr_t)a.X | (uintptr_t)a.in0 | (uintptr_t)a.in1 | (uintptr_t)a.in2 | (uintptr_t)a.out0;
    EXM_CHECK((al & 15) == 0, EXM_EUNSUPPORTED, "the PIPELINED schedule needs 16-byte aligned field pointers");
    if (cubic_kernel(P.kernel)) {
        EXM_CHECK(P.race != EXM_RACE_OWNER, EXM_EUNSUPPORTED, "owner-computes is for the mass action");
        switch (S) {
        case 8: launch_pipe_cubic<8>(P.kernel, P.race, a, t, lds, s); break;
        case 16: launch_pipe_cubic<16>(P.kernel, P.race, a, t, lds, s); break;
        default: return fail(EXM_ERANGE, "chunk_layers = %d: the PIPELINED schedule takes 8 or 16 on the cubic forms", S);
        }
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    if (cgdg_element(P.element)) {
        EXM_CHECK(P.race != EXM_RACE_OWNER, EXM_EUNSUPPORTED, "owner-computes is for the P1xP1 mass action");
        const bool dg1 = P.element == EXM_ELEMENT_P1DG1;
        switch (S) {
        case 8: dg1 ? launch_pipe_cgdg<2, 8>(P.race, a, t, lds, s) : launch_pipe_cgdg<1, 8>(P.race, a, t, lds, s); break;
        case 16:
            dg1 ? launch_pipe_cgdg<2, 16>(P.race, a, t, lds, s) : launch_pipe_cgdg<1, 16>(P.race, a, t, lds, s);
            break;
        default: return fail(EXM_ERANGE, "chunk_layers = %d: the PIPELINED schedule takes 8 or 16 on CG1xDG*", S);
        }
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    if (P.element == EXM_ELEMENT_P2P2) {
        EXM_CHECK(P.race != EXM_RACE_OWNER, EXM_EUNSUPPORTED, "owner-computes is not available on P2xP2");
        EXM_CHECK(t.edge_off != nullptr, EXM_EINVAL, "P2 needs the mesh's cell_edge map");
        switch (S) {
        case 8: launch_pipe_p2<8>(P.race, a, t, lds, s); break;
        case 16: launch_pipe_p2<16>(P.race, a, t, lds, s); break;
        default: return fail(EXM_ERANGE, "chunk_layers = %d: the PIPELINED schedule takes 8 or 16 on P2xP2", S);
        }
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    if (P.element != EXM_ELEMENT_P1P1) {
        EXM_CHECK(!t.vlo || P.element == EXM_ELEMENT_DG0DG0, EXM_EUNSUPPORTED,
                  "the PIPELINED schedule runs P1xP1 and DG0xDG0 on columns of different heights");
        switch (S) {
        case 8: launch_pipe_dg<8>(P.element, a, t, cstride, lds, s); break;
        case 16: launch_pipe_dg<16>(P.element, a, t, cstride, lds, s); break;
        case 32: launch_pipe_dg<32>(P.element, a, t, cstride, lds, s); break;
        case 20:
        case 26:
        case 34:
            EXM_CHECK(P.element == EXM_ELEMENT_DG0DG0 && !t.vlo, EXM_ERANGE,
                      "chunk_layers = %d: the PIPELINED schedule takes it on DG0xDG0 with columns of one height", S);
            if (S == 20)
                launch_pipe_dg<20>(P.element, a, t, cstride, lds, s);
            else if (S == 26)
                launch_pipe_dg<26>(P.element, a, t, cstride, lds, s);
            else
                launch_pipe_dg<34>(P.element, a, t, cstride, lds, s);
            break;
        default: return fail(EXM_ERANGE, "chunk_layers = %d: the PIPELINED schedule takes 8, 16 or 32", S);
        }
        EXM_TRY_HIP(hipGetLastError());
        return EXM_OK;
    }
    EXM_CHECK(P.race != EXM_RACE_OWNER || t.owned != nullptr, EXM_EINVAL, "owner-computes needs an owner plan");
    switch (S) {
    case 8: launch_pipe_s<8>(P.race, a, t, cstride, lds, s); break;
    case 12: launch_pipe_s<12>(P.race, a, t, cstride, lds, s); break;
    case 16: launch_pipe_s<16>(P.race, a, t, cstride, lds, s); break;
    case 20: launch_pipe_s<20>(P.race, a, t, cstride, lds, s); break;
    case 24: launch_pipe_s<24>(P.race, a, t, cstride, lds, s); break;
    case 32: launch_pipe_s<32>(P.race, a, t, cstride, lds, s); break;
    default: return fail(EXM_ERANGE, "chunk_layers = %d: the PIPELINED schedule takes 8, 12, 16, 20, 24 or 32 on P1xP1", S);
    }
    EXM_TRY_HIP(hipGetLastError());
    return EXM_OK;
}

}  // namespace exm
