// The coordinate field: placement of per-(vertex, level) coordinates into a
// P1 x P1 vector field, and the check that every vertex column is vertical.
//
// Section 4.1.1 carries the geometry as a vector-valued P1 x P1 field: a
// d-vector at every extruded vertex.  The element kernels of this library
// read (x, y) once per vertex column (at its first level) and z at every
// level, so they are exact only when x and y do not change along a column.
// A field is checked once per (space, address) before a loop uses it; the
// loop refuses a leaning column with EXM_EUNSUPPORTED rather than integrate
// over the wrong prism.
#include <algorithm>

#include "exm_internal.hpp"

namespace exm {

namespace {

// Levels lo .. hi of vertex column v (a uniform mesh: 0 .. n_layers).
struct VertexLevels {
    const int32_t* lo;   // [N0] or null
    const int32_t* hi;   // [N0] or null
    int32_t n_layers;
    __device__ __forceinline__ void get(int32_t v, int32_t& l0, int32_t& l1) const
    {
        l0 = lo ? lo[v] : 0;
        l1 = hi ? hi[v] : n_layers;
    }
};

// One thread per (vertex, level) of the full level grid: level l of vertex v
// is index v * (n_layers + 1) + l.  A thread whose level lies inside the
// vertex column compares the field's x and y at that level with those at the
// column's first level and records the vertex (+1) on a mismatch.
__global__ void k_field_vertical(const double* __restrict__ X, int64_t n_dofs, const int32_t* __restrict__ starts,
                                 int32_t n_vert, VertexLevels lv, int32_t* __restrict__ bad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nl = lv.n_layers + 1;
    if (t >= (int64_t)n_vert * nl) return;
    const int32_t v = (int32_t)(t / nl);
    const int32_t l = (int32_t)(t - (int64_t)v * nl);
    int32_t l0, l1;
    lv.get(v, l0, l1);
    if (l <= l0 || l > l1) return;
    const int64_t s = starts[v];
    const int64_t d = s + (l - l0);
    if (X[d] != X[s] || X[n_dofs + d] != X[n_dofs + s]) *bad = v + 1;
}

// The same check on per-(vertex, level) input xyz [N0 * (n_layers + 1) * 3].
__global__ void k_xyz_vertical(const double* __restrict__ xyz, int32_t n_vert, VertexLevels lv,
                               int32_t* __restrict__ bad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nl = lv.n_layers + 1;
    if (t >= (int64_t)n_vert * nl) return;
    const int32_t v = (int32_t)(t / nl);
    const int32_t l = (int32_t)(t - (int64_t)v * nl);
    int32_t l0, l1;
    lv.get(v, l0, l1);
    if (l <= l0 || l > l1) return;
    const double* p = xyz + 3 * t;
    const double* q = xyz + 3 * ((int64_t)v * nl + l0);
    if (p[0] != q[0] || p[1] != q[1]) *bad = v + 1;
}

// Component i of level l of vertex v goes to X[i * n_dofs + S(v) + l - lo(v)].
__global__ void k_place_coords(const double* __restrict__ xyz, int32_t n_vert, VertexLevels lv,
                               const int32_t* __restrict__ starts, int64_t n_dofs, double* __restrict__ X)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nl = lv.n_layers + 1;
    if (t >= (int64_t)n_vert * nl) return;
    const int32_t v = (int32_t)(t / nl);
    const int32_t l = (int32_t)(t - (int64_t)v * nl);
    int32_t l0, l1;
    lv.get(v, l0, l1);
    if (l < l0 || l > l1) return;
    const int64_t d = (int64_t)starts[v] + (l - l0);
    const double* p = xyz + 3 * t;
    X[d] = p[0];
    X[n_dofs + d] = p[1];
    X[2 * n_dofs + d] = p[2];
}

constexpr int kBlock = 256;

VertexLevels levels_of(const exm_mesh* m)
{
    VertexLevels lv;
    lv.lo = m->variable ? m->d_vert_lo.p : nullptr;
    lv.hi = m->variable ? m->d_vert_hi.p : nullptr;
    lv.n_layers = m->n_layers;
    return lv;
}

int32_t check_coord_space(const exm_space* space)
{
    EXM_CHECK(space != nullptr, EXM_EINVAL, "space is NULL");
    EXM_CHECK(space->element == EXM_ELEMENT_P1P1, EXM_EINVAL, "coordinates live on a P1xP1 space (element %d)",
              space->element);
    return EXM_OK;
}

// Run `launch` (which writes a vertex + 1 into the flag on a leaning column)
// on `stream` and wait for the verdict.
template <class Launch>
int32_t run_check(const exm_space* space, hipStream_t stream, Launch launch, int32_t* bad_vertex)
{
    std::lock_guard<std::mutex> lk(space->coords_mu);
    if (!space->coords_flag.p) {
        int32_t s = space->coords_flag.alloc(1);
        if (s != EXM_OK) return s;
    }
    int32_t* flag = space->coords_flag.p;
    EXM_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), stream));
    launch(flag);
    EXM_TRY_HIP(hipGetLastError());
    int32_t h = 0;
    EXM_TRY_HIP(hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    EXM_TRY_HIP(hipStreamSynchronize(stream));
    *bad_vertex = h - 1;
    return EXM_OK;
}

void remember(const exm_space* space, const void* X, bool ok)
{
    std::lock_guard<std::mutex> lk(space->coords_mu);
    auto& v = space->coords_ok;
    auto it = std::find(v.begin(), v.end(), X);
    if (ok && it == v.end()) v.push_back(X);
    if (!ok && it != v.end()) v.erase(it);
}

int32_t verify_field(const exm_space* space, const double* X, hipStream_t stream)
{
    const exm_mesh* m = space->mesh;
    const int64_t total = (int64_t)m->n[0] * (m->n_layers + 1);
    int32_t bad = -1;
    int32_t s = run_check(space, stream, [&](int32_t* flag) {
        hipLaunchKernelGGL(k_field_vertical, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, stream,
                           X, space->n_dofs, space->d_starts[0].p, m->n[0], levels_of(m), flag);
    }, &bad);
    if (s != EXM_OK) return s;
    remember(space, X, bad < 0);
    EXM_CHECK(bad < 0, EXM_EUNSUPPORTED,
              "the coordinate field leans: x or y of vertex %d changes along its column (the element kernels need "
              "vertical columns)", bad);
    return EXM_OK;
}

}  // namespace

int32_t ensure_vertical(const exm_space* space, const void* X, hipStream_t stream)
{
    {
        std::lock_guard<std::mutex> lk(space->coords_mu);
        const auto& v = space->coords_ok;
        if (std::find(v.begin(), v.end(), X) != v.end()) return EXM_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    EXM_TRY_HIP(hipStreamIsCapturing(stream, &cs));
    EXM_CHECK(cs == hipStreamCaptureStatusNone, EXM_EINVAL,
              "the coordinate field has not been checked for vertical columns: call exm_coordinates_verify (or "
              "build it with exm_space_coordinates) before capturing the stream");
    return verify_field(space, (const double*)X, stream);
}

}  // namespace exm

using namespace exm;

extern "C" {

int32_t exm_space_coordinates(const exm_space* space, const double* xyz, int32_t xyz_on_device, double* X,
                              void* stream)
{
    clear_error();
    int32_t s = check_coord_space(space);
    if (s != EXM_OK) return s;
    EXM_CHECK(xyz != nullptr && X != nullptr, EXM_EINVAL, "xyz or X is NULL");
    EXM_CHECK(xyz_on_device == 0 || xyz_on_device == 1, EXM_EINVAL, "xyz_on_device must be 0 or 1");
    s = check_pending();
    if (s != EXM_OK) return s;
    const exm_mesh* m = space->mesh;
    const int32_t nl = m->n_layers + 1;
    const int64_t total = (int64_t)m->n[0] * nl;
    hipStream_t st = (hipStream_t)stream;
    DevBuf<double> staged;
    const double* dxyz = xyz;
    if (!xyz_on_device) {
        // host input: checked here, before anything reaches the device
        for (int32_t v = 0; v < m->n[0]; ++v) {
            const int32_t l0 = m->variable ? m->lo[0][v] : 0;
            const int32_t l1 = m->variable ? m->hi[0][v] : m->n_layers;
            const double* q = xyz + 3 * ((int64_t)v * nl + l0);
            for (int32_t l = l0 + 1; l <= l1; ++l) {
                const double* p = xyz + 3 * ((int64_t)v * nl + l);
                EXM_CHECK(p[0] == q[0] && p[1] == q[1], EXM_EUNSUPPORTED,
                          "vertex %d leans: its x or y at level %d differs from level %d (the element kernels need "
                          "vertical columns)", v, l, l0);
            }
        }
        if ((s = staged.upload(xyz, (size_t)total * 3)) != EXM_OK) return s;
        dxyz = staged.p;
    } else {
        int32_t bad = -1;
        s = run_check(space, st, [&](int32_t* flag) {
            hipLaunchKernelGGL(k_xyz_vertical, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                               xyz, m->n[0], levels_of(m), flag);
        }, &bad);
        if (s != EXM_OK) return s;
        EXM_CHECK(bad < 0, EXM_EUNSUPPORTED,
                  "vertex %d leans: its x or y changes along its column (the element kernels need vertical columns)",
                  bad);
    }
    hipLaunchKernelGGL(k_place_coords, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, dxyz,
                       m->n[0], levels_of(m), space->d_starts[0].p, space->n_dofs, X);
    EXM_TRY_HIP(hipGetLastError());
    if (!xyz_on_device) EXM_TRY_HIP(hipStreamSynchronize(st));   // the staged copy is freed on return
    remember(space, X, true);
    return EXM_OK;
}

int32_t exm_coordinates_verify(const exm_space* space, const double* X, void* stream)
{
    clear_error();
    int32_t s = check_coord_space(space);
    if (s != EXM_OK) return s;
    EXM_CHECK(X != nullptr, EXM_EINVAL, "X is NULL");
    s = check_pending();
    if (s != EXM_OK) return s;
    return verify_field(space, X, (hipStream_t)stream);
}

}  // extern "C"
