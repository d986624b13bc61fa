/*
 * CPU oracle for the extruded-mesh numbering and column iteration of
 * Bercea et al., "A structure-exploiting numbering algorithm for finite
 * elements on extruded meshes" (arXiv 1604.05937).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the HIP
 * path is checked against.  It shares no code with the HIP library and must
 * never be linked into, or called from, the product path.
 *
 * Everything here is written for clarity, not speed: FP64 throughout, no
 * blocking, no fusion, the numbering as a literal counter loop and the cell
 * loop exactly in the paper's order, with the element integrals evaluated by
 * quadrature with a full Jacobian at every quadrature point.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* delta[(d1)*2 + d2] = number of DoFs attached to an extruded entity of type
 * (d1, d2): d1 the horizontal (base) dimension 0..2, d2 the vertical
 * dimension 0..1 (Section 3.1.2 entity pairs, Section 3.2). */
#define DELTA(delta, d1, d2) ((delta)[(d1) * 2 + (d2)])

/*
 * Algorithm 1 (Section 3.2): vertical-innermost numbering.
 *
 * Base entities (d1, i) are visited dimension by dimension (d1 = 0, 1, 2) and
 * by index within a dimension; for each, the layers l = 0..lam-1 are visited
 * and, inside a layer, first the horizontal entity (d1, 0) at level l and then
 * the vertical entity (d1, 1) over interval l receive the next delta numbers;
 * finally the top horizontal entity (d1, 0) at level lam.
 *
 * Output: first_d[d1][(i*(lam+1) + l)*2 + d2] = first DoF number of entity
 * ((d1, d2), (i, l)), or -1 for the non-existent vertical entity at l = lam.
 * The entity's DoFs are first .. first + delta - 1.  Returns the DoF count.
 */
int64_t oracle_alg1_number(const int32_t counts[3], int32_t lam, const int32_t delta[6],
                           int64_t* first0, int64_t* first1, int64_t* first2)
{
    int64_t* first[3] = {first0, first1, first2};
    int64_t c = 0;
    for (int d1 = 0; d1 < 3; ++d1) {
        for (int64_t i = 0; i < counts[d1]; ++i) {
            /* a NULL table (a dimension without DoFs) still advances the counter */
            int64_t* f = first[d1] ? first[d1] + i * (int64_t)(lam + 1) * 2 : NULL;
            for (int32_t l = 0; l < lam; ++l) {
                for (int d2 = 0; d2 < 2; ++d2) {
                    if (f) f[l * 2 + d2] = c;
                    c += DELTA(delta, d1, d2);
                }
            }
            if (f) f[lam * 2 + 0] = c;
            c += DELTA(delta, d1, 0);
            if (f) f[lam * 2 + 1] = -1;
        }
    }
    return c;
}

/*
 * Algorithm 1 with a layer range per entity column (the constant layer count
 * of the paper's exposition relaxed, Section 3.1): entity (d1, i) spans the
 * layers lo[d1][i] .. hi[d1][i] - 1, i.e. the levels lo .. hi.  The counter
 * visits, for each entity, its layers in order -- horizontal entity at the
 * layer's bottom level, then the vertical entity -- and finally its top level.
 * first_d[d1][(i*(lam_max+1) + l)*2 + d2] as in oracle_alg1_number with the
 * absolute level l; -1 outside the entity's range.
 */
int64_t oracle_alg1_number_var(const int32_t counts[3], int32_t lam_max, const int32_t delta[6],
                               const int32_t* lo0, const int32_t* hi0, const int32_t* lo1, const int32_t* hi1,
                               const int32_t* lo2, const int32_t* hi2,
                               int64_t* first0, int64_t* first1, int64_t* first2)
{
    int64_t* first[3] = {first0, first1, first2};
    const int32_t* lo[3] = {lo0, lo1, lo2};
    const int32_t* hi[3] = {hi0, hi1, hi2};
    int64_t c = 0;
    for (int d1 = 0; d1 < 3; ++d1) {
        for (int64_t i = 0; i < counts[d1]; ++i) {
            int64_t* f = first[d1] ? first[d1] + i * (int64_t)(lam_max + 1) * 2 : NULL;
            const int32_t a = lo[d1] ? lo[d1][i] : 0, b = hi[d1] ? hi[d1][i] : lam_max;
            for (int32_t l = a; l < b; ++l) {
                for (int d2 = 0; d2 < 2; ++d2) {
                    if (f) f[l * 2 + d2] = c;
                    c += DELTA(delta, d1, d2);
                }
            }
            if (f) f[b * 2 + 0] = c;
            c += DELTA(delta, d1, 0);
        }
    }
    return c;
}

/* The explicit lists for a layer range per cell: L(c) is the stencil of the
 * cell's bottom prism (layer cell_lo[c]); the offsets are those of
 * oracle_stencil. */
int32_t oracle_stencil_var(int32_t n_cells, int32_t lam_max, const int32_t delta[6], const int32_t* cell_vertex,
                           const int32_t* cell_edge, const int32_t* cell_lo,
                           const int64_t* first0, const int64_t* first1, const int64_t* first2, int64_t* lmap)
{
    const int64_t* first[3] = {first0, first1, first2};
    int32_t k = 0;
    for (int e = 0; e < 7; ++e) {
        int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
        k += 2 * DELTA(delta, d, 0) + DELTA(delta, d, 1);
    }
    for (int64_t c = 0; c < n_cells; ++c) {
        int64_t* row = lmap + c * k;
        int32_t p = 0;
        const int64_t b = cell_lo[c];
        for (int e = 0; e < 7; ++e) {
            int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
            int64_t i;
            if (d == 0) i = cell_vertex[c * 3 + e];
            else if (d == 1) i = cell_edge ? cell_edge[c * 3 + (e - 3)] : -1;
            else i = c;
            int nh = DELTA(delta, d, 0), nv = DELTA(delta, d, 1);
            if (nh + nv == 0) continue;
            const int64_t* f = first[d] + (i * (int64_t)(lam_max + 1) + b) * 2;
            for (int j = 0; j < nh; ++j) row[p++] = f[0 * 2 + 0] + j;   /* bottom level of the cell's first layer */
            for (int j = 0; j < nh; ++j) row[p++] = f[1 * 2 + 0] + j;   /* its top level */
            for (int j = 0; j < nv; ++j) row[p++] = f[0 * 2 + 1] + j;   /* its vertical entity */
        }
    }
    return k;
}

/*
 * The stencil of a prism (the explicit list L of Section 3.3): the DoFs of
 * all entities in the closure of base cell c extruded over one layer.  The
 * closure entities are taken in the order vertex 0, 1, 2 (cell_vertex order),
 * edge 0, 1, 2 (edge a opposite vertex a) and the cell itself; for each, its
 * delta(d,0) DoFs on the bottom horizontal entity, then its delta(d,0) DoFs on
 * the top horizontal entity, then its delta(d,1) DoFs on the vertical entity.
 *
 * Algorithm 2: the vertical offset of stencil position p is
 * delta(d,0) + delta(d,1), d the base entity dimension of position p.
 *
 * Writes L for layer 0 into lmap[c*k + p] (k = stencil size), offsets[p],
 * entity_dim[p]; returns k.
 */
int32_t oracle_stencil(int32_t n_cells, int32_t lam, const int32_t delta[6],
                       const int32_t* cell_vertex, const int32_t* cell_edge,
                       const int64_t* first0, const int64_t* first1, const int64_t* first2,
                       int64_t* lmap, int32_t* offsets, int32_t* entity_dim)
{
    const int64_t* first[3] = {first0, first1, first2};
    int32_t k = 0;
    /* Algorithm 2 over the stencil layout (same for every cell). */
    for (int e = 0; e < 7; ++e) {
        int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
        int n = 2 * DELTA(delta, d, 0) + DELTA(delta, d, 1);
        for (int j = 0; j < n; ++j) {
            if (offsets) offsets[k] = DELTA(delta, d, 0) + DELTA(delta, d, 1);
            if (entity_dim) entity_dim[k] = d;
            ++k;
        }
    }
    if (!lmap) return k;
    for (int64_t c = 0; c < n_cells; ++c) {
        int64_t* row = lmap + c * k;
        int32_t p = 0;
        for (int e = 0; e < 7; ++e) {
            int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
            int64_t i;
            if (d == 0) i = cell_vertex[c * 3 + e];
            else if (d == 1) i = cell_edge ? cell_edge[c * 3 + (e - 3)] : -1;
            else i = c;
            int nh = DELTA(delta, d, 0), nv = DELTA(delta, d, 1);
            if (nh + nv == 0) continue;
            const int64_t* f = first[d] + i * (int64_t)(lam + 1) * 2;
            for (int j = 0; j < nh; ++j) row[p++] = f[0 * 2 + 0] + j;   /* bottom, level 0 */
            for (int j = 0; j < nh; ++j) row[p++] = f[1 * 2 + 0] + j;   /* top, level 1 */
            for (int j = 0; j < nv; ++j) row[p++] = f[0 * 2 + 1] + j;   /* vertical, interval 0 */
        }
    }
    return k;
}

/* Forms evaluated by the oracle's element kernel. */
enum {
    ORACLE_MASS = 1,        /* out0 (+)= int in0 * v                              */
    ORACLE_CUBIC = 2,       /* out0 += int (in0^3 - in1) v                         */
    ORACLE_CUBIC_VJP = 3,   /* out0 += int 3 in0^2 in1 v ; out1 += -int in1 v      */
    ORACLE_CUBIC_JVP = 4,   /* out0 += int (3 in0^2 in1 - in2) v                   */
    ORACLE_CUBIC_FUSED = 5, /* out0 += int (u^3-f) v; out1 += int 3u^2 w v; out2 += -int w v
                               with u = in0, f = in1, w = in2                      */
    /* Magnitude forms: the same sums with every factor replaced by its absolute
     * value.  They bound the rounding error of any summation order of the
     * corresponding form and scale the componentwise parity tolerance. */
    ORACLE_MASS_ABS = 6,    /* out0 += int |in0| |v|                               */
    ORACLE_CUBIC_ABS = 7,   /* out0 += int (|in0|^3 + |in1|) |v|                   */
    ORACLE_VJP_ABS = 8      /* out0 += int 3 in0^2 |in1| |v| ; out1 += int |in1| |v| */
};

static double det3(const double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/*
 * Algorithm 3 (Section 3.3): iterate a stencil function over the prisms of
 * the extruded mesh.  For each base cell, the explicit lists are read once and
 * then, layer by layer, the kernel is applied and every DoF index is advanced
 * by its vertical offset.
 *
 * Two function spaces are involved, each with its own list (end of Section
 * 3.3): the coordinate space (P1 x P1, a 3-vector per DoF, stored [dof][xyz])
 * and the space V of the fields.  The kernel integrates its form with the
 * quadrature rule (qw, reference points implicit in the tabulations):
 *   phix[q*6 + p], dphix[(q*6 + p)*3 + r]  coordinate basis and its reference
 *                                           derivatives d/dxi, d/deta, d/dzeta
 *   phiv[q*k + p]                           basis of V
 * and |det J| of the full 3x3 Jacobian at every point.
 *
 * cells: the base cells to visit (NULL: all 0..n_iter-1).
 * cell_lam: layers of each cell's column (NULL: lam for every column); the
 * lists then hold the DoFs of the column's bottom prism.
 * write_mode: 1 = WRITE (assign), 0 = INC (add) for the outputs.
 */
void oracle_par_loop(int32_t form, int64_t n_iter, const int64_t* cells, int32_t lam, const int32_t* cell_lam,
                     const int64_t* mapx, const int32_t* offx, const double* X,
                     int32_t k, const int64_t* mapv, const int32_t* offv,
                     const double* in0, const double* in1, const double* in2,
                     double* out0, double* out1, double* out2, int32_t write_mode,
                     int32_t nq, const double* qw, const double* phix, const double* dphix,
                     const double* phiv)
{
    int64_t dx[6];
    int64_t* dv = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    double* e0 = (double*)malloc(sizeof(double) * (size_t)k);
    double* e1 = (double*)malloc(sizeof(double) * (size_t)k);
    double* e2 = (double*)malloc(sizeof(double) * (size_t)k);
    for (int64_t it = 0; it < n_iter; ++it) {
        int64_t c = cells ? cells[it] : it;
        /* (dof_0, ..., dof_{k-1}) <- L(c), for both spaces */
        for (int p = 0; p < 6; ++p) dx[p] = mapx[c * 6 + p];
        for (int p = 0; p < k; ++p) dv[p] = mapv[c * k + p];
        const int32_t nl = cell_lam ? cell_lam[c] : lam;   /* layers of this column */
        for (int32_t l = 0; l < nl; ++l) {
            /* S(f(dof_0), ..., f(dof_{k-1})): the element kernel */
            for (int p = 0; p < k; ++p) e0[p] = e1[p] = e2[p] = 0.0;
            for (int q = 0; q < nq; ++q) {
                double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int p = 0; p < 6; ++p)
                    for (int i = 0; i < 3; ++i)
                        for (int r = 0; r < 3; ++r)
                            J[i][r] += X[dx[p] * 3 + i] * dphix[(q * 6 + p) * 3 + r];
                double w = qw[q] * fabs(det3(J));
                double a = 0.0, b = 0.0, g = 0.0;
                const int absf = form >= ORACLE_MASS_ABS;
                for (int p = 0; p < k; ++p) {
                    double ph = absf ? fabs(phiv[q * k + p]) : phiv[q * k + p];
                    if (in0) a += (absf ? fabs(in0[dv[p]]) : in0[dv[p]]) * ph;
                    if (in1) b += (absf ? fabs(in1[dv[p]]) : in1[dv[p]]) * ph;
                    if (in2) g += (absf ? fabs(in2[dv[p]]) : in2[dv[p]]) * ph;
                }
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
                switch (form) {
                case ORACLE_MASS: s0 = a; break;
                case ORACLE_CUBIC: s0 = a * a * a - b; break;
                case ORACLE_CUBIC_VJP: s0 = 3.0 * a * a * b; s1 = -b; break;
                case ORACLE_CUBIC_JVP: s0 = 3.0 * a * a * b - g; break;
                case ORACLE_CUBIC_FUSED: s0 = a * a * a - b; s1 = 3.0 * a * a * g; s2 = -g; break;
                case ORACLE_MASS_ABS: s0 = a; break;
                case ORACLE_CUBIC_ABS: s0 = a * a * a + b; break;
                case ORACLE_VJP_ABS: s0 = 3.0 * a * a * b; s1 = b; break;
                default: break;
                }
                for (int p = 0; p < k; ++p) {
                    double ph = absf ? fabs(phiv[q * k + p]) : phiv[q * k + p];
                    e0[p] += w * s0 * ph;
                    e1[p] += w * s1 * ph;
                    e2[p] += w * s2 * ph;
                }
            }
            for (int p = 0; p < k; ++p) {
                if (write_mode) {
                    if (out0) out0[dv[p]] = e0[p];
                    if (out1) out1[dv[p]] = e1[p];
                    if (out2) out2[dv[p]] = e2[p];
                } else {
                    if (out0) out0[dv[p]] += e0[p];
                    if (out1) out1[dv[p]] += e1[p];
                    if (out2) out2[dv[p]] += e2[p];
                }
            }
            /* dof_j <- dof_j + offset(j) */
            for (int p = 0; p < 6; ++p) dx[p] += offx[p];
            for (int p = 0; p < k; ++p) dv[p] += offv[p];
        }
    }
    free(dv);
    free(e0);
    free(e1);
    free(e2);
}

/*
 * Matrix of a bilinear form, assembled by the same column iteration
 * (Algorithm 3; Section 5 names the assembly of the global system matrix as
 * the next use of the vertical structure).  For every prism, in Algorithm 3's
 * order, the element matrix
 *     A_e[p][j] = integral of s(x) phi_j phi_p |det J|
 * is computed by quadrature and emitted as k * k triplets (row dof_p,
 * column dof_j, value A_e[p][j]); the matrix is the sum of the triplets with
 * equal (row, column).
 *   form 1: mass, s = 1;
 *   form 2: Jacobian of the cubic residual integral (u^3 - f) v with respect
 *           to u, s = 3 u^2 (u = in0 on V);
 *   form 3, 4: the same with |phi| and |u| (the scales of the rounding error
 *           of any summation order).
 * cells: the base cells to visit (NULL: all 0 .. n_iter - 1).
 * rows, cols, vals: n_iter * lam * k * k entries each.
 */
void oracle_assemble(int32_t form, int64_t n_iter, const int64_t* cells, int32_t lam,
                     const int64_t* mapx, const int32_t* offx, const double* X,
                     int32_t k, const int64_t* mapv, const int32_t* offv, const double* in0,
                     int64_t* rows, int64_t* cols, double* vals,
                     int32_t nq, const double* qw, const double* phix, const double* dphix,
                     const double* phiv)
{
    int64_t dx[6];
    int64_t* dv = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    double* Ae = (double*)malloc(sizeof(double) * (size_t)k * (size_t)k);
    const int absf = form >= 3;
    const int jac = form == 2 || form == 4;
    int64_t t = 0;
    for (int64_t it = 0; it < n_iter; ++it) {
        const int64_t c = cells ? cells[it] : it;
        for (int p = 0; p < 6; ++p) dx[p] = mapx[c * 6 + p];
        for (int p = 0; p < k; ++p) dv[p] = mapv[c * k + p];
        for (int32_t l = 0; l < lam; ++l) {
            for (int64_t e = 0; e < (int64_t)k * k; ++e) Ae[e] = 0.0;
            for (int q = 0; q < nq; ++q) {
                double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
                for (int p = 0; p < 6; ++p)
                    for (int i = 0; i < 3; ++i)
                        for (int r = 0; r < 3; ++r)
                            J[i][r] += X[dx[p] * 3 + i] * dphix[(q * 6 + p) * 3 + r];
                double s = qw[q] * fabs(det3(J));
                if (jac) {
                    double u = 0.0;
                    for (int p = 0; p < k; ++p)
                        u += (absf ? fabs(in0[dv[p]]) : in0[dv[p]]) * (absf ? fabs(phiv[q * k + p]) : phiv[q * k + p]);
                    s *= 3.0 * u * u;
                }
                for (int p = 0; p < k; ++p) {
                    double pp = absf ? fabs(phiv[q * k + p]) : phiv[q * k + p];
                    for (int j = 0; j < k; ++j) {
                        double pj = absf ? fabs(phiv[q * k + j]) : phiv[q * k + j];
                        Ae[p * k + j] += s * pj * pp;
                    }
                }
            }
            for (int p = 0; p < k; ++p)
                for (int j = 0; j < k; ++j) {
                    rows[t] = dv[p];
                    cols[t] = dv[j];
                    vals[t] = Ae[p * k + j];
                    ++t;
                }
            for (int p = 0; p < 6; ++p) dx[p] += offx[p];
            for (int p = 0; p < k; ++p) dv[p] += offv[p];
        }
    }
    free(dv);
    free(Ae);
}

/*
 * Algorithm 3 over the horizontal facets (d2 = 0): lambda + 1 facets per
 * column, level l = 0 .. lambda, with the loop bound lambda - d2 inclusive.
 * Facet l lies between the prism of layer l - 1 (below; absent for l = 0)
 * and that of layer l (above; absent for l = lambda).  Its stencil is the
 * lists of both prisms, advanced by the offsets as in the cell loop.
 *
 * Form (the interior-penalty jump term of a field discontinuous across
 * levels, with zero outside the domain on the bottom and top facets):
 *     out_i += integral over the facet of [x] [v_i] dS,  [w] = w_below - w_above.
 * The facet integral uses the coordinate field's restriction to the level
 * (the vertices of the facet at their own heights, so a tilted facet has its
 * true area): dS = |t_xi x t_eta| w_q, t the tangents of the map.
 *   qw[nq]: triangle rule; psix[q*3 + a], dpsix[(q*3 + a)*2 + r]: the
 *   barycentric functions and their derivatives; phi_lo[q*k + p] /
 *   phi_hi[q*k + p]: the basis of V at zeta = 1 (below) / zeta = 0 (above).
 * absf: the same sum with every factor replaced by its absolute value.
 * cells: the base cells to visit (NULL: all 0 .. n_iter - 1).
 * out0 is incremented (the caller zeroes it for WRITE).
 */
void oracle_facet_loop(int64_t n_iter, const int64_t* cells, int32_t lam, const int64_t* mapx, const int32_t* offx,
                       const double* X, int32_t k, const int64_t* mapv, const int32_t* offv, const double* in0,
                       double* out0, int32_t absf, int32_t nq, const double* qw, const double* psix,
                       const double* dpsix, const double* phi_lo, const double* phi_hi)
{
    int64_t* dv = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    for (int64_t it = 0; it < n_iter; ++it) {
        const int64_t c = cells ? cells[it] : it;
        for (int p = 0; p < k; ++p) dv[p] = mapv[c * k + p];   /* layer 0 */
        for (int32_t l = 0; l <= lam; ++l) {
            const int below = l >= 1, above = l < lam;
            /* coordinate DoFs of the facet's three vertices at level l */
            int64_t fx[3];
            for (int a = 0; a < 3; ++a)
                fx[a] = above ? mapx[c * 6 + 2 * a] + (int64_t)l * offx[2 * a]
                              : mapx[c * 6 + 2 * a + 1] + (int64_t)(l - 1) * offx[2 * a + 1];
            for (int q = 0; q < nq; ++q) {
                double t[2][3] = {{0, 0, 0}, {0, 0, 0}};
                for (int a = 0; a < 3; ++a)
                    for (int r = 0; r < 2; ++r)
                        for (int i = 0; i < 3; ++i) t[r][i] += X[fx[a] * 3 + i] * dpsix[(q * 3 + a) * 2 + r];
                const double n0 = t[0][1] * t[1][2] - t[0][2] * t[1][1];
                const double n1 = t[0][2] * t[1][0] - t[0][0] * t[1][2];
                const double n2 = t[0][0] * t[1][1] - t[0][1] * t[1][0];
                const double dS = qw[q] * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
                double ulo = 0.0, uhi = 0.0;
                for (int p = 0; p < k; ++p) {
                    const double plo = absf ? fabs(phi_lo[q * k + p]) : phi_lo[q * k + p];
                    const double phi = absf ? fabs(phi_hi[q * k + p]) : phi_hi[q * k + p];
                    if (below) {
                        const double x = in0[dv[p] - offv[p]];   /* the prism below: one offset down */
                        ulo += (absf ? fabs(x) : x) * plo;
                    }
                    if (above) {
                        const double x = in0[dv[p]];
                        uhi += (absf ? fabs(x) : x) * phi;
                    }
                }
                const double jump = absf ? ulo + uhi : ulo - uhi;
                for (int p = 0; p < k; ++p) {
                    const double plo = absf ? fabs(phi_lo[q * k + p]) : phi_lo[q * k + p];
                    const double phi = absf ? fabs(phi_hi[q * k + p]) : phi_hi[q * k + p];
                    if (below) out0[dv[p] - offv[p]] += dS * jump * plo;
                    if (above) out0[dv[p]] += (absf ? 1.0 : -1.0) * dS * jump * phi;
                }
            }
            /* the prism above facet l is the prism below facet l + 1 */
            if (above)
                for (int p = 0; p < k; ++p) dv[p] += offv[p];
        }
    }
    free(dv);
}

/*
 * Algorithm 1 with a DoF count per entity: the paper fixes the count per
 * entity type for its exposition and notes that the algorithm does not need
 * it (Section 5).  Base entity (d1, i) carries dofs_d1[2i] DoFs on each of
 * its horizontal entities and dofs_d1[2i + 1] on each vertical one; the
 * counter visits the entities exactly as oracle_alg1_number does.  first_d
 * as there (an entity without DoFs still records the counter).
 */
int64_t oracle_alg1_number_mixed(const int32_t counts[3], int32_t lam, const int32_t* dofs0, const int32_t* dofs1,
                                 const int32_t* dofs2, int64_t* first0, int64_t* first1, int64_t* first2)
{
    int64_t* first[3] = {first0, first1, first2};
    const int32_t* dofs[3] = {dofs0, dofs1, dofs2};
    int64_t c = 0;
    for (int d1 = 0; d1 < 3; ++d1) {
        for (int64_t i = 0; i < counts[d1]; ++i) {
            int64_t* f = first[d1] + i * (int64_t)(lam + 1) * 2;
            const int32_t nh = dofs[d1][2 * i], nv = dofs[d1][2 * i + 1];
            for (int32_t l = 0; l < lam; ++l) {
                f[l * 2 + 0] = c;
                c += nh;
                f[l * 2 + 1] = c;
                c += nv;
            }
            f[lam * 2 + 0] = c;
            c += nh;
            f[lam * 2 + 1] = -1;
        }
    }
    return c;
}

/*
 * Explicit lists of a space with a DoF count per entity: the list of cell c
 * has its own length (list_off[c] .. list_off[c + 1]); entries in the order
 * of oracle_stencil (closure entities vertex 0, 1, 2, edge 0, 1, 2, cell; per
 * entity its bottom, top and vertical DoFs), for the bottom layer; the
 * vertical offset of every entry is the entity's DoFs per level (Algorithm 2
 * per entity).  With lmap NULL only list_off is filled.  Returns the total
 * length.
 */
int64_t oracle_stencil_mixed(int64_t n_cells, int32_t lam, const int32_t* dofs0, const int32_t* dofs1,
                             const int32_t* dofs2, const int32_t* cell_vertex, const int32_t* cell_edge,
                             const int64_t* first0, const int64_t* first1, const int64_t* first2,
                             int64_t* list_off, int64_t* lmap, int32_t* offsets)
{
    const int64_t* first[3] = {first0, first1, first2};
    const int32_t* dofs[3] = {dofs0, dofs1, dofs2};
    int64_t p = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
        list_off[c] = p;
        for (int e = 0; e < 7; ++e) {
            const int d = e < 3 ? 0 : (e < 6 ? 1 : 2);
            int64_t i;
            if (d == 0) i = cell_vertex[c * 3 + e];
            else if (d == 1) i = cell_edge ? cell_edge[c * 3 + (e - 3)] : -1;
            else i = c;
            if (i < 0) continue;
            const int32_t nh = dofs[d][2 * i], nv = dofs[d][2 * i + 1];
            if (!lmap) {
                p += 2 * nh + nv;
                continue;
            }
            const int64_t* f = first[d] + i * (int64_t)(lam + 1) * 2;
            for (int j = 0; j < nh; ++j) { lmap[p] = f[0] + j; offsets[p++] = nh + nv; }       /* bottom, level 0 */
            for (int j = 0; j < nh; ++j) { lmap[p] = f[2] + j; offsets[p++] = nh + nv; }       /* top, level 1 */
            for (int j = 0; j < nv; ++j) { lmap[p] = f[1] + j; offsets[p++] = nh + nv; }       /* vertical, interval 0 */
        }
    }
    list_off[n_cells] = p;
    return p;
}

/*
 * Greedy colouring of the base cells, used only to time the oracle on several
 * host threads (it is not a step of the method): cells in base order take the
 * smallest colour that no earlier cell sharing a vertex with them holds.  The
 * cells of one colour then share no vertex (hence no edge), so no DoF column
 * of a vertex or edge, and their increments cannot collide.  Writes colour[c]
 * and returns the number of colours (-1 if memory runs out).
 */
int32_t oracle_greedy_colour(int32_t n_cells, int32_t n_vertices, const int32_t* cell_vertex, int32_t* colour)
{
    int64_t* start = (int64_t*)calloc((size_t)n_vertices + 1, sizeof(int64_t));
    int32_t* around = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_cells * 3 + 1);
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_vertices + 1));
    int32_t* taken = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n_cells * 3 + 1));
    if (!start || !around || !fill || !taken) {
        free(start); free(around); free(fill); free(taken);
        return -1;
    }
    for (int64_t i = 0; i < (int64_t)n_cells * 3; ++i) start[cell_vertex[i] + 1]++;
    for (int32_t v = 0; v < n_vertices; ++v) start[v + 1] += start[v];
    for (int32_t v = 0; v <= n_vertices; ++v) fill[v] = start[v];
    for (int32_t c = 0; c < n_cells; ++c)
        for (int a = 0; a < 3; ++a) around[fill[cell_vertex[c * 3 + a]]++] = c;
    /* taken[k] == c marks colour k as held by a neighbour of cell c */
    for (int64_t k = 0; k < (int64_t)n_cells * 3 + 1; ++k) taken[k] = -1;
    int32_t n_colours = 0;
    for (int32_t c = 0; c < n_cells; ++c) colour[c] = -1;
    for (int32_t c = 0; c < n_cells; ++c) {
        for (int a = 0; a < 3; ++a) {
            const int32_t v = cell_vertex[c * 3 + a];
            for (int64_t j = start[v]; j < start[v + 1]; ++j) {
                const int32_t o = colour[around[j]];
                if (o >= 0) taken[o] = c;
            }
        }
        int32_t k = 0;
        while (taken[k] == c) ++k;
        colour[c] = k;
        if (k + 1 > n_colours) n_colours = k + 1;
    }
    free(start); free(around); free(fill); free(taken);
    return n_colours;
}
