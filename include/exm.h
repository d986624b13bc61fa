/*
 * exm -- extruded-mesh numbering and column iteration for AMD MI355X (gfx950).
 *
 * C ABI of libexm.so.  The operations follow the statement of the method in
 * Bercea et al., "A structure-exploiting numbering algorithm for finite
 * elements on extruded meshes, and its performance evaluation in Firedrake"
 * (arXiv 1604.05937):
 *   - an extruded mesh is an unstructured 2D base mesh replicated over
 *     lambda layers of prisms (Section 3.1);
 *   - a function space attaches delta((d1, d2)) DoFs to every extruded entity
 *     of type (d1, d2) and numbers them vertical-innermost (Algorithm 1);
 *   - a stencil over the prisms is given by one explicit list per base cell
 *     plus a constant vertical offset per list position (Algorithm 2), and the
 *     iteration walks every column by direct addressing (Algorithm 3).
 *
 * Conventions shared by every entry point:
 *   - Integers are int32 unless stated; DoF numbers and map entries are int32
 *     (a space with 2^31 or more DoFs is rejected with EXM_EOVERFLOW).
 *   - "host" pointers are read during the call only; the library copies what
 *     it keeps.  "device" pointers are HIP device memory owned by the caller
 *     and must stay valid until the stream work that uses them has finished.
 *   - Field data is FP64.  A vector field of dimension dim is stored
 *     component-major: component i of DoF n at data[i * n_dofs + n], so that
 *     every component of an entity column is one contiguous run.
 *   - Every entry point validates its arguments on the host before any device
 *     work and returns a negative status with a message for exm_last_error()
 *     on failure; nothing is launched then.  Errors raised by asynchronous
 *     device work surface as EXM_EHIP from a later call or from exm_sync().
 *   - Work is enqueued on the HIP stream passed as `stream` (NULL = the
 *     default stream).  Handles are not thread-safe.
 *   - Base-mesh conventions: cell_vertex lists the three vertices of each
 *     triangle; cell_edge[c*3 + a] is the edge opposite local vertex a, i.e.
 *     the edge joining vertices (a+1)%3 and (a+2)%3.
 */
#ifndef EXM_H
#define EXM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXM_ABI_VERSION 1

/* Status codes. */
#define EXM_OK 0
#define EXM_EINVAL (-1)        /* malformed argument (null pointer, bad enum, mismatch)   */
#define EXM_ERANGE (-2)        /* an index or count outside its valid range               */
#define EXM_EOVERFLOW (-3)     /* a size that does not fit the int32 numbering            */
#define EXM_ENOMEM (-4)        /* device or host allocation failed                        */
#define EXM_EHIP (-5)          /* a HIP runtime call or an earlier launch failed          */
#define EXM_EUNSUPPORTED (-6)  /* valid request that this library does not implement      */

/* Message of the last non-OK status returned on this thread ("" if none). */
const char* exm_last_error(void);

/* EXM_ABI_VERSION of the loaded library. */
int32_t exm_abi_version(void);

/* Wait for all work on `stream` and report any asynchronous device error. */
int32_t exm_sync(void* stream);

/* ------------------------------------------------------------------------
 * Extruded mesh (Section 3.1): base mesh adjacency + number of layers.
 *
 * n_vertices, n_edges, n_cells: N_0, N_1, N_2 of the triangular base mesh.
 * cell_vertex: host [n_cells * 3]; every entry in [0, n_vertices) and the
 *              three vertices of a cell distinct (EXM_ERANGE, EXM_EINVAL
 *              otherwise).  A vertex may belong to no cell: its columns
 *              receive nothing (zeros where a loop overwrites its output).
 * cell_edge:   host [n_cells * 3] or NULL (needed only by spaces with DoFs on
 *              edges); every entry in [0, n_edges) (EXM_ERANGE); edge a of
 *              cell c joins the cell's vertices (a+1)%3 and (a+2)%3, every
 *              cell that lists an edge sees the same two vertices, and no two
 *              edges join the same pair (EXM_EINVAL otherwise).
 * n_layers:    lambda >= 1, the number of layers (prisms per column).
 * The arrays are copied to the current HIP device.  Returns the handle in
 * *out (library-owned; free with exm_mesh_destroy).
 */
typedef struct exm_mesh exm_mesh;
int32_t exm_mesh_create(int32_t n_vertices, int32_t n_edges, int32_t n_cells,
                        const int32_t* cell_vertex, const int32_t* cell_edge,
                        int32_t n_layers, exm_mesh** out);
void exm_mesh_destroy(exm_mesh* mesh);

/* Extruded mesh with a layer range per cell column.  The constant layer count
 * of the paper's exposition is a simplification the method does not need
 * (Section 3.1, footnote; Section 5).
 * layers: host [n_cells * 2]; cell c carries the prisms of layers
 *         layers[2c] .. layers[2c+1] - 1, 0 <= layers[2c] < layers[2c+1] <= n_layers.
 * The column of a vertex or edge spans the union of the ranges of the cells
 * around it (the levels lo .. hi of exm_mesh_entity_layers); Algorithm 1 then
 * numbers every entity over its own range, so column starts become a prefix
 * sum, and a cell's explicit list is the stencil of its bottom prism, so that
 * L(c) + l * offset addresses layer layers[2c] + l of its column.  Loops on
 * such a mesh run the DIRECT schedule whatever the options ask, except the
 * PIPELINED schedule when asked for on the mass of P1P1 and DG0DG0 (n_layers
 * <= 2000) and GATHER when asked for on the mass of P1P1, CG1xDG0 and CG1xDG1;
 * they refuse EXM_RACE_OWNER with the tiled schedules (EXM_EUNSUPPORTED);
 * batches take uniform meshes only.
 * Other arguments and errors as exm_mesh_create; here every vertex must
 * belong to a cell (EXM_EINVAL). */
int32_t exm_mesh_create_var(int32_t n_vertices, int32_t n_edges, int32_t n_cells,
                            const int32_t* cell_vertex, const int32_t* cell_edge,
                            int32_t n_layers, const int32_t* layers, exm_mesh** out);

/* The same meshes from device-resident adjacency: cell_vertex, cell_edge
 * (or NULL) and layers (or NULL for n_layers everywhere) are HIP device
 * arrays of the sizes above (EXM_EINVAL if any is not device memory).  They
 * are copied back to the host once, because the race-resolution plans are
 * built there, then treated exactly as by exm_mesh_create and
 * exm_mesh_create_var; the caller may free them on return.  Synchronous. */
int32_t exm_mesh_create_device(int32_t n_vertices, int32_t n_edges, int32_t n_cells,
                               const int32_t* cell_vertex, const int32_t* cell_edge,
                               int32_t n_layers, const int32_t* layers, exm_mesh** out);

/* Layer range [lo, hi) of the column of every base entity of dimension d1
 * (0 and n_layers for a uniform mesh).  lo, hi: host [N_d1], either may be
 * NULL. */
int32_t exm_mesh_entity_layers(const exm_mesh* mesh, int32_t d1, int32_t* lo, int32_t* hi);

/* ------------------------------------------------------------------------
 * Function space: the vertical-innermost numbering of Algorithm 1 and the
 * explicit lists and offsets of Algorithms 2-3.
 *
 * delta: host [6], delta[d1*2 + d2] = DoFs on each extruded entity of type
 *        (d1, d2) (d1 = 0 vertex, 1 edge, 2 cell of the base; d2 = 0
 *        horizontal, 1 vertical).  Entries >= 0 and at most 64.
 * element: the local element the space's DoFs belong to, which the element
 *        kernels of exm_par_loop need (EXM_ELEMENT_NONE = numbering only).
 *        A named element requires the delta table it implies.
 *
 * Numbering (a reading where the paper leaves the order open): base entities
 * are visited dimension-major (d1 = 0, 1, 2), then by index; within an
 * entity with several DoFs, horizontal node index major, vertical minor.
 * The explicit list L(c) of base cell c lists its closure entities in the
 * order vertex 0, 1, 2, edge 0, 1, 2, cell; for each, its delta(d,0) DoFs on
 * the bottom horizontal entity, its delta(d,0) DoFs on the top horizontal
 * entity, then its delta(d,1) DoFs on the vertical entity, all for layer 0.
 * Its length is the arity k.  Layer l uses L(c)[p] + l * offset[p] with
 * offset[p] = delta(d,0) + delta(d,1), d the entity dimension of position p.
 *
 * The numbering is built on the device (kernels on `stream`).  The space
 * keeps a reference to `mesh`, which must outlive it.
 */
#define EXM_ELEMENT_NONE 0
#define EXM_ELEMENT_P1P1 1     /* CG1 x CG1, delta(0,0) = 1, arity 6            */
#define EXM_ELEMENT_DG0DG0 2   /* DG0 x DG0, delta(2,1) = 1, arity 1            */
#define EXM_ELEMENT_DG1DG1 3   /* DG1 x DG1, delta(2,1) = 6, arity 6            */
#define EXM_ELEMENT_P2P2 4     /* CG2 x CG2, delta(0,*) = delta(1,*) = 1, arity 18 */
/* The other tensor products of {CG1, DG0, DG1} (horizontal x vertical) of
 * the paper's study (Section 4.1.3); mass action only, DIRECT schedule (and
 * GATHER for CG1 x DG0 and CG1 x DG1). */
#define EXM_ELEMENT_P1DG0 5    /* CG1 x DG0, delta(0,1) = 1, arity 3            */
#define EXM_ELEMENT_P1DG1 6    /* CG1 x DG1, delta(0,1) = 2, arity 6            */
#define EXM_ELEMENT_DG0P1 7    /* DG0 x CG1, delta(2,0) = 1, arity 2            */
#define EXM_ELEMENT_DG0DG1 8   /* DG0 x DG1, delta(2,1) = 2, arity 2            */
#define EXM_ELEMENT_DG1P1 9    /* DG1 x CG1, delta(2,0) = 3, arity 6            */
#define EXM_ELEMENT_DG1DG0 10  /* DG1 x DG0, delta(2,1) = 3, arity 3            */
/* A space with a DoF count per entity (exm_space_create_mixed) whose cells
 * each carry DG0 x DG0 (1 DoF per layer) or DG1 x DG1 (6 DoFs per layer) and
 * no other entity carries DoFs: a mixed-degree DG space, mass action only,
 * DIRECT schedule. */
#define EXM_ELEMENT_DGMIX 11

typedef struct exm_space exm_space;
int32_t exm_space_create(const exm_mesh* mesh, const int32_t* delta, int32_t element,
                         void* stream, exm_space** out);
/* n_dofs (may be NULL) and arity k (may be NULL). */
int32_t exm_space_info(const exm_space* space, int64_t* n_dofs, int32_t* arity);
/* offsets: host [k] (Algorithm 2). */
int32_t exm_space_offsets(const exm_space* space, int32_t* offsets);
/* dst: device [N_d1], first DoF of the column of every base entity of
 * dimension d1 (-1 where the space has no DoFs on that column). */
int32_t exm_space_column_starts(const exm_space* space, int32_t d1, int32_t* dst, void* stream);
/* dst: device [n_cells * k], the explicit lists L(c) of layer 0, row-major.
 * A space made by exm_space_create_mixed has lists of different lengths:
 * EXM_EUNSUPPORTED here and in exm_space_offsets; use exm_space_lists. */
int32_t exm_space_bottom_map(const exm_space* space, int32_t* dst, void* stream);
void exm_space_destroy(exm_space* space);

/* Function space with a DoF count per entity.  The paper fixes the count per
 * entity type for its exposition and notes that neither the numbering nor
 * its performance depends on it (Section 5).
 * dofs_v, dofs_e, dofs_c: host [N_d * 2]; entity i of dimension d carries
 *   dofs_d[2i] DoFs on each of its horizontal entities (levels) and
 *   dofs_d[2i + 1] on each vertical one (layers), 0 .. 64 each.  dofs_e may be
 *   NULL when no edge carries DoFs (required when the mesh has no cell_edge).
 * Algorithm 1 numbers the entities in the same order as exm_space_create, so
 * column starts are a prefix sum of the column sizes (lambda + 1) n_h +
 * lambda n_v; an entity without DoFs gets the start of the next column.  The
 * list of cell c holds, per closure entity in the order of exm_space_create,
 * its bottom, top and vertical DoFs of layer 0: its length varies by cell,
 * and the vertical offset of every entry is its entity's DoFs per level
 * (Algorithm 2 per entity).  Uniform layer count only (EXM_EUNSUPPORTED on a
 * mesh with layer ranges).  element: EXM_ELEMENT_NONE (numbering only) or
 * EXM_ELEMENT_DGMIX (checked: every cell (0, 1) or (0, 6), nothing else). */
int32_t exm_space_create_mixed(const exm_mesh* mesh, const int32_t* dofs_v, const int32_t* dofs_e,
                               const int32_t* dofs_c, int32_t element, void* stream, exm_space** out);
/* Total length of the explicit lists (n_cells * k for a uniform space). */
int32_t exm_space_list_size(const exm_space* space, int64_t* total);
/* The explicit lists of any space: list_off device [n_cells + 1] (the list of
 * cell c is lists[list_off[c] .. list_off[c + 1] - 1]), lists device [total],
 * entry_offsets device [total] (the vertical offset of every entry). */
int32_t exm_space_lists(const exm_space* space, int32_t* list_off, int32_t* lists, int32_t* entry_offsets,
                        void* stream);

/* ------------------------------------------------------------------------
 * The coordinate field (Section 4.1.1: the geometry is a vector-valued
 * P1 x P1 field, a d-vector at every extruded vertex).
 *
 * The element kernels read (x, y) once per vertex column and z at every
 * level, so they need vertical columns: the (x, y) of a base vertex is the
 * same at every level of its column (z is free: terrain-following layers are
 * allowed).  Columns that lean are refused, never integrated wrongly.
 *
 * exm_space_coordinates: fills X, device FP64 [3 * n_dofs] component-major,
 *   the coordinate field of the P1 x P1 `space`, from xyz [N_0 * (lambda + 1)
 *   * 3]: the (x, y, z) of level l of base vertex v at xyz[3 * (v * (lambda +
 *   1) + l)] (levels outside a vertex column of a mesh with layer ranges are
 *   ignored).  xyz is host memory (xyz_on_device = 0: checked on the host, then
 *   staged; the call waits for `stream`) or device memory (1: checked on the
 *   device, synchronising `stream`).  EXM_EUNSUPPORTED, with X untouched, when
 *   the x or y of a vertex changes between two levels of its column.  The
 *   address X is remembered as checked (below).
 * exm_coordinates_verify: checks an existing coordinate field X of `space`
 *   (device) for vertical columns on `stream` and waits for the answer:
 *   EXM_OK, or EXM_EUNSUPPORTED naming a leaning vertex.  The address is
 *   remembered (or forgotten) accordingly.
 * A loop, matrix assembly or batch given a coordinate address its space has
 * not seen checked runs the same check first (synchronising its stream; or
 * EXM_EINVAL while the stream is being captured).  After changing a checked
 * field in place, or reusing its memory for another, call
 * exm_coordinates_verify again.
 */
int32_t exm_space_coordinates(const exm_space* space, const double* xyz, int32_t xyz_on_device, double* X,
                              void* stream);
int32_t exm_coordinates_verify(const exm_space* space, const double* X, void* stream);

/* ------------------------------------------------------------------------
 * Parallel loop over the prisms of an extruded mesh (Algorithm 3) applying a
 * local element kernel.
 *
 * Every kernel takes as args[0] the coordinate field: a P1 x P1 space
 * (EXM_ELEMENT_P1P1) on the same mesh, dim 3, EXM_READ, with vertical columns
 * (checked once per address, as described above).
 *
 *   EXM_K_MASS       y = M x, i.e. y_i = integral of x_h v_i, the residual of
 *                    Section 4.1.1 (args: X, x READ, y).  Every element: the
 *                    paper's nine {CG1, DG0, DG1} x {CG1, DG0, DG1} spaces,
 *                    P2P2 and DGMIX.  y is EXM_INC for spaces with DoFs
 *                    shared between cells or layers (P1P1, P2P2, P1DG0,
 *                    P1DG1, DG0P1, DG1P1), EXM_WRITE or EXM_INC for the
 *                    others.  The adjoint
 *                    of this linear residual with respect to x is the same
 *                    call with the cotangent as x (M is symmetric).
 *   EXM_K_CUBIC      F_i = integral (u^3 - f) v_i  (args: X, u, f READ, F INC), P1P1.
 *   EXM_K_CUBIC_VJP  g_u,i = integral 3 u^2 w v_i, g_f,i = -integral w v_i
 *                    (args: X, u, w READ, g_u INC, g_f INC), P1P1.
 *   EXM_K_CUBIC_FUSED  F, g_u, g_f in one sweep
 *                    (args: X, u, f, w READ, F INC, g_u INC, g_f INC), P1P1.
 *
 * INC adds into the caller's buffer (zero it first for a plain assembly);
 * WRITE overwrites every DoF of the space.  All field args of one call must
 * be on one space, and no output may share a byte with another argument,
 * the coordinate field included (EXM_EINVAL).  Floating-point results may differ in
 * the last bits between race strategies (different summation order).
 */
#define EXM_READ 1
#define EXM_WRITE 2
#define EXM_INC 3

#define EXM_K_MASS 1
#define EXM_K_CUBIC 2
#define EXM_K_CUBIC_VJP 3
#define EXM_K_CUBIC_FUSED 4
/* Matrices only (exm_matrix_assemble; exm_par_loop refuses it):
 *   EXM_K_CUBIC_JAC  J_ij = dF_i / du_j = integral 3 u^2 phi_j phi_i, the
 *                    Jacobian of EXM_K_CUBIC's residual (args: X, u READ), P1P1. */
#define EXM_K_CUBIC_JAC 5
/*   EXM_K_FACET_JUMP  the loop over horizontal facets (Algorithm 3 with d2 = 0:
 *                    lambda + 1 facets per column, level 0 .. lambda):
 *                    y_i = sum over facets of integral [x][v_i] dS, [w] the
 *                    value below the facet minus the value above, zero
 *                    outside the domain (the interior-penalty jump term of a
 *                    field discontinuous across levels) (args: X, x READ, y).
 *                    Spaces discontinuous across levels: DG0DG0, DG1DG1,
 *                    DG0DG1, DG1DG0 (y WRITE or INC), P1DG0, P1DG1 (y INC);
 *                    DIRECT schedule, uniform layer count. */
#define EXM_K_FACET_JUMP 6

typedef struct {
    void* data;               /* device FP64 [n_dofs * dim]               */
    const exm_space* space;   /* space the field lives on                 */
    int32_t dim;              /* components per DoF                       */
    int32_t access;           /* EXM_READ / EXM_WRITE / EXM_INC           */
} exm_arg;

/* Race resolution for INC into continuous spaces, where base cells share
 * DoF columns horizontally. */
#define EXM_RACE_AUTO 0       /* library choice (autotuned if available)                 */
#define EXM_RACE_ATOMIC 1     /* hardware FP64 atomic adds for DoFs another unit shares  */
#define EXM_RACE_COLOUR 2     /* units greedily coloured (no shared vertex within one    */
                              /* colour), one launch per colour, plain read-add-write    */
#define EXM_RACE_OWNER 3      /* owner computes (PIPELINED schedule, P1xP1): base        */
                              /* vertices are split into tiles, each tile sums and       */
                              /* stores only the columns it owns, and a cell on a tile   */
                              /* boundary is computed by every tile owning one of its    */
                              /* vertices; no atomics and a single launch.  The GATHER   */
                              /* schedule reports this race too (each vertex column owns */
                              /* its outputs)                                            */

/* Work schedule of the column loop. */
#define EXM_SCHED_AUTO 0
#define EXM_SCHED_DIRECT 1    /* one wavefront takes cols_per_wave base cells side by side,  */
                              /* 64 / cols_per_wave consecutive layers each (one per lane),  */
                              /* gathering straight from HBM; the unit of colouring is the   */
                              /* base cell                                                  */
#define EXM_SCHED_TILED 2     /* one workgroup takes a compact tile of about tile_cells base  */
                              /* cells (grown breadth-first over cells sharing a vertex,      */
                              /* seeded in the base ordering); its                            */
                              /* wavefronts walk the tile's cells like DIRECT but sum every   */
                              /* update in LDS, and the workgroup adds each (vertex or edge,  */
                              /* level) sum to the output once; the unit of colouring is the  */
                              /* tile.  DG spaces, which share no DoFs, run DIRECT.           */
#define EXM_SCHED_STAGED 3    /* like TILED, but the workgroup also copies every column       */
                              /* segment its tile touches (coordinates and inputs) into LDS   */
                              /* once per chunk of chunk_layers layers, loading the next      */
                              /* chunk while it computes the current one; the element kernels */
                              /* read LDS only.  P1xP1, DG0DG0 and DG1DG1 (P2P2 runs TILED)   */
#define EXM_SCHED_PIPELINED 4 /* like STAGED, but the column segments (coordinates, inputs)   */
                              /* reach LDS through asynchronous global-to-LDS copies issued   */
                              /* one chunk ahead, so a chunk's loads, the previous chunk's    */
                              /* stores and the current chunk's element kernels overlap.      */
                              /* Mass action of P1xP1, P2xP2 and the six spaces               */
                              /* discontinuous horizontally (there only z goes through LDS),  */
                              /* and the cubic forms on P1xP1; other kernels fall back to     */
                              /* STAGED.  Field pointers must be 16-byte aligned.             */
#define EXM_SCHED_CHUNKED 5   /* P1xP1 mass action: one workgroup per (tile, chunk of        */
                              /* chunk_layers layers); consecutive chunks overlap by one     */
                              /* layer so that each writes whole levels, the workgroups are  */
                              /* independent and the grid runs chunk by chunk.  Same race    */
                              /* strategies and alignment as PIPELINED; other kernels run    */
                              /* PIPELINED                                                   */
#define EXM_SCHED_GATHER 6    /* mass action of P1xP1, CG1xDG0 and CG1xDG1: the loop turned  */
                              /* to the output columns                                       */
                              /* (owner computes).  A wavefront owns a base vertex and 62    */
                              /* levels of its column, walks the fan of cells around it      */
                              /* (each neighbouring column read once) and sums the rows of   */
                              /* that vertex of the prisms around each level: every output   */
                              /* DoF is written once, no atomics, colours, LDS or barriers.  */
                              /* waves_per_block 1..4; the race is reported as               */
                              /* EXM_RACE_OWNER; other kernels run DIRECT                    */

typedef struct {
    int32_t race;              /* EXM_RACE_*                                             */
    int32_t schedule;          /* EXM_SCHED_*                                            */
    int32_t cols_per_wave;     /* DIRECT, TILED: base cells side by side in one          */
                               /* wavefront, each taking 64 / cols_per_wave lanes =      */
                               /* layers per step: 1..16 (0 = choose)                    */
    int32_t waves_per_block;   /* DIRECT: 1..4; TILED: 1..8; STAGED, PIPELINED: 4 (0 = choose) */
    int32_t tile_cells;        /* TILED, STAGED, PIPELINED: 8..1024 target cells per tile */
                               /* (0 = choose)                                           */
    int32_t chunk_layers;      /* STAGED: 8, 16, 32 or 64; PIPELINED: 8, 12, 16, 20, 24  */
                               /* or 32 on P1xP1, 8, 16 or 32 on DG (and 20, 26 or 34 on */
                               /* DG0xDG0 with columns of one height: 20, 50 and 100     */
                               /* layers in one, two and three chunks); CHUNKED: 8, 16   */
                               /* or 32 per chunk (0 = choose)                           */
} exm_loop_opts;

/* opts may be NULL (all defaults). */
int32_t exm_par_loop(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args,
                     const exm_loop_opts* opts, void* stream);

/* The launch configuration exm_par_loop uses for these arguments when opts is
 * NULL or has zero fields (filled into *chosen). */
int32_t exm_par_loop_config(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args,
                            const exm_loop_opts* opts, exm_loop_opts* chosen);

/* Number of colours of the base-cell colouring used by EXM_RACE_COLOUR for
 * this space (builds it if needed). */
int32_t exm_mesh_colours(const exm_mesh* mesh, int32_t* n_colours);

/* ------------------------------------------------------------------------
 * Read-out of the race-resolution plans a loop uses (built on first use, as
 * a loop would), so that they can be checked.  The paper's CPU runs need no
 * such plan (flat MPI, one process per core); on a GPU, increments into DoF
 * columns shared between base cells race, and these plans are what resolve
 * it (the reuse between neighbouring cells is the subject of Section 4.3).
 *
 *   EXM_PLAN_CELL_COLOURS  units = base cells; the greedy colouring of
 *                          EXM_RACE_COLOUR under DIRECT (target ignored):
 *                          no two cells of one colour share a vertex.
 *   EXM_PLAN_TILES         units = tiles of about `target` base cells (TILED,
 *                          STAGED, PIPELINED, CHUNKED with EXM_RACE_ATOMIC or
 *                          EXM_RACE_COLOUR): every cell in one tile; per tile
 *                          its vertices (bit 31 set when another tile also
 *                          touches the vertex) and, when the mesh has
 *                          cell_edge, its edges likewise; tile colours with no
 *                          shared vertex within a colour.
 *   EXM_PLAN_OWNER         units = owner tiles of about target / 2 base
 *                          vertices (EXM_RACE_OWNER): the first owned[t]
 *                          vertices of tile t are its own (every vertex owned
 *                          by one tile), its cells are all cells with an
 *                          owned vertex, its other vertices are read only;
 *                          one colour.
 *
 * exm_mesh_plan_info gives the sizes; exm_mesh_plan_read copies the arrays
 * into caller-owned host memory (each pointer may be NULL to skip it):
 * colour [n_units]; cell_off, vert_off, edge_off [n_units + 1] into cells
 * [n_cell_entries], verts [n_vert_entries], edges [n_edge_entries];
 * local_cv, local_ce [n_cell_entries * 3]: the unit-local index of each
 * vertex (edge) of each listed cell; owned [n_units].  Synchronous.
 */
#define EXM_PLAN_CELL_COLOURS 1
#define EXM_PLAN_TILES 2
#define EXM_PLAN_OWNER 3

typedef struct {
    int32_t n_units;
    int32_t n_colours;
    int64_t n_cell_entries;
    int64_t n_vert_entries;
    int64_t n_edge_entries;
} exm_plan_info;

typedef struct {
    int32_t* colour;
    int32_t* cell_off;
    int32_t* cells;
    int32_t* vert_off;
    int32_t* verts;
    int32_t* owned;
    int32_t* edge_off;
    int32_t* edges;
    uint16_t* local_cv;
    uint16_t* local_ce;
} exm_plan_arrays;

int32_t exm_mesh_plan_info(const exm_mesh* mesh, int32_t kind, int32_t target, exm_plan_info* info);
int32_t exm_mesh_plan_read(const exm_mesh* mesh, int32_t kind, int32_t target, const exm_plan_arrays* out);

/* ------------------------------------------------------------------------
 * Autotuner: times the candidate launch configurations of `kernel` on these
 * arguments (outputs are written to scratch copies, the caller's buffers are
 * not modified) and records the fastest for the (kernel, element, layer
 * count, cell count) bucket in the process-wide table used when opts is NULL.
 * The choice is returned in *best (may be NULL).  Synchronises `stream`.
 */
int32_t exm_autotune(int32_t kernel, const exm_mesh* iterset, int32_t nargs, const exm_arg* args,
                     void* stream, exm_loop_opts* best);
/* Save / load the tuning table as text (one entry per line). */
int32_t exm_autotune_save(const char* path);
int32_t exm_autotune_load(const char* path);

/* ------------------------------------------------------------------------
 * Batched assembly: many extruded meshes, several fields per mesh, forward
 * residual (EXM_K_MASS) plus its adjoint, in two launches captured in a HIP
 * graph, one per kind of item: the P1 x P1 items on owner tiles and the
 * DG0 x DG0 items on tiles (the PIPELINED tile walk, one workgroup per tile
 * of any item of the kind, every field of the item through one tile
 * set-up), or, where no tiling fits or on request, persistent kernels over
 * work units of base vertices (P1) or base cells (DG0).  The fields of a
 * mesh share its lists and geometry (end of Section 3.3).
 *
 * Item m: a space (EXM_ELEMENT_P1P1 or EXM_ELEMENT_DG0DG0) and its coordinate
 * field on the same mesh; n_fields inputs f[j] with outputs b[j] = M f[j], and
 * optionally cotangents w[j] with adjoint outputs g[j] = M^T w[j] = M w[j].
 * Pointer arrays are host arrays of device pointers (copied at create).
 * Outputs are overwritten.  P1 items run on owner tiles (each vertex
 * column written once by the one tile that owns it; no atomics, so the
 * result does not depend on the order in which work runs) or on shared
 * tiles (a column only one tile touches is written by it; the columns of
 * vertices on tile boundaries are zeroed first, in the same graph, and the
 * tiles add into them with FP64 atomics, so their last bits depend on the
 * order); on vertex units each column is written by its own wavefront as in
 * EXM_SCHED_GATHER.  Tiles need 16-byte aligned coordinates (and P1
 * fields); otherwise the kind runs on work units.
 * The meshes, spaces and buffers must outlive the batch.
 */
typedef struct {
    const exm_space* space;
    const exm_space* coord_space;
    const double* coords;
    int32_t n_fields;
    const double* const* f;   /* [n_fields] */
    double* const* b;         /* [n_fields] */
    const double* const* w;   /* [n_fields] or NULL */
    double* const* g;         /* [n_fields] or NULL (NULL iff w is NULL) */
} exm_batch_item;

typedef struct exm_batch exm_batch;
/* opts may be NULL; opts->schedule = EXM_SCHED_GATHER puts both kinds on
 * work units; opts->cols_per_wave applies to DG0 work units when set;
 * opts->tile_cells sets the work-unit size (base cells of DG0 units, base
 * vertices of P1 units, scaled by 64 / layers) and makes each kind take the
 * first tiling that fits; 0 = timed choice of unit size and tilings;
 * opts->chunk_layers fixes the tiles' chunk length (8 or 16 for P1, 8, 16,
 * 32 or 34 for DG0); opts->race = EXM_RACE_OWNER or EXM_RACE_ATOMIC restricts
 * the P1 items to owner or to shared tiles (0 = timed choice of both). */
int32_t exm_batch_create(int32_t n_items, const exm_batch_item* items, const exm_loop_opts* opts,
                         void* stream, exm_batch** out);
/* Replay the captured graph on `stream`. */
int32_t exm_batch_launch(exm_batch* batch, void* stream);
/* Work units (cell or vertex groups) of the kinds that run on work units
 * (0 when both run on tiles) and persistent workgroups per work-unit kernel. */
int32_t exm_batch_info(const exm_batch* batch, int64_t* n_units, int32_t* n_blocks);
/* Tile size (target cells per tile) and chunk length of the tiles of one
 * kind of item (element EXM_ELEMENT_P1P1 or EXM_ELEMENT_DG0DG0, else
 * EXM_EINVAL); both 0 when that kind runs on work units or the batch has
 * none.  Either pointer may be NULL. */
int32_t exm_batch_tiles(const exm_batch* batch, int32_t element, int32_t* tile_cells, int32_t* chunk_layers);
void exm_batch_destroy(exm_batch* batch);

/* ------------------------------------------------------------------------
 * Matrices of bilinear forms on one space, in a layout that uses the
 * vertical alignment of the numbering (Section 5 names the sparse system
 * matrix as the next place to exploit it).
 *
 * With Algorithm 1's numbering, node alpha of the column of base entity e
 * holds the DoFs c0 + s * w, slot s = 0 .. lambda (a node on the levels) or
 * 0 .. lambda - 1 (a node inside the layers), c0 = S(e) + alpha, w the DoFs
 * per level of the column (Algorithm 2's offset).  Such a run is a class.
 * Two DoFs couple iff they share a prism, so the classes a class couples with
 * are those of the base cells around its entity (the pattern, one per class,
 * the same at every level) and the slots differ by -1, 0 or +1.  The matrix
 * is stored as, per pattern entry, band = 3 values per slot (slot distance
 * -1, 0, +1; band = 1 on spaces with no level nodes, whose couplings stay in
 * one layer), slot-innermost: no per-entry column index.  Entries at slots
 * where the two classes share no prism are zero and are not exported.
 *
 * exm_matrix_create: builds the pattern of `space` (uniform layer count only:
 *   EXM_EUNSUPPORTED on a mesh with layer ranges) on the host and allocates
 *   the values on the device (zero).  The space must outlive the matrix.
 * exm_matrix_info: n_rows (= n_dofs), nnz (structural entries, the CSR
 *   count), n_pattern (class pairs), n_stored (values held: n_pattern *
 *   band * (lambda + 1)).  NULL outputs are skipped.
 * exm_matrix_assemble(kernel, A, nargs, args, stream): overwrite the values
 *   with the matrix of
 *     EXM_K_MASS        M_ij = integral phi_j phi_i (args: X), any element;
 *     EXM_K_CUBIC_JAC   integral 3 u^2 phi_j phi_i (args: X, u on A's space), P1P1.
 *   X as for exm_par_loop.  Every value is computed by one thread from the
 *   prisms that contribute to it (no atomics): the result is bitwise
 *   reproducible.
 * exm_matrix_spmv(A, x, y, access, stream): y = A x (EXM_WRITE) or
 *   y += A x (EXM_INC); x, y device [n_rows], distinct.
 * exm_matrix_csr(A, rowptr, col, val, stream): the same matrix in CSR,
 *   device arrays rowptr [n_rows + 1] (int64), col [nnz] (int32, ascending
 *   within a row), val [nnz], caller-owned.  Allocates scratch and waits for
 *   `stream` before returning.
 */
typedef struct exm_matrix exm_matrix;
int32_t exm_matrix_create(const exm_space* space, exm_matrix** out);
int32_t exm_matrix_info(const exm_matrix* A, int64_t* n_rows, int64_t* nnz, int64_t* n_pattern, int64_t* n_stored);
int32_t exm_matrix_assemble(int32_t kernel, exm_matrix* A, int32_t nargs, const exm_arg* args, void* stream);
int32_t exm_matrix_spmv(const exm_matrix* A, const double* x, double* y, int32_t access, void* stream);
int32_t exm_matrix_csr(const exm_matrix* A, int64_t* rowptr, int32_t* col, double* val, void* stream);
void exm_matrix_destroy(exm_matrix* A);

/* exm_matrix_csr without allocating, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same rowptr, col and val as exm_matrix_csr.  The row counts
 * go straight into rowptr, which is scanned in place; the scan's segment
 * totals live in a workspace the library holds on each GPU for the life of
 * the process (512 KiB), so n_rows is limited to 65536 * 8192 = 536,870,912
 * (EXM_ERANGE beyond).  Asynchronous on `stream`; it calls no hipMalloc,
 * hipFree, memset or synchronisation.  Every call on one GPU shares that
 * workspace: calls that overlap on one GPU (other streams, other threads)
 * race and must be ordered by the caller. */
int32_t exm_matrix_csr_noalloc(const exm_matrix* A, int64_t* rowptr, int32_t* col, double* val, void* stream);

/* ------------------------------------------------------------------------
 * STREAM triad a_i = b_i + alpha c_i (FP64), the bandwidth yardstick of
 * Section 4.2.1.  block: threads per workgroup (64..1024, multiple of 64);
 * grid: workgroups (0 = one element, or one 16-byte pair, per thread).  All
 * three arrays device [n], distinct.  When all three are 16-byte aligned the
 * kernel moves 16-byte pairs with non-temporal loads and stores (on gfx950
 * about 8 % faster than one element per lane, so the yardstick is not low).
 */
int32_t exm_stream_triad(double* a, const double* b, const double* c, double alpha, int64_t n,
                         int32_t block, int32_t grid, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EXM_H */
