/*
 * pmg.h -- C interface of the MI355X (gfx950) local p-multigrid vertex-patch smoother
 * library (libpmg.so).
 *
 * The library solves the homogeneous Dirichlet problem A u = b of the Q_p Laplacian
 * -div(grad u) = f on a structured mesh of the unit square or cube (paper Sec. 2,
 * eq. bilinear-form and eq. matrix) with an h-multigrid preconditioned flexible CG whose
 * smoother is the multiplicative vertex-patch smoother (Sec. 2.1, Alg. 1) with a local
 * p-multigrid patch solver (Sec. 2.2, Alg. 2 and Alg. 3).  Every operator is applied
 * matrix-free by sum factorization in hand-written HIP kernels.
 *
 * Conventions shared by all entry points
 *   - Vectors are caller-owned device pointers (float64 for PMG_FP64, float32 for
 *     PMG_FP32) of length N(l) = (p*n_l + 1)^dim on h-level l: one entry per node of the
 *     degree-p node grid, boundary nodes included, lexicographic with x fastest: node
 *     (i, j, k) has index i + m*(j + m*k), m = p*n_l + 1.
 *   - Cells are numbered cx + n*(cy + n*cz); cell-local nodes a + (p+1)*(b + (p+1)*e);
 *     the patch of interior vertex (vx, vy, vz), 1 <= v <= n-1, has index
 *     (vx-1) + (n-1)*((vy-1) + (n-1)*(vz-1)); its closure is the node box
 *     p(v-1) <= i <= p(v+1) per direction, its interior the open box; both are listed x
 *     fastest.  Patch colors are sum_k (v_k mod 2) 2^k (2^dim colors; two patches of one
 *     color never have one's interior inside the other's closure, Sec. 4.4).
 *   - h-levels are numbered 0 (coarsest) .. n_hlevels-1 (finest); p-levels 0 (degree 1)
 *     .. n_plevels-1 (degree p).
 *   - Dirichlet rows are identity rows: (A u)_i = u_i on boundary nodes and interior rows
 *     do not see boundary values.
 *   - Streams are hipStream_t passed as void*; NULL is the default stream.  Device entry
 *     points enqueue work and return without synchronizing, except pmg_solve and
 *     pmg_batch_solve.
 *   - Every function returns PMG_OK (0) or a negative status; pmg_last_error() gives a
 *     thread-local message.  Arguments are validated before anything is enqueued, so a
 *     failed call leaves its outputs untouched.  No C++ exception crosses the interface.
 *   - Handles are library-owned; a problem may be used by one stream at a time.
 *     Device buffers are allocated in pmg_device_init only; later calls allocate
 *     nothing.
 */
#ifndef PMG_H
#define PMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PMG_OK = 0,
  PMG_ERR_INVALID_ARG = -1,
  PMG_ERR_UNSUPPORTED = -2,
  PMG_ERR_OUT_OF_MEMORY = -3,
  PMG_ERR_DEVICE = -4,
  PMG_ERR_NOT_CONVERGED = -5,
  PMG_ERR_BREAKDOWN = -6,
  PMG_ERR_STATE = -7
};

/* Arithmetic of a call: vectors and computation in float64 or float32.  PMG_FP32_BF16
 * computes in float32 with float32 vectors but reads the stored operator data of the
 * general path (per-Gauss-point metric, per-patch inverse diagonals) in bfloat16; on the
 * Cartesian path there is no stored operator data and it equals PMG_FP32. */
enum { PMG_FP64 = 0, PMG_FP32 = 1, PMG_FP32_BF16 = 2 };

/* Local patch solver (Sec. 2.2): one half V-cycle (no post-smoothing, Sec. 2.2.1) or a
 * full V-cycle per Richardson step, or the exact patch solve by fast diagonalization of the
 * Cartesian patch operator (the comparison solver of Sec. 4.3, Table 3; Cartesian path
 * only). */
enum { PMG_LOCAL_HALF_V = 0, PMG_LOCAL_FULL_V = 1, PMG_LOCAL_DIRECT = 2 };

/* Richardson preconditioner of the p-levels inside the local p-multigrid (Sec. 2.2): the
 * diagonal (damped Jacobi, default damping 4 / (3 lambda_max(D^-1 A))) or the
 * Cartesian-reinforced one (fast-diagonalization inverse of the Cartesian patch operator
 * with diagonal scaling; on the Cartesian path it is the inverse of the patch operator,
 * default damping 1).  Cartesian path only. */
enum { PMG_SMOOTHER_JACOBI = 0, PMG_SMOOTHER_REINFORCED = 1 };

/* Lanes per patch of the Cartesian smoother launches: by launch size (a color with at
 * most 4 patches per compute unit runs 256 lanes per patch, larger colors the per-degree
 * count: 64 for p <= 3, 128 for p = 4, 256 or 512 above; in 3D at p = 4 and 5 an FP32 color
 * with at least 64 patches per compute unit runs half the per-degree count, 64 and 128
 * lanes, when the local solver is the default one half V-cycle), or always one of them:
 * NARROW the per-degree count, WIDE 256, HALF half the per-degree count where the degree has
 * that kernel (3D p = 4, 5 with the default local solver; elsewhere the per-degree count).
 * The arithmetic is the same; the choice only trades latency against occupancy. */
enum { PMG_LANES_AUTO = 0, PMG_LANES_NARROW = 1, PMG_LANES_WIDE = 2, PMG_LANES_HALF = 3 };

typedef struct {
  int local_solver; /* PMG_LOCAL_HALF_V (default), PMG_LOCAL_FULL_V or PMG_LOCAL_DIRECT */
  int n_local_iter; /* Richardson steps of LocalSolve (Alg. 2), >= 1; default 1          */
  int n_pre;        /* smoother applications before the coarse correction, default 1     */
  int n_post;       /* smoother applications after it (descending colors), default 1     */
  int max_iter;     /* outer flexible-CG iteration limit, default 200                    */
  double rtol;      /* outer stop: |b - A x|_2 <= rtol |b|_2, default 1e-8               */
  int n_omega;      /* 0: library damping; else the number of valid entries in omega     */
  double omega[8];  /* Jacobi damping per p-level, coarsest first (entry 0 is unused)    */
  int patch_lanes;  /* PMG_LANES_AUTO (default), _NARROW, _WIDE or _HALF                 */
  int local_smoother; /* PMG_SMOOTHER_JACOBI (default) or PMG_SMOOTHER_REINFORCED       */
} pmg_config;

typedef struct {
  int iterations;      /* outer iterations performed                                  */
  double rel_residual; /* final |b - A x|_2 / |b|_2 (recursively updated residual)    */
  double seconds;      /* wall time of the call                                       */
  int status;          /* same value as the return code                               */
} pmg_solve_info;

typedef struct pmg_mesh pmg_mesh;
typedef struct pmg_problem pmg_problem;

/* Thread-local text of the last error. */
const char *pmg_last_error(void);

/* Fills cfg with the defaults listed in pmg_config. */
void pmg_default_config(pmg_config *cfg);

/* Mesh hierarchy M_0 ... M_L of nested structured meshes (Sec. 2).
 *   dim       2 or 3.
 *   n_cells   host array of cells per direction on the finest mesh (dim entries are read),
 *             each in [2, 1024].  The kernels index square and cubic node grids, so the
 *             entries must be equal (UNSUPPORTED otherwise); n below is that count.
 *   n_hlevels number of h-levels, or 0: halve n while it is even and above 3.
 *   vertices  NULL for the uniform Cartesian unit box.  Otherwise host array of
 *             (n+1)^dim * dim doubles (vertex-major, x fastest) of a distorted mesh (Sec. 4
 *             moves interior vertices of a Cartesian grid); every cell is the multilinear
 *             image of the reference cell, coarser levels take the fine vertices at their
 *             stride (topological nesting, Sec. 2).  Such meshes use the general path:
 *             the metric w mu |det J| J^-1 J^-T is stored per Gauss point and the patch
 *             diagonals per patch.
 * The mesh owns a copy of everything it needs; *out is set on success only. */
int pmg_setup_mesh(int dim, const int32_t *n_cells, int n_hlevels, const double *vertices, pmg_mesh **out);

/* Dimension and number of h-levels (either may be NULL); if n_cells is not NULL it
 * receives the cells per direction of each level, coarsest first (host array of
 * n_hlevels entries). */
int pmg_mesh_levels(const pmg_mesh *m, int *dim, int *n_hlevels, int32_t *n_cells);

void pmg_destroy_mesh(pmg_mesh *m);

/* Degree-p discretization, patch maps and p-hierarchy on every h-level (host only).
 *   degree    1 <= p <= 8.
 *   p_levels  NULL: the paper's hierarchy (Sec. 2.2): 1, 3, 7, ... below p, then p.
 *             Else n_plevels ascending degrees starting at 1 and ending at p; supported
 *             lists are the paper's and 1, 2, ..., p for p <= 4.
 *   cfg       NULL for pmg_default_config().
 * The mesh may be destroyed afterwards. */
int pmg_setup_dofmap(const pmg_mesh *m, int degree, const int32_t *p_levels, int n_plevels,
                     const pmg_config *cfg, pmg_problem **out);

/* Sizes (every output may be NULL): dim, counts of h- and p-levels, n_cells[l] = n_l,
 * n_nodes[l] = N(l) and n_patches[l] = (n_l - 1)^dim per h-level (host arrays of
 * n_hlevels entries), degrees of the p-levels and the Jacobi damping actually used per
 * p-level (n_plevels entries). */
int pmg_problem_sizes(const pmg_problem *pr, int *dim, int *n_hlevels, int *n_plevels, int32_t *n_cells,
                      int64_t *n_nodes, int64_t *n_patches, int32_t *degrees, double *omega);

/* Index maps of h-level `hlevel` at the degree of p-level `plevel`, computed by the same
 * index arithmetic the kernels use, into caller-owned host arrays (any may be NULL):
 *   cell_dofs      n_l^dim x (q+1)^dim
 *   patch_interior (n_l-1)^dim x (2q-1)^dim
 *   patch_closure  (n_l-1)^dim x (2q+1)^dim
 *   patch_color    (n_l-1)^dim                                                   */
int pmg_export_maps(const pmg_problem *pr, int hlevel, int plevel, int32_t *cell_dofs,
                    int32_t *patch_interior, int32_t *patch_closure, uint8_t *patch_color);

/* Physical Gauss points of h-level `hlevel` at the degree of p-level `plevel`:
 * n_l^dim cells x (q+1)^dim points x dim doubles (cells and points lexicographic, x
 * fastest), into a caller-owned host array.  Used to evaluate a coefficient. */
int pmg_get_qpoints(const pmg_problem *pr, int hlevel, int plevel, double *xyz);

/* Coefficient mu of the bilinear form (Sec. 3: mu at quadrature points) on h-level
 * `hlevel`, p-level `plevel`: host array with one positive value per Gauss point in the
 * layout of pmg_get_qpoints (NULL restores mu = 1).  The library copies it.  Every level
 * is rediscretized with its own values (Sec. 2).  Must precede pmg_device_init; a problem
 * with a coefficient uses the general path. */
int pmg_set_coefficient(pmg_problem *pr, int hlevel, int plevel, const double *a_q);

/* Uploads the operator tables and allocates every device workspace on the current HIP
 * device.  Must be called once before any entry point below.  On the general path it
 * also computes the metric of every level, the per-patch inverse diagonals (on the
 * device, from element diagonals) and the dense inverse of the coarsest interior operator
 * (Cholesky on the device). */
int pmg_device_init(pmg_problem *pr);

/* v = A_l u on h-level `hlevel` (eq. matrix): matrix-free sum-factorized apply of the
 * degree-p operator; boundary rows copy u.  u and v must not overlap. */
int pmg_apply_operator(pmg_problem *pr, int hlevel, int prec, const void *u, void *v, void *stream);

/* v = M_l u on h-level `hlevel`: the consistent mass matrix of the degree-p elements (the
 * Gram matrix of the nodal basis, Sec. 2, with the exact (p+1)-point Gauss rule per
 * direction) on the Cartesian mesh, matrix-free and sum-factorized like the operator apply;
 * rows and columns of the Dirichlet boundary nodes are zero.  Used to form the right-hand
 * side b = M f of a nodal source f.  u and v: device vectors of the level's
 * (p n + 1)^dim nodes in the precision `prec`, must not overlap; launched on `stream`.
 * Returns PMG_ERR_UNSUPPORTED on the general (mapped-mesh) path. */
int pmg_mass_operator(pmg_problem *pr, int hlevel, int prec, const void *u, void *v, void *stream);

/* r = b - A_l u on h-level `hlevel` (boundary rows: b_i - u_i).  r must not overlap u, b. */
int pmg_residual(pmg_problem *pr, int hlevel, int prec, const void *b, const void *u, void *r,
                 void *stream);

/* One application of the multiplicative vertex-patch smoother (Alg. 1) on h-level
 * `hlevel`, updating u in place: colors ascending (color_dir = +1) or descending (-1),
 * every patch of a color in parallel.  For each patch: gather the closure of u, form the
 * patch residual r_j = Pi_j b - Pi_j Abar_j ubar_j, run LocalSolve (Alg. 2 with Alg. 3
 * cycles over the p-levels, damped Jacobi with precomputed inverse diagonals, exact 1x1
 * solve at degree 1) and add d_j to the patch interior of u.  Requires hlevel >= 1 and
 * n_l >= 2. */
int pmg_smooth(pmg_problem *pr, int hlevel, int prec, int color_dir, void *u, const void *b,
               void *stream);

/* LocalSolve (Alg. 2) alone for a contiguous range of patches of h-level `hlevel`:
 * r and d hold n_patches blocks of (2p-1)^dim patch-interior values (x fastest), block i
 * belonging to patch first_patch + i. */
int pmg_local_solve(pmg_problem *pr, int hlevel, int prec, int first_patch, int n_patches,
                    const void *r, void *d, void *stream);

/* Restriction by the transposed embedding (Sec. 2): coarse = R fine, fine on h-level
 * `hlevel` >= 1, coarse on hlevel-1; coarse boundary entries are set to zero. */
int pmg_restrict(pmg_problem *pr, int hlevel, int prec, const void *fine, void *coarse, void *stream);

/* fine += P coarse (embedding, Sec. 2); fine boundary entries are left unchanged. */
int pmg_prolongate_add(pmg_problem *pr, int hlevel, int prec, const void *coarse, void *fine,
                       void *stream);

/* Exact solve on the coarsest mesh: z = A_0^{-1} r (interior, computed in float64 for
 * either precision), z_i = r_i on boundary nodes.  Cartesian path: fast diagonalization;
 * general path: the stored dense inverse. */
int pmg_coarse_solve(pmg_problem *pr, int prec, const void *r, void *z, void *stream);

/* One h-multigrid V(n_pre, n_post) cycle from a zero guess on the finest level:
 * z = V(r).  r and z are float64; mg_prec selects the arithmetic of the whole cycle
 * (PMG_FP32: r is rounded to float32 on entry, z widened on exit, the coarse solve
 * stays float64). */
int pmg_vcycle(pmg_problem *pr, int mg_prec, const double *r, double *z, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pmg_vcycle with every work buffer of
 * the cycle (per-level residuals, corrections and residual products, the intermediates of
 * the transfer passes, the coarse solve's work vectors and, for FP32 multigrid, the float32
 * copies of r and z) taken from one static device array of PMG_NOALLOC_SCRATCH_BYTES per GPU
 * instead of the problem's buffers.  The call allocates nothing and computes exactly what
 * pmg_vcycle computes (the same kernels in the same order).
 *   - The problem must be device-initialized and its device current; problems whose
 *     kernels need a global-memory workgroup arena are UNSUPPORTED.
 *   - INVALID_ARG, before anything is enqueued, when the cycle needs more work memory than
 *     the array holds (e.g. 3D Q4 fits up to 32^3 cells in FP64).
 *   - Every call on a GPU uses that GPU's one array, which keeps the last call's contents
 *     (every buffer is written before it is read, so nothing is cleared): calls that may
 *     overlap on one GPU (other streams, other threads) race and must be serialized by the
 *     caller. */
#define PMG_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int pmg_vcycle_noalloc(pmg_problem *pr, int mg_prec, const double *r, double *z, void *stream);

/* Flexible CG (float64 vectors, dot products and updates) preconditioned by pmg_vcycle
 * in mg_prec, until |b - A x|_2 <= rtol |b|_2 or max_iter.  Synchronizes the stream once
 * per iteration for the convergence test.  Returns PMG_ERR_NOT_CONVERGED or
 * PMG_ERR_BREAKDOWN (a non-positive or non-finite curvature) with info filled; x then
 * holds the last iterate. */
int pmg_solve(pmg_problem *pr, int mg_prec, const double *b, double *x, int x_is_initial_guess,
              pmg_solve_info *info, void *stream);

void pmg_destroy_problem(pmg_problem *pr);

/* ---- Batches of independent problems (an extension: the paper solves one problem at
 * a time and names the barriers between colors as the main cost on coarse meshes,
 * Sec. 4.4) ----
 *
 * A batch holds up to PMG_BATCH_MAX device-initialized problems of the Cartesian 3D path
 * with the paper's p-hierarchy (Sec. 2.2), any mix of mesh sizes and degrees.  Their
 * V-cycles are aligned by depth below the finest level: each V-cycle stage (one color
 * sweep, the residual, one 1D transfer pass, the coarse solves, ...) of all problems is
 * one persistent launch per degree present (independent launches, run as parallel graph
 * branches when the stage is small), and the whole cycle, together with the vector updates of the outer
 * flexible CG, is captured once as a HIP graph.  The arithmetic of every problem equals that of pmg_vcycle and
 * pmg_solve on it (the same kernel bodies and tables); only the reduction trees of the
 * CG dot products differ.
 *
 * The batch uses the problems' own work buffers: while a batch call runs, no other call
 * may use its problems, and a problem may belong to several batches used one at a time.
 * The problems must outlive the batch.  Batch entry points are not thread-safe for one
 * batch. */
#define PMG_BATCH_MAX 16
typedef struct pmg_batch pmg_batch;

/* Builds the stage tables of both multigrid precisions (PMG_FP64 only where every
 * degree's patch arena fits in LDS: all degrees up to 8 with one Richardson step) and
 * allocates the batch state.  Launch parameters, per degree: persistent workgroups per CU
 * of the patch and apply kernels, the apply tile; plus the number of work items up to which
 * the launches of one stage run as parallel graph branches.
 * tuning_cache_path: NULL uses built-in defaults; otherwise a JSON object of
 * "arch/3d/precision/knob": value entries is read, and the first batch call in a
 * precision measures the entries it lacks on the device (seconds: whole V-cycles per
 * candidate, on the problems' work buffers) and rewrites the file with them.  Errors:
 * INVALID_ARG (n outside [1, PMG_BATCH_MAX], NULL or repeated problems, a problem
 * without pmg_device_init or on another device), UNSUPPORTED (2D, general path, or a
 * p-hierarchy other than the paper's). */
int pmg_batch_create(pmg_problem *const *problems, int n, const char *tuning_cache_path, pmg_batch **out);

/* Launches and stages of one V-cycle of the batch in mg_prec (for inspection). */
int pmg_batch_stats(const pmg_batch *bt, int mg_prec, int *n_stages, int *n_launches);

/* z[k] = V_k(r[k]) for every problem k of the batch, as pmg_vcycle (float64 vectors on
 * the finest level of problem k; mg_prec as there).  Enqueues without synchronizing. */
int pmg_batch_vcycle(pmg_batch *bt, int mg_prec, const double *const *r, double *const *z, void *stream);

/* Solves A_k x[k] = b[k] for every problem k by the flexible CG of pmg_solve from a zero
 * guess, all problems iterating together; a problem stops iterating once it meets its
 * own rtol (or breaks down, or reaches its max_iter) while the others go on.
 * infos[k] (may be NULL) receives its iterations, relative residual, status, and the
 * wall time of the whole batch solve.  Synchronizes once per iteration.  Returns PMG_OK
 * when every problem converged, else the status of the first problem that did not. */
int pmg_batch_solve(pmg_batch *bt, int mg_prec, const double *const *b, double *const *x, pmg_solve_info *infos,
                    void *stream);

void pmg_destroy_batch(pmg_batch *bt);

/* ------------------------------------------------------------------------------------
 * General hexahedral (2D: quadrilateral) meshes with stored maps.
 *
 * Sec. 3 (implementation of the patch smoother): the cells forming each vertex patch are
 * identified at setup, and a patch gathers, evaluates and scatters through its cells' DoF
 * indices.  Sec. 4.4: the patches are colored with DSATUR so that no two patches of one
 * color share a DoF whose update would race, and the smoother runs color by color.
 *
 * Vectors have one entry per node of the caller's numbering (n_dofs entries, float64 or
 * float32 device pointers).  Homogeneous Dirichlet conditions hold on the nodes of faces
 * that belong to one cell only; their rows are identity rows as on the structured box.
 * Each cell is the multilinear image of the reference cell under its corners, and the
 * operator is the same stored-metric sum factorization as the general path above.
 * A vertex patch exists at every vertex on no boundary face; it must have 2^dim cells
 * forming a 2x2(x2) block.  Patches are numbered by ascending vertex index; two patches
 * conflict when they share a cell.  DSATUR (Brelaz 1979) colors the uncolored patch with
 * the most distinct neighbour colors, ties to the most uncolored neighbours, then to the
 * lowest index, with the smallest free color.  The apply adds cell contributions color by
 * color over a DSATUR coloring of the cells (cells conflict when they share a vertex).
 * Single h-level: the smoother and the operator; no h-hierarchy is built on these meshes.
 * ------------------------------------------------------------------------------------ */
typedef struct pmg_hex pmg_hex;

/* Host-only setup from caller arrays (copied):
 *   vertices       n_vertices * dim doubles, vertex-major.
 *   cell_vertices  n_cells * 2^dim vertex indices, the cell's corners in its own
 *                  lexicographic order (x fastest).
 *   cell_dofs      n_cells * (degree+1)^dim node indices in [0, n_dofs), the cell's
 *                  Gauss-Lobatto nodes in the same local order.
 * Cells may be numbered, rotated and reflected arbitrarily: the library brings every
 * face-connected set of cells into one common frame (mirrored if needed so that
 * det J > 0) and permutes each cell's lists to it.  cfg: local_solver (half or full
 * V-cycle), n_local_iter and omega are used; NULL for the defaults.  The p-hierarchy is
 * the paper's (Sec. 2.2: 1, 3, 7, ... below the degree).  Errors: INVALID_ARG (indices out
 * of range, a face shared by more than two cells, corners that are not a hexahedron,
 * inverted or degenerate cells, a node map that differs on a shared face), UNSUPPORTED (a
 * set of cells with no common orientation, an interior vertex without 2^dim cells, the
 * direct or Cartesian-reinforced local solvers). */
int pmg_setup_hex(int dim, int degree, int64_t n_vertices, const double *vertices, int64_t n_cells,
                  const int32_t *cell_vertices, int64_t n_dofs, const int32_t *cell_dofs, const pmg_config *cfg,
                  pmg_hex **out);

/* Counts, the p-level degrees (coarsest first) and their Jacobi damping; any output may be
 * NULL. */
int pmg_hex_sizes(const pmg_hex *h, int64_t *n_patches, int *n_patch_colors, int *n_cell_colors, int *n_plevels,
                  int32_t *degrees, double *omega);

/* Copies of the stored maps (any output may be NULL): per patch its vertex, its color, its
 * 2^dim cells (block position dx + 2 dy + 4 dz) and its (2 degree + 1)^dim closure nodes
 * in the common frame (x fastest; -1 for Dirichlet nodes); per cell its color; per node 1
 * on the Dirichlet boundary. */
int pmg_hex_export(const pmg_hex *h, int32_t *patch_vertex, int32_t *patch_color, int32_t *patch_cells,
                   int32_t *patch_closure, int32_t *cell_color, uint8_t *boundary);

/* Device data on the current device: the maps, the metric of every p-level per Gauss point
 * and the per-patch inverse diagonals.  The only call that allocates device memory. */
int pmg_hex_device_init(pmg_hex *h);

/* v = A u (identity rows on Dirichlet nodes); prec PMG_FP64 or PMG_FP32. */
int pmg_hex_apply(pmg_hex *h, int prec, const void *u, void *v, void *stream);

/* r = b - A u. */
int pmg_hex_residual(pmg_hex *h, int prec, const void *b, const void *u, void *r, void *stream);

/* One application of the vertex-patch smoother (Alg. 1, LocalSolve by Alg. 2 / Alg. 3 as
 * on the structured box), colors ascending (color_dir = +1) or descending (-1), the
 * patches of one color in parallel; u is updated in place. */
int pmg_hex_smooth(pmg_hex *h, int prec, int color_dir, void *u, const void *b, void *stream);

void pmg_hex_destroy(pmg_hex *h);

#ifdef __cplusplus
}
#endif

#endif /* PMG_H */
