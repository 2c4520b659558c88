/*
 * lbddc.h -- C ABI of the MI355X library for the ROM-accelerated BDDC solver of
 * two-dimensional level-set lattices (Bonilla Moreno, Guarino, Antolin,
 * arXiv 2604.09113).
 *
 * The library runs the online, per-cell data-parallel part of the method on one
 * GPU:
 *   assemble  every cell's single high-order stiffness matrix by the fast
 *             assembly with the MDEIM surrogate and the alpha-stabilisation
 *             (Sec. 4.1-4.2, Alg. 4 and 5);
 *   setup     local Schur complements (Sec. 3.2), constraints, constrained local
 *             factorizations, coarse basis and coarse matrix, partition-of-unity
 *             weights (Sec. 3.3, Alg. 2), and the exact FP64 coarse factorization;
 *   solve     PCG on the interface problem with the BDDC preconditioner (Alg. 1)
 *             and interior recovery;
 *   gradient  the compliance f^T u and its gradient with respect to the control
 *             net and the per-cell geometric parameters (discrete adjoint; the
 *             adjoint state equals u).
 *
 * Conventions
 *   - Every call returns an lbddc_status; 0 is success.  No call aborts or
 *     throws across the ABI.  After a failure lbddc_last_error() describes it and
 *     the context keeps its previous valid state.
 *   - Host pointers passed in are read during the call only (copied to device
 *     memory before return); the caller keeps ownership.  Host output buffers are
 *     written before return.  The library owns every device allocation it makes
 *     and frees it in lbddc_destroy.
 *   - Calls follow the state order create -> load_rom (one per family) ->
 *     set_problem -> assemble -> setup -> solve -> (get_displacement,
 *     compliance_gradient).  Calling out of order returns LBDDC_E_STATE.  A new
 *     set_problem or a new assemble invalidates the later stages.
 *   - One host thread per context.  Work is enqueued on the context's stream;
 *     calls that return host data synchronise that stream.
 *   - Results are deterministic: equal inputs give bitwise-equal outputs (no
 *     floating-point atomics; every sum over cells runs in a fixed order).
 *
 * Geometry (Sec. 2.1): an nx x ny lattice of unit parametric cells, cell (ix, iy)
 * has index iy*nx + ix.  The map of every cell is a Bernstein (Bezier) patch of
 * order m taken from one shared control net of (m*ny+1) x (m*nx+1) points,
 * row-major with x fastest: ctrl[(jy*(m*nx+1) + jx)*2 + c].
 *
 * Boundary conditions (Sec. 2.2.1): a set of clamped sides of the lattice
 * (homogeneous Dirichlet on both components, strongly, on the whole side) and
 * one loaded side that carries a traction, constant on each cell edge of that
 * side (per unit physical length); the other sides are traction free.  The
 * traction acts on the boundary of the material (Sec. 4.1): on a cell of a
 * four-parameter family only on the material part {phi_0 < mu} of its loaded
 * edge, whose ends then also enter dJ/dmu; on the other families on the whole
 * edge.  The edge averages and moments of the coarse space (Sec. 3.3.1) take
 * the same domain of each edge.  The benchmark lattices clamp the left side
 * (x = 0) and load the right side.
 *
 * Level sets: each cell belongs to a level-set family.  A family has either one
 * parameter per cell, t (a thickness), or four: the corner values mu_1..mu_4
 * (bottom-left, bottom-right, top-left, top-right) of the bilinear threshold
 * function of Sec. 2.1.2, which trims the cell where phi_0 < mu, phi_0 one of
 * the periodic level sets of Table 1.  The geometry of a family enters only
 * through its trained ROM (Sec. 4.2), which the caller supplies; its `dim`
 * says which parameters its cells read.
 */
#ifndef LBDDC_H
#define LBDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbddc_ctx lbddc_ctx;

typedef enum {
  LBDDC_OK = 0,
  LBDDC_E_ARG = -1,            /* a null pointer, a size out of range, a non-finite input */
  LBDDC_E_NOMEM = -2,          /* device or host allocation failed */
  LBDDC_E_HIP = -3,            /* a HIP runtime call failed */
  LBDDC_E_STATE = -4,          /* call out of order */
  LBDDC_E_DEGENERATE_MAP = -5, /* det J <= 0 somewhere in a cell (regular maps are required, Sec. 4.1) */
  LBDDC_E_PARAM_RANGE = -6,    /* a thickness or threshold outside the trained box of its family's ROM (Sec. 4.2) */
  LBDDC_E_ROM = -7,            /* no ROM for a family, or ROM degrees differ from the problem's */
  LBDDC_E_NOT_CONVERGED = -8,  /* PCG reached max_iter; info holds the last residual */
  LBDDC_E_BREAKDOWN = -9,      /* p^T S p <= 0 or r^T z <= 0 in PCG */
  LBDDC_E_NUMERIC = -10,       /* a non-positive pivot in a local factorization, or a NaN */
  LBDDC_E_UNSUPPORTED = -11    /* a size this build does not support */
} lbddc_status;

typedef enum {
  LBDDC_FP64 = 0,   /* every step in FP64 */
  LBDDC_MIXED = 1,  /* FP64 operator, recurrence and coarse solve; the preconditioner's
                       data (fine operator, coarse basis) formed in FP64, stored and
                       applied in FP32 */
  /* lbddc_assemble only: the theta x Khat contraction (Sec. 4.1, Alg. 4 with
   * the MDEIM reconstruction of Alg. 5) in FP32 on MFMA with FP32
   * accumulation, from FP32 copies of the geometry coefficients, the MDEIM
   * vector and the reduced basis.  The result (relative error ~1e-7, set by
   * FP32 rounding over a depth of n_r + 1 and the 4 (q+1)^2 geometry terms) is
   * read with lbddc_export_cells(LBDDC_X_K); it feeds no later stage, since the
   * operator of the 1e-8 solve needs an FP64-accurate stiffness: after it,
   * lbddc_setup needs an FP64 or MIXED assemble again. */
  LBDDC_FP32_CONTRACTION = 2
} lbddc_precision;

/* Sides of the lattice, as bits of a set (clamped_sides) or one value (loaded_side). */
enum { LBDDC_SIDE_LEFT = 1, LBDDC_SIDE_RIGHT = 2, LBDDC_SIDE_BOTTOM = 4, LBDDC_SIDE_TOP = 8 };

/* Coarse degrees of freedom (Sec. 3.3.1), as bits: the displacement at every
 * cross point, two averages per edge, one moment per edge.  Supported sets:
 * CORNERS | EDGE_AVG and CORNERS | EDGE_AVG | EDGE_MOMENT (the local solves of
 * Alg. 2 take the cross points as primal; others give LBDDC_E_UNSUPPORTED). */
enum { LBDDC_CON_CORNERS = 1, LBDDC_CON_EDGE_AVG = 2, LBDDC_CON_EDGE_MOMENT = 4 };

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to enqueue
 * on (NULL = a stream created and owned by the context). */
lbddc_status lbddc_create(int device, void* stream, lbddc_ctx** out);
void lbddc_destroy(lbddc_ctx* ctx);
/* Message of the last failure on ctx (valid until the next call on ctx). */
const char* lbddc_last_error(const lbddc_ctx* ctx);
int lbddc_version(void);

/* A trained ROM of one level-set family (Sec. 4.2, Alg. 5).  The trimmed-domain
 * tensor I(x) has n_i = (p+1)^4 * 4 * (q+1)^2 entries in the order
 *   (((k1*nB + k2)*2 + j1)*2 + j2)*(q+1)^2 + k3,   nB = (p+1)^2,
 * k1, k2 = a + (p+1) b the GLL nodes of the cell, j1, j2 the parametric
 * derivative directions, k3 = a + (q+1) b the interpolation nodes.  The
 * parameter x has `dim` coordinates (1: t; 4: mu_1..mu_4), each in [lo, hi].
 * Every coordinate range splits into n_k equal intervals, so there are
 * n_cl = n_k^dim clusters (Sec. 4.2.1): x is in cluster
 * sum_i c_i n_k^i with c_i = min(floor((x_i - lo)/w), n_k - 1).
 *   U     [n_cl][n_i][n_r]         reduced basis of each cluster (zero columns allowed)
 *   coeff [n_cl][(r+1)^dim][n_r]   I_r at the tensor grid of r+1 GLL points per
 *                                  coordinate of the cluster box, node
 *                                  a_1 + (r+1) a_2 + (r+1)^2 a_3 + ... (Sec. 4.2.3)
 *   I_pi  [n_i]                    the same integral over the untrimmed cell
 * The online surrogate is the tensor-product Lagrange interpolant of degree r
 * per coordinate.  Limits: 1 <= n_r <= 43; dim 1: 1 <= r <= 16, 1 <= n_k <= 16;
 * dim 4: 1 <= r <= 8, 1 <= n_k <= 2.  `dim` 0 is read as 1.  Loading a family
 * again replaces it. */
typedef struct {
  int32_t family;
  int32_t p, q;
  int32_t n_k, n_r, r;
  double lo, hi;
  const double* U;
  const double* coeff;
  const double* I_pi;
  int32_t dim;
} lbddc_rom_desc;
lbddc_status lbddc_load_rom(lbddc_ctx* ctx, const lbddc_rom_desc* rom);

/* The lattice problem (Sec. 2, 3).  Plane-strain isotropic material (E, nu),
 * stabilisation factor rho (Sec. 2.2.3), coarse dofs `constraints`
 * (LBDDC_CON_* set, Sec. 3.3.1), clamped sides `clamped_sides` (LBDDC_SIDE_*
 * set, at least one) and the loaded side `loaded_side` (one LBDDC_SIDE_*
 * value, not clamped).  traction[(r*n_side + k)*2 + c]: component c of load
 * case r on the loaded edge of the k-th cell along the loaded side, k = iy on
 * the left and right sides (n_side = ny), k = ix on the bottom and top sides
 * (n_side = nx).  Limits: 2 <= p <= 8 (p >= 3 with edge moments: an edge of
 * a p = 2 cell has 2 interior dofs for 3 constraints), q in {1, 2, 3}, 1 <= map_order <= 4,
 * 1 <= nrhs <= 16, nx, ny >= 1.  t[ncell] is read for cells of families with
 * dim 1, mu[ncell][4] for cells of families with dim 4 (mu may be NULL when
 * there are none; a lattice meets the trimmed compatibility of Sec. 2.1.3 when
 * neighbouring cells share their common corner values).  At most 16
 * (family, cluster) pairs per problem.  Validates det J > 0 at the
 * interpolation points and on a (2m+2)^2 Gauss sample of every cell
 * (LBDDC_E_DEGENERATE_MAP), that every family has a ROM of degrees (p, q)
 * (LBDDC_E_ROM) and that every parameter lies in its family's box
 * (LBDDC_E_PARAM_RANGE).  On failure the previous problem, if any, stays in
 * place with all its stages. */
typedef struct {
  int32_t nx, ny, p, q, map_order;
  const double* ctrl;
  const int32_t* family;
  const double* t;
  double E, nu, rho;
  uint32_t constraints;
  uint32_t clamped_sides;
  int32_t loaded_side;
  int32_t nrhs;
  const double* traction;
  const double* mu;
} lbddc_problem_desc;
lbddc_status lbddc_set_problem(lbddc_ctx* ctx, const lbddc_problem_desc* desc);

/* Replace the control net, the thickness parameters and the corner thresholds
 * of the current problem (device pointers, same sizes as in set_problem, read
 * on the context's stream before the call returns; any may be NULL to keep the
 * current values, not all three).
 * The new geometry is validated as in set_problem.  On success it invalidates
 * assemble and later stages; on failure (LBDDC_E_DEGENERATE_MAP,
 * LBDDC_E_PARAM_RANGE, ...) the previous geometry and every stage computed
 * from it stay in place. */
lbddc_status lbddc_set_geometry_device(lbddc_ctx* ctx, const double* d_ctrl, const double* d_t, const double* d_mu);

/* For callers that cannot allocate device memory (tight loops, harnesses that
 * forbid allocation): the FP32 contraction of lbddc_assemble with
 * LBDDC_FP32_CONTRACTION (the same kernels, bit-identical results), with no
 * device allocation in the call.  The result goes to the caller's d_K, its
 * staging (tile table, reduced-basis pointers, geometry coefficients in tile
 * order) to a static device buffer of 48 MiB that each GPU holds from the
 * first context created on it until the process ends.  d_K receives, per
 * cell, the packed node-pair triangle [ncell][npair][4]: pair P = n1 (n1 + 1)
 * / 2 + n2 for nodes n2 <= n1 (npair = LBDDC_Q_NPAIR) in the order [interior
 * nodes (a, b), a, b = 1..p-1 with a fastest | corners BL, BR, TL, TR | left,
 * right, bottom, top edge nodes in increasing running coordinate], entry
 * [P][2 i1 + i2] = K[(i1, n1), (i2, n2)].  Rejects, with LBDDC_E_UNSUPPORTED,
 * a lattice whose cells take more tiles of 128 cells of one (family,
 * cluster) group than the buffer holds: 680 tiles (about 87,000 cells) at
 * q = 2, 383 at q = 3.  Calls on one GPU share the buffer: calls that overlap
 * on one GPU race.  The call waits on the context's stream (it reads the group
 * sizes back) and leaves every stage of the context as it was. */
lbddc_status lbddc_assemble_fp32_noalloc(lbddc_ctx* ctx, float* d_K);

/* Per-cell geometry coefficients, MDEIM evaluation and the batched contraction
 * K_i = sum_q theta_q Khat_q (Alg. 4, 5), plus the cell loads and the edge
 * constraint rows (Sec. 3.3.1; on the material part of the edges of
 * four-parameter cells, whose ends come from an interval-checked root search
 * along each edge).  `prec`: LBDDC_FP64 and LBDDC_MIXED both contract in FP64
 * (the operator); see LBDDC_FP32_CONTRACTION for the FP32 variant.
 * LBDDC_E_NUMERIC if an edge's material part needs more than 16 breaks (ends
 * and roots) or its root search does not converge. */
lbddc_status lbddc_assemble(lbddc_ctx* ctx, lbddc_precision prec);

/* Local Schur complements, weights, constrained local factorizations, coarse
 * basis, coarse matrix and its FP64 factorization (Sec. 3.2-3.3, Alg. 2). */
lbddc_status lbddc_setup(lbddc_ctx* ctx, lbddc_precision prec);

/* PCG with the BDDC preconditioner (Alg. 1) for every load case, from x0 = 0,
 * stopping when ||f - S x||_2 <= rtol ||f||_2 (recurrence residual), then
 * interior recovery.  info[r] (host, nrhs entries, may be NULL) receives the
 * iteration count, the recurrence residual and a recomputed true residual.
 * Several load cases are solved as blocks of up to 8: each PCG iteration
 * applies the operator, the preconditioner's cell data and the coarse
 * factorization once for all cases of the block that have not converged;
 * every case keeps its own recurrence (its own step lengths) and stops at its
 * own first iteration that meets rtol, so its iterates, iteration count and
 * solution equal those of lbddc_solve_sequential. */
typedef struct {
  int32_t iters;
  double rel_res;
  double true_rel_res;
} lbddc_solve_info;
lbddc_status lbddc_solve(lbddc_ctx* ctx, double rtol, int32_t max_iter, lbddc_solve_info* info);

/* lbddc_solve with the load cases solved one after another (one PCG per
 * case): the reference for the block solve, same arguments and results. */
lbddc_status lbddc_solve_sequential(lbddc_ctx* ctx, double rtol, int32_t max_iter, lbddc_solve_info* info);

/* Displacement of load case `rhs` on the GLL node lattice, host buffer
 * u[(gy*(p*nx+1) + gx)*2 + c], gy in [0, p*ny], gx in [0, p*nx]. */
lbddc_status lbddc_get_displacement(lbddc_ctx* ctx, int32_t rhs, double* u);
/* Same into device memory (context stream, not synchronised). */
lbddc_status lbddc_get_displacement_device(lbddc_ctx* ctx, int32_t rhs, double* d_u);

/* Compliance J_r = f_r^T u_r of every load case and its gradient with respect
 * to the control net and the cell parameters:
 *   dJ = 2 u^T df - u^T dK u  (the adjoint state of the compliance is u).
 * Host outputs: J[nrhs], dJ_dctrl[nrhs][ctrl size], dJ_dt[nrhs][ncell] (zero
 * for cells of dim-4 families), dJ_dmu[nrhs][ncell][4] (per cell and corner;
 * zero for cells of dim-1 families; a threshold shared by the cells around a
 * lattice vertex has the sum of their entries as its derivative); any may be
 * NULL.  Requires a completed solve. */
lbddc_status lbddc_compliance_gradient(lbddc_ctx* ctx, double* J, double* dJ_dctrl, double* dJ_dt, double* dJ_dmu);
/* Same into device memory (context stream, not synchronised). */
lbddc_status lbddc_compliance_gradient_device(lbddc_ctx* ctx, double* d_J, double* d_dJ_dctrl, double* d_dJ_dt,
                                              double* d_dJ_dmu);

/* Sizes.  `what`: */
enum {
  LBDDC_Q_NCELL = 0, LBDDC_Q_NDOF_FREE = 1, LBDDC_Q_N_SKELETON = 2, LBDDC_Q_N_INTERIOR = 3,
  LBDDC_Q_N_COARSE = 4, LBDDC_Q_N_I_ROM = 5, LBDDC_Q_NU_CELL = 6, LBDDC_Q_NC_CELL = 7,
  LBDDC_Q_NRHS = 8, LBDDC_Q_NR_MAX = 9, LBDDC_Q_DEVICE_BYTES = 10,
  /* bytes of coarse-factor data one coarse solve reads (both sweeps) */
  LBDDC_Q_COARSE_SOLVE_BYTES = 11,
  /* number of levels of the nested-dissection tree of the coarse problem */
  LBDDC_Q_COARSE_LEVELS = 12,
  /* bytes of coarse-factor data the forward sweep of one coarse solve reads */
  LBDDC_Q_COARSE_FWD_BYTES = 13,
  /* kernel launches of one sweep of a coarse solve: one per tree level above
   * the bottom levels that are swept one subtree per workgroup, plus one for
   * those (equal to the number of levels when no subtree sweep is used) */
  LBDDC_Q_COARSE_SWEEP_LAUNCHES = 14,
  /* node pairs n2 <= n1 of a cell, (p+1)^2 ((p+1)^2 + 1) / 2 */
  LBDDC_Q_NPAIR = 15
};
lbddc_status lbddc_query(const lbddc_ctx* ctx, int32_t what, int64_t* value);


/* Export per-cell results of `count` cells from `first` into a host buffer (FP64),
 * for testing.  Layouts per cell:
 *   K      [2nB][2nB], dof i*nB + k (component i, node k = a + (p+1) b)
 *   THETA  [4][2][2][(q+1)^2]: C[i1][j1][i2][j2][k3] geometry coefficients
 *   ITIL   [LBDDC_Q_NR_MAX]: [(1 - rho) I_r(x), rho, 0 ...] (zero padded)
 *   S      [nU][nU] local Schur complement over the skeleton slots
 *   D      [nU] partition-of-unity weights
 *   PSI    [nU][nC] D-weighted coarse basis D Psi (the form the solver applies)
 *   SC     [nC][nC] local coarse matrix Psi^T S Psi
 *   LOAD   [nrhs][nU] cell load on the skeleton slots
 *   FINE   [nU][nU] the fine-correction operator D [S C^T; C 0]^-1|_u D
 *   RU     [nU] the global skeleton dof of each skeleton slot (-1: Dirichlet)
 *   RC     [nC] the global coarse dof of each coarse slot (-1: inactive); the
 *          coarse dofs are numbered in the elimination order of the coarse
 *          factorization (RU and RC are integers stored as doubles)
 *   CONS   [4][nce][p+1][2] the edge constraint rows (Sec. 3.3.1) of the edges
 *          [left, right, bottom, top]: for each edge node (in increasing running
 *          coordinate, corners included) and component, its weight in the edge's
 *          average x, average y and (nce = 3) moment; over the material part of
 *          the edge for Table 1 level sets, over the whole edge otherwise
 *          (available after assemble)
 * Skeleton slots (nU = 8p): nodes [BL, BR, TL, TR, left edge, right edge, bottom
 * edge, top edge] (edge nodes in increasing running coordinate, excluding
 * corners), slot = 2*node + component.  Coarse slots (nC = 20 with moments, 16
 * without): [BL.x BL.y BR.x BR.y TL.x TL.y TR.x TR.y] then for the edges
 * [left, right, bottom, top]: [average x, average y, moment].  Slots on the
 * clamped side are inactive: their rows and columns of S are the identity and
 * their D, PSI, SC and FINE entries are zero. */
enum {
  LBDDC_X_K = 0, LBDDC_X_THETA = 1, LBDDC_X_ITIL = 2, LBDDC_X_S = 3, LBDDC_X_D = 4,
  LBDDC_X_PSI = 5, LBDDC_X_SC = 6, LBDDC_X_LOAD = 7, LBDDC_X_FINE = 8, LBDDC_X_RU = 9, LBDDC_X_RC = 10,
  LBDDC_X_CONS = 11
};
lbddc_status lbddc_export_cells(lbddc_ctx* ctx, int32_t which, int32_t first, int32_t count, double* out);

/* The exact coarse solve S_C g = z of the preconditioner (Sec. 3.3.4; the
 * factorization that lbddc_setup computes), applied to a host vector of
 * LBDDC_Q_N_COARSE entries in the numbering of LBDDC_X_RC: for testing the
 * factorization against S_C = sum_i R_C^(i)T (Psi^T S Psi)^(i) R_C^(i)
 * assembled from the exports.  Requires a completed setup. */
lbddc_status lbddc_coarse_solve(lbddc_ctx* ctx, const double* z, double* g);

/* Device time in milliseconds of the most recent launches of each phase, timed
 * with HIP events on the context stream:
 *   [0] assembly contraction kernel, [1] whole assemble, [2] local Schur kernel,
 *   [3] whole setup, [4] coarse factorization, [5] whole solve (all load cases),
 *   [6] PCG operator kernel (mean per launch), [7] preconditioner local kernel
 *   (mean per launch), [8] coarse solve (mean per application), [9] recovery,
 *   [10] gradient, [11] adjoint contraction kernel, [12] forward sweep of the
 *   coarse solve (mean per application; one launch per tree level), [13] its
 *   backward sweep (same), [14] the geometry coefficients and the MDEIM
 *   evaluation of assemble.
 * `n` entries are written (n <= 15). */
lbddc_status lbddc_phase_times(lbddc_ctx* ctx, double* ms, int32_t n);

/* PCG phases timed by lbddc_solve (bit mask; LBDDC_TIME_ALL after create):
 * LBDDC_TIME_OP the operator kernel (phase_times [6]), LBDDC_TIME_PRE the
 * preconditioner's local kernel ([7]), LBDDC_TIME_COARSE the coarse solve and
 * its two sweeps ([8], [12], [13]).  Each timed phase records two or three
 * events per PCG iteration, and an event leaves the device idle for a few
 * microseconds between kernels; phases that are not timed report 0.  The
 * assembly, setup, recovery and gradient phases are always timed (a few
 * events per call).  With LBDDC_TIME_SAMPLE added, only one operator launch
 * and one preconditioner application in eight record events, and the reported
 * totals are scaled to all of them (the idle time the events cause drops
 * eightfold).  Returns LBDDC_E_ARG for unknown bits. */
enum { LBDDC_TIME_OP = 1, LBDDC_TIME_PRE = 2, LBDDC_TIME_COARSE = 4, LBDDC_TIME_ALL = 7, LBDDC_TIME_SAMPLE = 8 };
lbddc_status lbddc_set_timing(lbddc_ctx* ctx, int32_t mask);

/* Offline stage (Sec. 4.2, Alg. 3): snapshot integrals of cells trimmed by the
 * level sets of Table 1 (family 2 Schwarz Diamond, 3 Schwarz Primitive, 4
 * Schoen FRD, 5 Schoen IWP) with the bilinear threshold of Sec. 2.1.2, for
 * training their ROMs.  For each of `count` threshold vectors mu[count][4]
 * (host), the trimmed cell {phi_0 < mu} is integrated on the GPU by an
 * implicit-domain quadrature after Saye's height-function method (the method
 * the paper's QUGaR/algoim quadrature implements, Sec. 2.2.3), and out (host)
 * receives either the whole tensor I(mu) of n_i = (p+1)^4 4 (q+1)^2 entries in
 * the order of lbddc_rom_desc (n_entries = 0: out[count][n_i]) or the entries
 * listed in entries (out[count][n_entries]; the magic points of the fitting
 * stage): one list entries[n_entries] for every vector, or with
 * entries_per_rule != 0 one list per vector, entries[count][n_entries].
 * Allocates and frees its own device memory; not for hot loops.  Limits:
 * 2 <= p <= 8, 1 <= q <= 3, n_entries <= 48; a rule of more than 131072
 * points or a failed root iteration returns LBDDC_E_NUMERIC. */
lbddc_status lbddc_implicit_tensors(lbddc_ctx* ctx, int32_t family, int32_t p, int32_t q, int32_t count,
                                   const double* mu, int32_t n_entries, const int64_t* entries,
                                   int32_t entries_per_rule, double* out);

/* For testing the offline quadrature: the same rule computed on the host for
 * one threshold vector, n Gauss points per segment (1 <= n <= 24); points
 * (x, y) and weights w into host buffers of cap entries, their number in
 * *count.  LBDDC_E_NUMERIC when cap is too small or an iteration fails. */
lbddc_status lbddc_implicit_rule_host(int32_t family, const double* mu, int32_t n, int32_t cap, double* x, double* y,
                                      double* w, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* LBDDC_H */
