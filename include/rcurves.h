/*
 * rcurves.h -- C ABI of librcurves.so, the MI355X (gfx950) hot path of
 * "Repulsive Curves" (Yu, Schumacher, Crane): the discrete tangent-point
 * energy and its differential, the fractional Sobolev-Slobodeckij operator
 * A = B + B0, the constrained (projected) Sobolev gradient, the line-search
 * step with constraint projection, and a Barnes-Hut far field.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Curves are graphs G = (V, E) with vertex coordinates gamma: V -> R^3
 *   (paper Sec. 4, "Notation").  Edges are oriented pairs (i1, i2).
 * - Vertex arrays (gamma, dE, X, Y, g) are DEVICE pointers to double
 *   [n_vertices][3] (vertex-major, xyz interleaved).  The state is always
 *   float64; `rc_dtype` selects the precision in which the pair kernels
 *   evaluate the energy, the differential and the operator.
 * - The caller allocates and owns every array it passes.  The library never
 *   frees caller memory.  All workspace is allocated by rc_create and
 *   released by rc_destroy.
 * - Every call is ordered on the context's stream.  Calls whose results are
 *   scalars needed for control flow (solver iterations, line search)
 *   synchronise that stream internally; rc_energy, rc_differential and
 *   rc_sobolev_apply do not synchronise.
 * - Errors: argument and parameter errors are returned synchronously and
 *   leave outputs untouched.  Every call returns RC_OK on success.
 *   rc_last_error() gives a human-readable message for the last failure on
 *   the calling thread.  Conditions found on the device (non-finite input,
 *   a zero-length edge, coincident vertices of disjoint edges, a non-finite
 *   energy or differential) do not stop the stream: the kernel that finds
 *   one latches an RC_FLAG_* bit into the context's device status word, and
 *   the solver's own failures (no convergence, singular factorisation,
 *   projection, line search) latch theirs too; rc_sync_status() reads and
 *   clears them.
 * - One context per stream; contexts are independent and not thread-safe.
 */
#ifndef RCURVES_H
#define RCURVES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rc_ctx rc_ctx;
typedef struct rc_mlp rc_mlp;
typedef void* rc_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
  RC_OK = 0,
  RC_ERR_ARG = 1,           /* null pointer, bad size, bad index, bad enum */
  RC_ERR_PARAM_RANGE = 2,   /* alpha <= 1 or beta outside [alpha+2, 2 alpha+1) (Lemma FiniteTangentPointEnergy) */
  RC_ERR_DEGENERATE = 3,    /* zero-length edge, or coincident vertices of disjoint edges */
  RC_ERR_NONFINITE = 4,     /* a result is Inf or NaN */
  RC_ERR_NOT_CONVERGED = 5, /* iterative solve hit its iteration limit */
  RC_ERR_PROJECTION = 6,    /* constraint projection did not reach its tolerance */
  RC_ERR_LINESEARCH = 7,    /* no step length passed (projection + Armijo) */
  RC_ERR_SINGULAR = 8,      /* a factorisation broke down */
  RC_ERR_NOMEM = 9,
  RC_ERR_HIP = 10,          /* a HIP runtime call failed */
  RC_ERR_UNSUPPORTED = 11   /* topology or option the library does not handle */
} rc_status;

typedef enum { RC_F64 = 0, RC_F32 = 1 } rc_dtype;

/* Bits of the status word (rc_stats.flags after rc_sync_status).  The first
 * four are set on the device by the kernel that meets the condition; the
 * others by the calls that return the matching rc_status. */
enum {
  RC_FLAG_INPUT_NONFINITE = 1u << 0,  /* a vertex coordinate is Inf or NaN (RC_ERR_NONFINITE) */
  RC_FLAG_ZERO_EDGE = 1u << 1,        /* an edge of length 0: T_I undefined (RC_ERR_DEGENERATE) */
  RC_FLAG_PAIR_OVERFLOW = 1u << 2,    /* a pair sum of a finite, non-degenerate edge is not finite:
                                         coincident (or nearly coincident) vertices of disjoint edges,
                                         where the energy of Sec. 4.1 is infinite (RC_ERR_DEGENERATE) */
  RC_FLAG_RESULT_NONFINITE = 1u << 3, /* an energy or differential entry is Inf or NaN (RC_ERR_NONFINITE);
                                         also set by an obstacle penalty that a midpoint reaches */
  RC_FLAG_NOT_CONVERGED = 1u << 4,    /* RC_ERR_NOT_CONVERGED was returned */
  RC_FLAG_SINGULAR = 1u << 5,         /* RC_ERR_SINGULAR was returned */
  RC_FLAG_PROJECTION = 1u << 6,       /* RC_ERR_PROJECTION was returned */
  RC_FLAG_LINESEARCH = 1u << 7        /* RC_ERR_LINESEARCH was returned */
};

/* Constraint flags (paper Sec. 7.1). */
enum {
  RC_C_BARYCENTER = 1,   /* Phi = sum_I l_I (x_I - x0), 3 rows */
  RC_C_TOTAL_LENGTH = 2, /* Phi = L0 - sum_I l_I, 1 row */
  RC_C_EDGE_LENGTH = 4   /* Phi_I = l0_I - l_I, one row per edge */
};

/* Solver kinds for the projected Sobolev gradient (Sec. 4.3.1, App. B.3). */
typedef enum {
  RC_SOLVE_DENSE = 0,    /* assembled FP64 A, Cholesky of Abar + C^T C, Schur complement */
  RC_SOLVE_PCG_JACOBI = 1, /* matrix-free projected PCG, Jacobi preconditioner */
  RC_SOLVE_PCG_MG = 2,   /* matrix-free projected PCG, multigrid V-cycle preconditioner */
  RC_SOLVE_PCG_LEARNED = 4, /* the multigrid V-cycle with learned smoother weights: the MLP attached by
                              rc_learned_attach predicts a diagonal scaling per vertex that places the
                              top of the smoother's spectrum at 1, which fixes the Chebyshev interval (no
                              spectral estimate); one closed loop numbered along itself.  (The value 3
                              is not a solver kind.) */
  RC_SOLVE_MG_FMG = 5      /* the paper's standalone multigrid (App. B.3.1): full-multigrid initialisation
                              (right-hand side coarsened to the coarsest level, direct saddle solve there,
                              prolonged level by level with smoothing after each refinement), then
                              V-cycles with a projected CG smoother (cheb_degree CG steps per visit) until
                              the relative residual reaches tol; no outer Krylov method.  rc_stats
                              .iterations counts the V-cycles (the initialisation not included) */
} rc_solver;

typedef struct {
  int32_t solver;        /* rc_solver */
  double tol;            /* relative residual ||P(b - Abar x)|| / ||P b|| (FP64 true residual) */
  int32_t max_iter;      /* PCG iterations (all restarts together) */
  int32_t replace_every; /* FP64 true-residual replacement period (0 = only at convergence) */
  int32_t mg_min_vertices; /* coarsest multigrid level size (vertices per loop, total) */
  int32_t cheb_degree;   /* smoothing steps per V-cycle visit (Chebyshev degree; CG steps for RC_SOLVE_MG_FMG) */
  int32_t op_f64;        /* 1 = the PCG operator runs in FP64 even when dtype is F32 */
  int32_t lowp;          /* precision path (see rc_lowp_assemble): 0 = off; 1 = BF16, 2 = FP16
                            assembled blocks in the multigrid smoothers of the finest levels, the
                            Krylov recurrence on the operator chosen by lowp_outer, and the FP64
                            matrix-free operator for the true residuals (iterative refinement) */
  int32_t lowp_band;     /* FP32 band half-width along the chains, 0..64 */
  int32_t lowp_min_vertices; /* smoothed multigrid levels with at least this many vertices use their
                                own 16-bit block (the finest level always does when lowp != 0) */
  int32_t lowp_outer;    /* Krylov operator of the precision path: 0 = the matrix-free operator
                            (FP64 when op_f64 != 0, else the context precision), 1 = the assembled
                            FP32 block, refined by the FP64 true residuals (inner_tol) */
  double inner_tol;      /* refinement sweep: restart from the FP64 true residual once the recurrence
                            residual has dropped by this factor (0 = only at tol) */
  int32_t fallback_after; /* multilevel and learned preconditioners: when > 0, stop after the residual
                             has grown in this many consecutive iterations, or at max_iter, and solve
                             again with the multigrid preconditioner (rc_stats.fallback = 1) */
  double bct_theta;      /* > 0: the operator of the finest level and of every multigrid level with at
                            least bct_min_vertices vertices is the block-cluster-tree product of
                            rc_sobolev_apply_bct (App. B.2) with this admissibility parameter, each level
                            with its own tree built at its curve (the PCG residual and the line search's
                            projection solves use it too); needs lowp = 0.  0 = exact operators */
  int32_t bct_min_vertices;
} rc_solve_opts;

/* Options of the batch step (rc_batch_step). */
typedef struct {
  double tol;            /* relative residual of each instance's projected PCG (FP32 operator) */
  int32_t max_iter;      /* PCG iterations of the gradient solve (a fixed count in a captured step) */
  int32_t ls_rounds;     /* step lengths tried: tau0, tau0/2, ... */
  int32_t proj_iters;    /* constraint projection iterations per trial step */
  int32_t proj_max_iter; /* PCG iterations of each projection solve */
  double proj_tol;       /* relative PCG tolerance of the projection solves */
  double accept_tol;     /* a trial is accepted only if |Phi| <= accept_tol times the constraint scale */
  double c_armijo;       /* sufficient-decrease constant */
  double tau0;           /* first step length (after normalising each instance's gradient) */
  int32_t graph;         /* 1 = capture the whole step in a hipGraph on first use and replay it */
  int32_t check_every;   /* without graph: stop the PCG once every instance has converged, checked
                            every check_every iterations (0 = run max_iter) */
  int32_t coarse;        /* 1 = two-level preconditioner: loop blocks plus the coarse space of per-loop
                            translations (instances of at most 64 loops); 0 = loop blocks only */
  int32_t op_assembled;  /* 1 = the solves' operator is each instance's block of Abar assembled in FP32
                            once per step at gamma (sum of n_i^2 * 4 bytes of device memory, allocated on
                            first use), applied in difference form; 0 = the matrix-free FP32 operator */
  int32_t refine;        /* rc_batch_gradient only: 0 = one PCG solve to tol judged by its FP32 recurrence;
                            k > 0 = iterative refinement, k sweeps (at most 20), each a PCG solve to
                            inner_tol of the FP64 true residual P (dE - Abar g) (FP64 matrix-free
                            operator) added to g; the reported residual is the final FP64 true one */
  double inner_tol;      /* relative PCG tolerance of one refinement sweep */
} rc_batch_opts;

typedef struct {
  double c_armijo;       /* sufficient-decrease constant */
  double shrink;         /* step shrink factor */
  double tau0;           /* first step length (after normalising g) */
  int32_t max_backtracks;
  int32_t max_proj_iter; /* projection iterations per trial step */
  double proj_tol;       /* relative projection tolerance (times mean edge length) */
  double proj_solve_tol; /* PCG tolerance of the projection increments: C x = -Phi holds exactly
                            whatever it is; it only sets how close x is to the A-norm minimiser.
                            The first increment of a trial step is solved to this relative
                            tolerance, each later one to the same absolute accuracy but at least to
                            2 % relative (an inexact Newton iteration; PCG solvers only) */
  int32_t ccd;           /* 1 = start the search at 2/3 of the first collision time tau_max of the curve
                            moved along -g/|g| (Sec. 4.4; rc_first_collision_time), sought up to
                            1.5 tau0, so tau0 without a collision; 0 = start at tau0 */
  double bh_theta;       /* > 0 (and < 0.5): rc_step's energy and differential and the search's trial
                            energies are the Barnes-Hut approximations of rc_bh_differential (App. B.1,
                            the edge-midpoint discretisation, leaf size 32) with this parameter, for
                            large curves; the energy0 given to rc_line_search_step must then be one
                            too.  0 = the exact all-pairs sums */
  int32_t bh_refit;      /* with bh_theta > 0: 1 = the trial energies re-fit the tree that rc_step
                            built at the step's curve (rc_bh_refit_differential) instead of building a
                            new one; 0 (default) = build at every trial.  The two approximations of a
                            trial energy differ by about as much as the Armijo margin of a step on a
                            large curve, so they can accept different lengths */
} rc_ls_opts;

typedef struct {
  double energy;         /* energy before the step */
  double energy_new;     /* energy after the step */
  double grad_norm;      /* Euclidean norm of the projected gradient */
  double residual;       /* final relative FP64 residual of the gradient solve */
  double tau;            /* accepted step length (0 if none) */
  int32_t iterations;    /* PCG iterations of the gradient solve */
  int32_t proj_solve_iterations; /* PCG iterations spent in projection solves */
  int32_t backtracks;
  int32_t proj_iters;    /* projection iterations at the accepted step */
  int32_t status;        /* rc_status of the last call */
  int32_t sweeps;        /* FP64 true-residual evaluations of the gradient solve (refinement sweeps) */
  double t_eval_ms;      /* rc_step: energy + differential phase (HIP events) */
  double t_solve_ms;     /* rc_step: constraint/multigrid setup + gradient solve */
  double t_search_ms;    /* rc_step: line search with projection */
  int32_t fallback;      /* 1 when the gradient solve fell back to the multigrid preconditioner */
  uint32_t flags;        /* rc_sync_status: the RC_FLAG_* bits latched since the last read */
  double tau_max;        /* line search with ccd = 1: the first collision time (inf if none within
                            the searched range) */
} rc_stats;

/* Waits for the context's stream, reads the RC_FLAG_* bits latched since the
 * last call (device word and solver word), clears them, and returns the status
 * they mean, in the order input non-finite (RC_ERR_NONFINITE), zero-length
 * edge or pair overflow (RC_ERR_DEGENERATE, Lemma FiniteTangentPointEnergy and
 * Sec. 4.1: the energy of coincident points of disjoint edges is infinite),
 * non-finite result (RC_ERR_NONFINITE), RC_ERR_SINGULAR, RC_ERR_NOT_CONVERGED,
 * RC_ERR_PROJECTION, RC_ERR_LINESEARCH; RC_OK when none is set.
 * out_h (host, may be NULL): status and flags are written, other fields are
 * left as they are. */
rc_status rc_sync_status(rc_ctx* ctx, rc_stats* out_h);

/* Default option values. */
void rc_default_solve_opts(rc_solve_opts* o);
void rc_default_ls_opts(rc_ls_opts* o);

/* Last error message of the calling thread ("" if none). */
const char* rc_last_error(void);

/* Create a context for a curve network with n_vertices vertices and n_edges
 * edges.  `edges_h` is a HOST array int32 [n_edges][2] of oriented edges
 * (i1, i2), 0 <= i < n_vertices, i1 != i2 (paper Sec. 4, "Notation").
 * alpha, beta: tangent-point exponents, alpha > 1, alpha + 2 <= beta < 2 alpha + 1
 * (Lemma FiniteTangentPointEnergy; eq. TangentPointKernel).
 * dtype: precision of the pair kernels.  stream: HIP stream for all work.
 * Networks with junctions (vertices of degree >= 3, Sec. 7.3) take the pair
 * kernels, the matrix-free operator, dense assembly, every constraint, the
 * dense and Jacobi-PCG solvers and the step; multigrid and the assembled
 * 16-bit operator need every vertex to have degree <= 2 (loops and open
 * paths) and give RC_ERR_UNSUPPORTED on other graphs. */
rc_status rc_create(int32_t n_vertices, int32_t n_edges, const int32_t* edges_h,
                    double alpha, double beta, rc_dtype dtype, rc_stream stream,
                    rc_ctx** out);
rc_status rc_destroy(rc_ctx* ctx);

/* Chooses how an RC_F32 context with alpha = 2 on one network of vertex
 * degree <= 2 (loops and open paths) evaluates the energy and differential:
 * enable != 0 (the default for such contexts) regroups the trapezoid sum of
 * eq. DiscreteEnergy by vertex pair (v, w): for alpha = 2,
 * sum_{I at v, J at w} l_I l_J |T_I x d|^2 = (sum_{I at v} l_I |T_I x d|^2)
 * (sum_{J at w} l_J) whenever the edges at v and at w are disjoint, so one
 * pair of vertices replaces four vertex pairs of four edge pairs; pairs of
 * vertices at most 32 steps apart along a chain are summed in FP64 in the
 * edge-pair form.  enable = 0 uses the edge-pair form everywhere.  The sums are
 * the same; the rounding differs.  Other contexts: RC_ERR_UNSUPPORTED for
 * enable != 0.  Synchronises the stream when enabling. */
rc_status rc_use_vertex_pairs(rc_ctx* ctx, int32_t enable);

/* Discrete energy (eqs. DiscreteEnergy, DiscreteKernel): the sum over ordered
 * pairs of edges sharing no vertex of l_I l_J * 1/4 sum_{i in I, j in J} k(g_i, g_j, T_I).
 * gamma: device double [nV][3].  energy: device double [1] (written). */
rc_status rc_energy(rc_ctx* ctx, const double* gamma, double* energy);

/* Energy and its exact differential dE = dE/dgamma (Sec. 4.1).
 * dE: device double [nV][3] (written).  energy may be NULL. */
rc_status rc_differential(rc_ctx* ctx, const double* gamma, double* energy, double* dE);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): energy and
 * differential as rc_differential computes them on an RC_F64 context, with no
 * context and no allocation.  Its workspace (edge geometry, pair partial sums,
 * per-edge values; about 32 MB) is one static device array that each GPU the
 * library runs on holds until the process ends.
 * gamma: device double [n_vertices][3]; edges: DEVICE int32 [n_edges][2]
 * oriented (i1, i2), every vertex of degree <= 2 (loops and open paths: then
 * dE is bitwise reproducible; a higher degree gives the same sums in an
 * unfixed rounding order); energy: device double [1] or NULL; dE: device
 * double [n_vertices][3], overwritten.  1 <= n_edges <= 16384 and
 * 2 <= n_vertices <= 1048576, else RC_ERR_ARG; (alpha, beta) as rc_create,
 * else RC_ERR_PARAM_RANGE.  An edge whose endpoints are out of range or equal
 * is not read: it makes the energy NaN.  Stream-ordered on `stream`, no
 * synchronisation.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other threads) race. */
rc_status rc_differential_noalloc(const double* gamma, int32_t n_vertices, const int32_t* edges, int32_t n_edges,
                                  double alpha, double beta, double* energy, double* dE, rc_stream stream);

/* Y = Abar X with A = B + B0 (eqs. DiscreteHighOrderPart, Sec. 4.2.3,
 * eq. VectorInnerProduct), evaluated matrix-free from gamma in the context's
 * dtype.  X, Y: device double [nV][3]; Y is overwritten. */
rc_status rc_sobolev_apply(rc_ctx* ctx, const double* gamma, const double* X, double* Y);

/* Same, with the precision chosen per call (RC_F64 or RC_F32). */
rc_status rc_sobolev_apply_prec(rc_ctx* ctx, const double* gamma, const double* X, double* Y,
                                rc_dtype prec);

/* diag(A) (the Jacobi preconditioner): device double [nV] (written). */
rc_status rc_sobolev_diag(rc_ctx* ctx, const double* gamma, double* diag);

/* Dense A = B + B0 in FP64: device double [nV][nV] row-major (written).
 * Any graph. */
rc_status rc_assemble_dense(rc_ctx* ctx, const double* gamma, double* A);

/* Choose the constraint set (bitwise OR of RC_C_*) and its targets.  With
 * edge-length constraints every edge at a junction (a vertex of degree >= 3)
 * and one edge per closed loop are rows of the projector's small dense block
 * (at most 120 such rows with the barycenter and total length, else
 * RC_ERR_UNSUPPORTED); the other edge rows form tridiagonal paths.
 * x0_h: HOST double[3] barycenter target, or NULL = the length-weighted
 * barycenter of gamma_ref.  total_len0: target total length, or a negative
 * value = that of gamma_ref.  edge_len0: DEVICE double [nE] target lengths,
 * or NULL = those of gamma_ref.  gamma_ref: device double [nV][3]. */
rc_status rc_set_constraints(rc_ctx* ctx, uint32_t mask, const double* gamma_ref,
                             const double* x0_h, double total_len0, const double* edge_len0);

/* Point constraints (Sec. 7.1): Phi_{point,i} = gamma_i - x_i, 3 rows per
 * pinned vertex i, whose Jacobian is the identity block at vertex i.
 * vertices_h: HOST int32 [npt], distinct vertex indices, none of them held
 * on a surface (rc_set_surface_constraints); targets_h: HOST
 * double [npt][3] the points x_i.  npt in [0, nV]; 0 removes them.  They
 * join the set chosen by rc_set_constraints (which keeps them) in every
 * solver, the projection and the step; the other constraints keep their
 * targets.  The iterative solvers eliminate them (the projector onto null(C)
 * with the pinned entries zero is F - F C^T (C F C^T)^-1 C F, F the free-vertex
 * mask), so they add no rows to the small dense block of the projector; an
 * edge-length row whose two ends are both pinned is then implied by the pins
 * and is given a zero multiplier.  On a coarser multigrid level the coarse
 * vertices a pinned vertex interpolates from are pinned (coarsening stops
 * before a level would be more than a quarter pinned).
 * Errors: RC_ERR_ARG (npt out of range, null pointers, a vertex out of range,
 * given twice or held on a surface, a non-finite target).  Pins that leave the remaining
 * constraints dependent (for instance every vertex pinned with the barycenter
 * constraint) give RC_ERR_SINGULAR in the solve. */
rc_status rc_set_point_constraints(rc_ctx* ctx, int32_t npt, const int32_t* vertices_h, const double* targets_h);

/* Surface constraints (Sec. 7.1): Phi_{surface,i} = f(gamma_i), one row per
 * held vertex i, with Jacobian row grad f(gamma_i)^T at vertex i; f is the
 * signed distance of
 *   RC_SURFACE_SPHERE: params_h = (c_x, c_y, c_z, r), f = |x - c| - r, r > 0;
 *   RC_SURFACE_TORUS:  params_h = (c_x, c_y, c_z, R, r), the torus about the
 *     z axis through c, f = sqrt((rho - R)^2 + (z - c_z)^2) - r with rho the
 *     distance from that axis, R > r > 0.
 * vertices_h: HOST int32 [n] distinct vertex indices, none of them pinned;
 * n in [0, nV], 0 removes the constraint.  Like the point constraints they
 * are eliminated in the iterative solvers (the projector's W_v = I - n_v n_v^T
 * at a held vertex, n_v the unit normal at gamma_v) and join every solver,
 * the projection and the step; on a coarser multigrid level a held vertex
 * that the coarsening keeps stays held.  Errors: RC_ERR_ARG (n out of
 * range, unknown kind, null pointers, non-finite or out-of-range parameters,
 * a vertex out of range, given twice or pinned). */
enum { RC_SURFACE_SPHERE = 1, RC_SURFACE_TORUS = 2 };
rc_status rc_set_surface_constraints(rc_ctx* ctx, int32_t kind, const double* params_h, int32_t n,
                                     const int32_t* vertices_h);

/* Tangent constraints (Sec. 7.1): the unit tangent T_I of each listed edge
 * is held parallel to a direction X.  The printed rows T_I - X have a rank-2
 * Jacobian (T_I stays a unit vector), so the constraint is taken as the two
 * independent rows (u . T_I, v . T_I), (u, v) the orthonormal basis of the
 * plane orthogonal to X/|X| with u = X x e_m / |X x e_m| (e_m the coordinate
 * axis of the smallest |X_m|, the first on ties) and v = X x u; they vanish
 * exactly when T_I is parallel to X, and a step from near X stays on that
 * branch.  Jacobian of b . T_I: (b - (b . T_I) T_I) / l_I at i2, its negative
 * at i1; the rows are dimensionless, so the step's projection tolerance for
 * them is proj_tol itself.  edges_h: HOST int32 [n], distinct edge indices;
 * dirs_h: HOST double [n][3], nonzero directions X.  n in [0, nE]; 0 removes
 * them.  Each adds two rows to the projector's small dense block (the fused
 * projector serves up to 8 such rows with barycenter, total length and loop
 * cuts); the coarser multigrid levels do not carry them (the V-cycle projects
 * every prolonged correction onto the finest level's constraints).  Errors:
 * RC_ERR_ARG (n out of range, null pointers, an edge out of range or given
 * twice, a zero or non-finite direction), RC_ERR_UNSUPPORTED (more than 120
 * rows in the dense block). */
rc_status rc_set_tangent_constraints(rc_ctx* ctx, int32_t n, const int32_t* edges_h, const double* dirs_h);

/* Phi(gamma) (Sec. 7.1) in the row order barycenter (3), total length (1),
 * points (3 each, in the order given), surface (1 per held vertex, in the
 * order given), tangents (2 each, in the order given), edge lengths (nE),
 * restricted to the active set.  phi: device double [k]. */
rc_status rc_constraint_values(rc_ctx* ctx, const double* gamma, double* phi);

/* Number of active constraint rows k. */
int32_t rc_constraint_count(const rc_ctx* ctx);

/* Y = P X with P = I - C^T (C C^T)^-1 C the Euclidean projector onto null(C),
 * C = dPhi(gamma) (App. B.3.3, eq. ProjectedSystem).  X may equal Y. */
rc_status rc_project(rc_ctx* ctx, const double* gamma, const double* X, double* Y);

/* Projected Sobolev gradient: solve eq. GradientSaddlePointProblem
 *   [Abar C^T; C 0] [g; lambda] = [dE; 0]
 * (dense FP64, or projected PCG on P Abar P y = P dE, App. B.3.3).
 * dE, g: device double [nV][3].  opts: host, NULL = defaults.
 * stats: host, may be NULL (iterations, residual). */
rc_status rc_sobolev_gradient(rc_ctx* ctx, const double* gamma, const double* dE, double* g,
                              const rc_solve_opts* opts, rc_stats* stats);

/* Backtracking step of Sec. 4.4 with the constraint projection of
 * Sec. 4.3.2 (eq. ConstraintSaddlePointProblem, solved through eq.
 * SaddleSolutionTransformation on the PCG paths): normalise g, start at
 * tau0, shrink until projection succeeds and the Armijo condition holds at
 * the projected curve.  gamma: device double [nV][3], updated in place on
 * success (left unchanged on RC_ERR_LINESEARCH).  energy0: energy at gamma.
 * tau_h: host, accepted step length. */
rc_status rc_line_search_step(rc_ctx* ctx, double* gamma, double energy0, const double* dE,
                              const double* g, const rc_ls_opts* ls, const rc_solve_opts* so,
                              double* tau_h, rc_stats* stats);

/* One projected Sobolev step: energy and differential, projected gradient,
 * line search.  gamma is updated in place.  stats: host, may be NULL. */
rc_status rc_step(rc_ctx* ctx, double* gamma, const rc_solve_opts* so, const rc_ls_opts* ls,
                  rc_stats* stats);

/* First collision time (Sec. 4.4, time stepping): the smallest t in (0, horizon]
 * at which two edges sharing no vertex touch when the curve moves as
 * gamma - t D (every vertex on a straight line), or +inf.  Exact per pair: the
 * four endpoints are coplanar at a root of the cubic det[p2 - p1, q1 - p1,
 * q2 - p1](t), and the segments touch there iff their distance is below 1e-9
 * times the pair's size; pairs moving inside one plane meet where an endpoint
 * reaches the other segment.  FP64.  gamma, D: device double [nV][3];
 * t: device double [1]; horizon > 0 (else RC_ERR_ARG).  No synchronisation. */
rc_status rc_first_collision_time(rc_ctx* ctx, const double* gamma, const double* D, double horizon, double* t);

/* Block cluster tree (App. B.2): builds a BVH over the tangent-points of gamma
 * (leaves of at most leaf_size <= 32 edges, the builder of rc_bh_differential)
 * and splits the block (root, root) recursively into blocks (T, S) of BVH
 * nodes; a block is a leaf when it is admissible (eq. BCTAdmissibilityTest:
 * max(r_x^T, r_x^S) < theta |c_T - c_S| and max(r_T^T, r_T^S) < theta) or
 * when both nodes are BVH leaves, otherwise its internal node(s) are split.
 * theta > 0, 1 <= leaf_size <= 32, else RC_ERR_ARG.  Synchronises (the block
 * lists are formed on the host from the node data).  The tree is kept until
 * the next build. */
rc_status rc_bct_build(rc_ctx* ctx, const double* gamma, double theta, int32_t leaf_size);

/* Counts of the last tree: stats_h (host int64[4]) = BVH nodes, admissible
 * blocks, inadmissible leaf blocks, edge pairs summed directly in them. */
rc_status rc_bct_stats(rc_ctx* ctx, int64_t* stats_h);

/* Y = A^ X: the 0th-order hierarchical product (App. B.2) with A = B + B0 in
 * its kernel-matrix form (App. B.3.4, eqs. LowOrderDecomposition /
 * LowOrderKernel, and the high-order analogue with k_{0, 2 sigma + 1} and the
 * difference operator D), the kernel matrices sampled at edge midpoints with
 * the pairs sharing a vertex left out.  Admissible blocks are the rank-1
 * blocks L_T k(p_T, p_S) L_S^T with the nodes' tangent-points (centre, mean
 * tangent) and edge-length vectors; leaf blocks are summed exactly.  FP64
 * sums, symmetric for any theta, A^ 1 = 0 exactly; as theta -> 0 it is the
 * kernel-matrix form exactly.  gamma must be the curve of the last
 * rc_bct_build (its tree is used); X, Y: device double [nV][3]. */
rc_status rc_sobolev_apply_bct(rc_ctx* ctx, const double* gamma, const double* X, double* Y);

/* Barnes-Hut energy and differential (App. B.1): a BVH over the tangent-points
 * (T_I, x_I) in R^6 built on the device, admissibility
 * r_x < theta |x_I - xbar_B| and r_T < theta (eq. BarnesHutCondition), far
 * field per eq. BVHNodeTPE, near field summed directly with the edge-midpoint
 * rule.  FP32 arithmetic.  theta in (0, 0.5): then a target's own cluster is
 * never admissible.  leaf_size in [1, 256]: most edges per leaf.
 * energy: device double [1]; dE: device double [nV][3]. */
rc_status rc_bh_differential(rc_ctx* ctx, const double* gamma, double theta, int32_t leaf_size,
                             double* energy, double* dE);

/* Barnes-Hut energy and differential on the tree of the context's last
 * rc_bh_differential (or Barnes-Hut rc_step), re-fitted to gamma instead of
 * built anew: the nodes keep their edges and only their centres, lengths,
 * mean tangents and radii are recomputed (one launch), as the paper suggests
 * for small time steps (Limitations and Conclusion); the admissibility test reads the re-fitted
 * radii, so the result is a valid Barnes-Hut sum whose clusters are looser
 * the further gamma is from the curve the tree was built for.  Same
 * arguments, outputs and theta range as rc_bh_differential; RC_ERR_ARG when
 * no tree has been built on the context. */
rc_status rc_bh_refit_differential(rc_ctx* ctx, const double* gamma, double theta, double* energy, double* dE);

/* Work of the last rc_bh_differential: cluster (far-field) interactions and
 * edge pairs visited in leaves (near field, excluded pairs included), the
 * number of BVH nodes and levels.  Synchronises the stream. */
rc_status rc_bh_last_work(rc_ctx* ctx, int64_t* far_pairs, int64_t* near_pairs, int32_t* nodes, int32_t* depth);

/* Exact edge-midpoint energy and differential (the theta -> 0 limit of
 * rc_bh_differential), in the context's dtype. */
rc_status rc_midpoint_differential(rc_ctx* ctx, const double* gamma, double* energy, double* dE);

/* Precision path: the Sobolev block A = B + B0 (Sec. 4.2.2-4.2.3, the entries of
 * the dense matrix the increments of those sections assemble) stored in 16 bits.
 * S = D^-1/2 A D^-1/2 with D = diag(A) from FP64 per-edge sums; off-diagonal
 * entries of S more than `band` steps apart along a chain are computed in FP32
 * and rounded to BF16 (fmt 1) or FP16 (fmt 2); those within the band are
 * computed in FP64 and kept in FP32; the diagonal is recomputed in FP64 as
 * minus the row sums of the stored values, so the stored operator
 * A^ = D^1/2 (S^_off + diag sigma) D^1/2 maps constants to zero.
 * With with_f32 != 0 the same pass also keeps every entry of S in FP32 (the
 * non-band ones as evaluated in FP32), with its own recomputed diagonal.
 * gamma: device double [nV][3].  fmt: 1 or 2 (else RC_ERR_ARG); band: 0..64
 * (else RC_ERR_ARG).  Needs every vertex of degree <= 2 (RC_ERR_UNSUPPORTED).
 * The context owns the blocks (about nV^2 * 2 bytes, plus nV^2 * 4 with
 * with_f32, of device memory) and replaces them on the next call; the
 * solver's precision option reassembles them at the curve being solved.
 * RC_ERR_NOMEM when they do not fit. */
rc_status rc_lowp_assemble(rc_ctx* ctx, const double* gamma, int32_t fmt, int32_t band, int32_t with_f32);

/* Y = A^ X with the last assembled block.  f32 = 0: the 16-bit block, with
 * X' = D^1/2 X scaled by a power of two and split into hi + lo 16-bit parts,
 * MFMA products with FP32 accumulation; f32 = 1: the FP32 block (FP32 MFMA).
 * Band and diagonal terms and the final D^1/2 scaling in FP64.
 * X, Y: device double [nV][3]; Y is overwritten.  RC_ERR_ARG if that block
 * has not been assembled. */
rc_status rc_lowp_apply(rc_ctx* ctx, const double* X, double* Y, int32_t f32);

/* Sphere-obstacle penalty (Sec. 7.1, surface potential with M a sphere of
 * centre c and radius R): weight * sum_I l_I Psi(|x_I - c|), with Psi the
 * closed-form integral of |x_M - y|^-(beta - alpha) over the sphere and one
 * midpoint sample per edge.  It is added to every energy and differential of
 * the context (single curves and batches).  center_h: host double[3];
 * radius > 0; weight > 0, or weight = 0 to remove it (else RC_ERR_ARG).  An
 * edge midpoint on or inside the sphere gives an infinite energy. */
rc_status rc_set_obstacle(rc_ctx* ctx, const double* center_h, double radius, double weight);

/* Penalties of Sec. 7.1, added to every energy and differential of the
 * context's all-pairs evaluations (rc_energy, rc_differential, rc_step
 * without bh_theta, and the line search): w_length sum_I l_I (total length),
 * w_diff sum over vertices of degree two of (l_I - l_J)^2 with I, J the
 * vertex's edges (length difference), and w_field sum_I l_I |T_I x X|^2 for
 * the constant unit field X = field_h / |field_h| (field potential; field_h
 * host double[3], read only when w_field > 0).  Weights finite and >= 0
 * (else RC_ERR_ARG); all zero removes them.  Not for batch contexts. */
rc_status rc_set_penalties(rc_ctx* ctx, double w_length, double w_diff, double w_field, const double* field_h);

/* Triangulated-surface potential (Sec. 7.1, surface potential): weight times
 * the double integral of |x_M - gamma|^-(beta - alpha) over the curve and the
 * surface M, sampled at the edge midpoints x_I (weight l_I) and the triangle
 * centroids c_T (weight the area A_T): weight sum_I l_I sum_T A_T
 * |c_T - x_I|^-(beta - alpha), added with its differential to every all-pairs
 * energy and differential of the context (like rc_set_penalties).  The sum
 * over triangles runs over a bounding-sphere tree of M built here on the host
 * (the surface does not move): a node whose triangles lie in a sphere of
 * radius r around their area-weighted centre c_B, with r < theta |c_B - x_I|,
 * counts as one sample of its total area at c_B; theta = 0 sums every
 * triangle.  P_h: HOST double [nP][3]; F_h: HOST int32 [nF][3] vertex indices
 * (orientation unused).  weight finite and >= 0, 0 removes the potential;
 * theta in [0, 1).  Errors: RC_ERR_ARG (weight or theta out of range, fewer
 * than 3 vertices or 1 triangle, an index out of range, a non-finite vertex).
 * Not for batch contexts; rc_step with a Barnes-Hut energy (bh_theta > 0)
 * rejects it as it rejects the penalties.  A midpoint on a centroid gives an
 * infinite energy. */
rc_status rc_set_surface_potential(rc_ctx* ctx, int32_t nP, const double* P_h, int32_t nF, const int32_t* F_h,
                                   double weight, double theta);

/* ------------------------------------------------------------------------
 * Batches: many independent curve networks ("instances", e.g. packings of
 * closed loops) in one context.  Pair sums (energy, differential, operator)
 * run over pairs of edges of the same instance only, as one persistent launch
 * over work items (target tile, source range) ordered longest first.
 * ---------------------------------------------------------------------- */

/* Creates a batch context.  inst_vertex_off_h: host int32[n_inst + 1],
 * increasing, from 0 to n_vertices: instance i owns vertices
 * [off[i], off[i+1]).  edges_h: host int32[n_edges][2], grouped by instance in
 * instance order, every edge inside one instance.  Other arguments and
 * errors as rc_create.  rc_energy / rc_differential / rc_sobolev_apply then
 * give the sums over all instances (the block-diagonal operator); the
 * single-network solver calls return RC_ERR_UNSUPPORTED on a batch. */
rc_status rc_create_batch(int32_t n_inst, const int32_t* inst_vertex_off_h, int32_t n_vertices, int32_t n_edges,
                          const int32_t* edges_h, double alpha, double beta, rc_dtype dtype, rc_stream stream,
                          rc_ctx** out);

/* Number of instances (0 for a single-network context). */
int32_t rc_batch_size(const rc_ctx* ctx);

/* Per-instance energies (device double[n_inst]) and, when dE != NULL, the
 * differential (device double[nV][3]); the obstacle is included when set. */
rc_status rc_batch_energies(rc_ctx* ctx, const double* gamma, double* energies, double* dE);

/* Work-item shape of the batch pair kernels: source ranges of src_chunk
 * edges (256 .. 2^20) and blocks_per_cu persistent workgroups per compute
 * unit (1 .. 32).  Synchronises the stream. */
rc_status rc_batch_tiling(rc_ctx* ctx, int32_t src_chunk, int32_t blocks_per_cu);

/* Chooses the work-item shape of the batch pair kernels by timing candidate
 * source-range lengths (512 .. 4096) and persistent workgroups per compute
 * unit (4, 8, 16) on one energy + differential and one operator application
 * at gamma (device double[nV][3]), and keeps the fastest.  cache_path (host
 * string or NULL): a JSON file of earlier choices keyed by GPU architecture,
 * kernel and size class; a hit skips the timing, a new result is added.
 * Outputs (host): the chosen src_chunk, blocks_per_cu and the timed ms per
 * (energy + differential + operator).  Synchronises the stream. */
rc_status rc_batch_autotune(rc_ctx* ctx, const double* gamma, const char* cache_path, int32_t* src_chunk,
                            int32_t* blocks_per_cu, double* ms);

/* Defaults of rc_batch_opts. */
void rc_default_batch_opts(rc_batch_opts* opts);

/* Constraint targets of every instance from gamma_ref (device double
 * [nV][3]): the length-weighted barycenter of the instance (Sec. 7.1,
 * barycenter) and the length of each of its loops (Sec. 7.1, total length,
 * one row per loop).  Needed before rc_batch_gradient / rc_batch_step. */
rc_status rc_batch_set_constraints(rc_ctx* ctx, const double* gamma_ref);

/* Projected Sobolev gradient of every instance (eq.
 * GradientSaddlePointProblem with that instance's constraints): PCG with the
 * FP32 operator, the loop-block preconditioner and per-instance scalars, to
 * opts->tol or opts->max_iter.  dE, g: device double[nV][3]. */
rc_status rc_batch_gradient(rc_ctx* ctx, const double* gamma, const double* dE, double* g,
                            const rc_batch_opts* opts);

/* One projected Sobolev step of every instance (Sec. 4.3-4.4): energy and
 * differential, gradient as rc_batch_gradient, then per instance: normalise,
 * try tau0, tau0/2, ... (opts->ls_rounds lengths), project each trial back
 * onto the constraints (opts->proj_iters increments of eq.
 * ConstraintSaddlePointProblem via eq. SaddleSolutionTransformation, with
 * the operator and Jacobian frozen at gamma), accept the first length that
 * satisfies Armijo and |Phi| <= opts->accept_tol.  gamma (device, in place)
 * changes only for instances that accepted.  With opts->graph = 1 the step is
 * captured once as a hipGraph (fixed trip counts, no host synchronisation)
 * and replayed; a change of gamma's address or of the options recaptures.
 * stats_h: host double[n_inst][8] or NULL: (E0, E1, tau, PCG iterations,
 * PCG residual, status 0 accepted / 1 no step / 2 singular constraints, |g|,
 * halvings); filling it synchronises. */
rc_status rc_batch_step(rc_ctx* ctx, double* gamma, const rc_batch_opts* opts, double* stats_h);

/* Y = Abar X for every instance at gamma with the FP32 operator: matrix-free
 * (assembled = 0) or from the per-instance blocks assembled at gamma
 * (assembled = 1, the operator of rc_batch_opts.op_assembled).  X, Y: device
 * double[nV][3]. */
rc_status rc_batch_sobolev_apply(rc_ctx* ctx, const double* gamma, const double* X, double* Y, int32_t assembled);

/* Iterations and relative residual of every instance in the last batch PCG
 * solve (host double[n_inst] each); synchronises. */
rc_status rc_batch_pcg_state(rc_ctx* ctx, double* iters_h, double* res_h);

/* ------------------------------------------------------------------------
 * Learned smoother weights of the multigrid V-cycle (App. B.3.1 hierarchy;
 * the learned part is not in the paper).  For a single closed loop whose
 * vertices are numbered along it, an MLP (8 -> 64 -> 64 -> 1, ReLU,
 * softplus) maps per-vertex features of every smoothed level l to
 * p_v = 1 + y_v, a prediction of T_v = r_v lambda_l with
 * r_v = sum_w |A_l,vw| / A_l,vv and lambda_l the largest eigenvalue of
 * diag(r_v A_l,vv)^-1 A_l (<= 1 by Gershgorin), so that diag(T_v A_l,vv)^-1
 * A_l tops out at exactly 1.  The smoother uses the diagonal
 * D_v = 1.05 p_v A_l,vv and the Chebyshev interval [0.2, 1] without the power
 * iteration of RC_SOLVE_PCG_MG; its degree-2 polynomial still damps
 * eigenvalues up to 1.2, so predictions low by up to ~14% keep it
 * convergent.  The V-cycle stays linear and symmetric, so PCG applies;
 * RC_SOLVE_PCG_LEARNED falls back to RC_SOLVE_PCG_MG when its residual keeps
 * growing (fallback_after).
 * ---------------------------------------------------------------------- */

/* Number of MLP parameters (4,801), flat order W1 [8][64], b1 [64],
 * W2 [64][64], b2 [64], W3 [64], b3 [1]. */
int32_t rc_mlp_n_params(void);

/* Creates an MLP on `stream` with parameters theta_h (host float[n_params],
 * NULL = zeros).  Weights are held in FP32 (master, Adam state) and FP16
 * (used by the forward pass); biases in FP32. */
rc_status rc_mlp_create(const float* theta_h, rc_stream stream, rc_mlp** out);
rc_status rc_mlp_destroy(rc_mlp* mlp);
/* Copies the FP32 parameters to / from the host; set also resets Adam. */
rc_status rc_mlp_get(rc_mlp* mlp, float* theta_h);
rc_status rc_mlp_set(rc_mlp* mlp, const float* theta_h);
/* Y = y(X) for N rows: X device float[N][8], Y device float[N]. */
rc_status rc_mlp_forward(rc_mlp* mlp, const float* X, int32_t N, float* Y);
/* grad = d(sum_r dY[r] y(X[r]))/dtheta (device float[n_params]); runs the
 * forward pass itself.  X, dY: device float. */
rc_status rc_mlp_backward(rc_mlp* mlp, const float* X, int32_t N, const float* dY, float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient grad
 * (device float[n_params]) and learning rate lr > 0. */
rc_status rc_mlp_adam(rc_mlp* mlp, const float* grad, float lr);

/* Attaches mlp (NULL detaches) to the context for RC_SOLVE_PCG_LEARNED; the
 * caller keeps ownership. */
rc_status rc_learned_attach(rc_ctx* ctx, rc_mlp* mlp);

/* Level sizes of the hierarchy for coarsest size n_min (sizes_h: host
 * int32[max_levels]); returns the number of levels in *levels. */
rc_status rc_learned_levels(rc_ctx* ctx, int32_t n_min, int32_t* sizes_h, int32_t max_levels, int32_t* levels);

/* Features of every level at gamma (levels stacked, finest first): X device
 * float[N][8] with N the sum of the level sizes; diag (optional) device
 * double[N] the level diagonals.  RC_ERR_UNSUPPORTED unless the curve is one
 * closed loop numbered along itself. */
rc_status rc_learned_features(rc_ctx* ctx, const double* gamma, int32_t n_min, float* X, double* diag);

/* Training targets at gamma: R device float[N] (levels stacked as for
 * rc_learned_features), T_v = r_v lambda_l from each level's dense FP64
 * operator (assembled in a temporary buffer of nV^2 doubles; nV <= 16,384),
 * lambda_l the Rayleigh quotient after 60 power steps from the alternating
 * vector (a lower bound, within ~0.5% here).  Synchronises the stream. */
rc_status rc_learned_targets(rc_ctx* ctx, const double* gamma, int32_t n_min, float* R);

/* One regression step of the MLP on rows X (device float[N][8]) with targets
 * R (device float[N], > 1): p = 1 + y(X), loss = mean of
 * w (log p - log R)^2 with w = 4 where p < R (an interval short of the
 * spectrum) and 1 elsewhere; *loss_h receives the loss before the step, grad (optional,
 * device float[n_params]) its gradient, and lr > 0 takes one Adam step
 * (lr = 0: none).  Synchronises the MLP's stream. */
rc_status rc_mlp_fit_step(rc_mlp* mlp, const float* X, const float* R, int32_t N, float lr, double* loss_h,
                          float* grad);

/* Kernel timing with HIP events on the context's stream.  rc_profile_enable
 * clears earlier records and, when enable != 0, brackets every launch of the
 * FP32/FP64 pair kernels with a pair of events.  rc_profile_read synchronises
 * the stream and returns the summed duration (ms) and the launch count of
 * which = 0: the energy + differential pair kernel, 1: the FP32 operator pair
 * kernel on the finest level (coarse multigrid levels are not timed), 2: the
 * 16-bit assembled product kernel on the finest level, 3: the FP32 assembled
 * product kernel, 4: the FP64 operator pair kernel on the finest level, 5: the
 * batch's assembled per-instance product (not recorded inside a captured step),
 * 6: the Barnes-Hut traversal kernel. */
rc_status rc_profile_enable(rc_ctx* ctx, int32_t enable);
rc_status rc_profile_read(rc_ctx* ctx, int32_t which, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* RCURVES_H */
