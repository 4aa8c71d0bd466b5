// Solver state of a context: constraints, dense saddle factorisation and the
// multigrid hierarchy, each held per level (level 0 is the context's curve).
#pragma once

#include <memory>
#include <vector>

#include "k_linalg.h"
#include "rc_internal.h"

namespace rc {

// Constraint Jacobian C of one curve, split into "path" rows (edge-length
// rows in chain order, a block-tridiagonal C_p C_p^T) and dense "border" rows
// (barycenter, total length, and the first edge of every loop, whose removal
// leaves the path rows tridiagonal).  C C^T is solved through the border
// Schur complement S = K_bb - K_pb^T K_pp^-1 K_pb.
// Vertices held on an implicit surface (Sec. 7.1, Phi = f(gamma_i)), f the signed distance of a
// sphere (par = c, r) or of a torus about the z axis through c (par = c, R, r).
struct SurfSpec {
  int kind = 0;  // 0 none, RC_SURFACE_SPHERE, RC_SURFACE_TORUS
  double par[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  std::vector<int> verts;
  bool operator==(const SurfSpec& o) const {
    for (int q = 0; q < 5; ++q)
      if (par[q] != o.par[q]) return false;
    return kind == o.kind && verts == o.verts;
  }
  bool operator!=(const SurfSpec& o) const { return !(*this == o); }
};

// Edges whose unit tangent is prescribed (Sec. 7.1), as the two rows (u . T_I, v . T_I) over an
// orthonormal basis (u, v) of the plane orthogonal to the direction X.
struct TangentSpec {
  std::vector<int> edges;
  std::vector<double> basis;  // [n][6]: u then v
  bool operator==(const TangentSpec& o) const { return edges == o.edges && basis == o.basis; }
  bool operator!=(const TangentSpec& o) const { return !(*this == o); }
};

struct Cons {
  uint32_t mask = 0;
  int bary = 0, total = 0, edge = 0;
  int nb = 0, np = 0, ncut = 0, k = 0;  // border rows, path rows, cut edges, all rows
  // point constraints (Sec. 7.1) are eliminated rather than bordered: with F = diag(free),
  // free[v] = 0 at the pinned vertices, the projector onto null(C) n {x_P = 0} is
  // F - F C^T (C F C^T)^-1 C F, the weighted projector with W = F (and the smoother's
  // W = D^-1 F), so they add no border rows
  int npt = 0, nbt = 0, nd = 0;         // pinned vertices; barycenter + total rows; rows before the edge rows
                                        // (nbt + 3 npt + nsf + 2 ntg)
  double total0 = 0.0;
  std::vector<int> h_pt;                // pinned vertices, in row order
  int* pt = nullptr;
  double* ptx = nullptr;                // their targets x_i [npt][3]
  // surface constraints, eliminated the same way with W_v = w_v (I - n_v n_v^T)
  SurfSpec surf;
  int nsf = 0;
  int* sf = nullptr;                    // [nsf] the held vertices, in row order
  double* sgrad = nullptr;              // [nsf][3] grad f at the prepared curve
  double* nrm = nullptr;                // [nV][3] unit normals there (zero at other vertices)
  // tangent constraints: two rows of the projector's dense block each, after barycenter and total
  TangentSpec tang;
  int ntg = 0;
  int* tg = nullptr;                    // [ntg] edges
  double* tgb = nullptr;                // [ntg][6] bases
  int ext_tg = 0;                       // first tangent row in the external order
  bool elim = false;                    // point or surface constraints present
  double* free = nullptr;               // [nV] 0 at pinned vertices, else 1 (elim)
  double* weff = nullptr;               // [nV] the weights of the prepared factors (w or 1) * free
  std::vector<int> h_path_edge, h_path_prev, h_cut_edge, h_edge_path_row;
  int *path_edge = nullptr, *path_prev = nullptr, *cut_edge = nullptr, *edge_path_row = nullptr;
  double *x0 = nullptr, *len0 = nullptr, *ones = nullptr;
  double *geo = nullptr, *geo_eval = nullptr, *vals = nullptr;
  double *rows = nullptr, *ta = nullptr, *td = nullptr, *tc = nullptr;
  double *Kpb = nullptr, *Z = nullptr, *Sinv = nullptr, *tri_scratch = nullptr;
  double *wp = nullptr, *yp = nullptr, *wb = nullptr, *yb = nullptr, *dots = nullptr, *rhs = nullptr;
  double* small = nullptr;
  double* part = nullptr;  // partial sums of the three-launch projector
  // block-partitioned path solve: partition, spikes (V then W), reduced
  // inverse, and scratch (local solutions [max(nb, 1)][np], boundary values
  // [max(nb, 1)][nr], right-hand sides of the spikes [2 np])
  TriBlocks tri;
  double *sp_VW = nullptr, *sp_Rt = nullptr, *sp_g = nullptr, *sp_U = nullptr, *sp_tmp = nullptr;
  // packed path rows and vertices for the projector (vertex degree <= 2)
  ProjRow* prow = nullptr;
  ProjVert* pvert = nullptr;
  double* rowsW = nullptr;  // W rows (weighted factors only)
};

// Dense FP64 saddle solve on one curve: H = Abar + C^T C (Cholesky),
// W = H^-1 C^T, S = C W.  Projected gradient with right-hand side b:
// x = X b with X = H^-1 - W S^-1 W^T (kept explicitly, so a solve is one
// matrix-vector product); projection increment: x = -W S^-1 phi.
struct Dense {
  int nV = 0, k = 0;
  double *A = nullptr, *Cd = nullptr, *CtC = nullptr, *H = nullptr, *W = nullptr, *S = nullptr, *Sinv = nullptr,
         *X = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  int* info = nullptr;
  int* gjm = nullptr;        // Gauss-Jordan bookkeeping
  long long* gjo = nullptr;
  double* gjc = nullptr;     // Gauss-Jordan column panel scratch
};

struct Level {
  Curve curve;
  Cons cons;
  Cons cons_w;             // the same constraints with C W C^T (the smoother's weighted projector)
  int* fine_of = nullptr;  // coarse vertex -> fine vertex index
  int2* prolong = nullptr; // fine vertex -> (coarse a, coarse b): value (x_a + x_b) / 2
  int *restr_off = nullptr, *restr_idx = nullptr;  // coarse vertex -> fine vertices that reference it
  double* gamma = nullptr; // the level's vertex positions [nV][3]
  LowpOp lowp;             // assembled 16-bit operator of the level (precision path)
  Bvh bvh;                 // the level's block cluster tree (hierarchical operator)
  Bct bct;
};

struct MGLevelState {
  double *diag = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *pw = nullptr;
  double* w = nullptr;  // 1 / diag (weighted smoother)
  double lmax = 0.0;
};

// Batch solver state: the union of independent instances, each with its
// own barycenter and per-loop length constraints, PCG scalars and line search.
constexpr int kBatchScal = 16;  // per-instance PCG scalars
constexpr int kBatchLs = 16;    // per-instance line-search values
struct Batch {
  bool ready = false;
  int n_inst = 0, nq = 0;
  std::vector<int> h_chain_voff, h_inst_qoff, h_chain_eoff;
  int *chain_vert = nullptr, *chain_voff = nullptr, *chain_of_vertex = nullptr, *chain_inst = nullptr;
  int *inst_qoff = nullptr, *chain_eoff = nullptr, *chain_edges = nullptr;
  long long* blk_off = nullptr;   // offsets of the loop blocks in Minv
  size_t blk_total = 0;
  int max_chain = 0;
  double *Minv = nullptr, *gj_col = nullptr;
  float* MinvF = nullptr;          // FP32 copy of the inverted loop blocks (the preconditioner's operand)
  double *x0 = nullptr, *L0 = nullptr;
  double *Jv = nullptr, *Lv = nullptr, *qsum = nullptr, *Sinv = nullptr, *cq = nullptr, *yb = nullptr, *yq = nullptr;
  double *dvec = nullptr;
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *b = nullptr, *t = nullptr;
  double *sc = nullptr, *ls = nullptr, *energy = nullptr, *stats = nullptr;
  double *trial = nullptr, *ghat = nullptr, *dE = nullptr, *g = nullptr, *inc = nullptr;
  double *phiq = nullptr, *phib = nullptr;
  int* mask = nullptr;             // per-instance work mask of the pair kernels
  int gj_steps = 0, n_prec = 0;
  std::vector<int> h_gj_step_off, h_gj_tiles;
  int *gj_list = nullptr, *gj_pre = nullptr;
  int2* prec_items = nullptr;
  // coarse space of per-loop translations (two-level preconditioner)
  bool coarse = false;      // available (every instance has at most kCoarseMax loops)
  bool use_coarse = false;  // chosen by the options of the current solve
  // assembled per-instance blocks of Abar (FP32, row-major, diagonal unused)
  bool use_asm = false;
  float* Aasm = nullptr;
  long long* aoff = nullptr;
  size_t asm_total = 0;
  int n_asm_items = 0, n_rb = 0;
  int4* asm_items = nullptr;   // (instance, tile row, tile col >= tile row) of 16 x 16
  int2* rb_items = nullptr;    // (instance, first of 16 rows)
  int max_loops = 0, n_cpl = 0;
  int *cedge_loop = nullptr, *inst_ceoff = nullptr;
  int2* cpl_items = nullptr;
  float* Wp = nullptr;                 // [nE][max_loops] per-target-edge couplings
  double *Wc = nullptr, *Ainv = nullptr;  // [n_inst][max_loops^2]
  double *rsum = nullptr, *cl = nullptr;  // [nq][3]
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool captured = false;
  rc_batch_opts cap_opts{};
  const double* cap_gamma = nullptr;
};

}  // namespace rc

struct rc_ctx {
  int nV = 0, nE = 0;
  double alpha = 0, beta = 0;
  rc_dtype dtype = RC_F64;
  hipStream_t stream = nullptr;
  rc::Curve curve;
  rc::Cons cons;
  rc::Cons cons_w;        // finest level's constraints with C W C^T (weighted smoother)
  bool mg_weighted = false;  // smoothers use the weighted projector
  // FP64 work vectors [3 nV]
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr, *tmp2 = nullptr;
  double *diag = nullptr, *scal = nullptr, *red = nullptr, *trial = nullptr, *zmin = nullptr, *inc = nullptr;
  double *phi = nullptr, *dx = nullptr, *dEs = nullptr, *gs = nullptr;
  // multigrid: levels[0] is a placeholder for the finest level (curve, cons)
  std::vector<std::unique_ptr<rc::Level>> levels;
  std::vector<rc::MGLevelState> mg;
  rc::Dense coarse;  // dense saddle of the coarsest level
  bool mg_built = false;
  int mg_min = 0, cheb_deg = 0;
  // dense direct path on the finest level
  rc::Dense dense;
  rc::Bvh bvh;
  rc::CcdBuffers ccd;
  rc::Bvh bct_bvh;  // the block cluster tree's own BVH
  rc::Bct bct;
  double bct_theta = 0.0;  // the solver's hierarchical operator (0 = exact)
  int bct_min_v = 0;
  rc::KernelTimer timer;
  unsigned* status_dev = nullptr;  // device status word (RC_FLAG_* bits latched by kernels)
  unsigned* setup_flags = nullptr;  // device word: kSetup* bits latched by the constraint set-up (setup_check)
  unsigned status_host = 0;        // RC_FLAG_* bits latched by the host-side solver
  // precision path: the finest level's assembled 16-bit operator; levels
  // 0 .. lowp_levels-1 use their assembled operator in the current solve
  rc::LowpOp lowp;
  int lowp_levels = 0, lowp_fmt = 0, lowp_band = 0, lowp_outer = 0;
  int last_sweeps = 0;  // FP64 true-residual evaluations of the last PCG solve
  // PCG's residual norms are relative to |P b|; with pcg_ref > |P b| the tolerance is relative to pcg_ref
  // instead (an absolute target, capped at 0.02 relative); last_bnorm is the last solve's |P b|
  double pcg_ref = 0.0, last_bnorm = 0.0;
  rc::Batch batch;      // batch contexts only
  // learned / hand-weighted multilevel preconditioner
  rc_mlp* mlp = nullptr;          // attached, not owned
  int learn_nmin = -1, learn_N = 0, learn_cap = 0;
  std::vector<int> learn_off;     // row offset of every level
  double* learn_diag = nullptr;
  double* learn_scratch = nullptr;
  float *learn_X = nullptr, *learn_Y = nullptr;
  bool mg_learned = false;  // the V-cycle's smoothers take the attached MLP's weights
  bool mg_cg = false;       // the standalone multigrid with CG smoothing (no Chebyshev interval)
  // point constraints of the finest level (kept across rc_set_constraints)
  std::vector<int> pts;
  std::vector<double> pts_x;
  rc::SurfSpec surf;
  rc::TangentSpec tang;
  size_t phi_cap = 0;  // rows the phi buffer holds (twice)
};

struct rc_mlp {
  rc::Mlp m;
};

namespace rc {

rc_status sync(rc_ctx* c);
rc_status fetch(rc_ctx* c, const double* dev, double* host, int n);
bool trace_on();

rc_status cons_alloc(rc_ctx* c, const Curve& cv, Cons& k, uint32_t mask, const std::vector<int>& pts = {},
                     const SurfSpec* surf = nullptr, const TangentSpec* tang = nullptr);
void cons_free(Cons& k);
// Failures of the constraint set-up latched in rc_ctx::setup_flags.
constexpr unsigned kSetupGram = 1u;   // the path block's tridiagonal factorisation broke down
constexpr unsigned kSetupSchur = 2u;  // the border Schur complement is singular
// Enqueues the factors of C C^T (or C W C^T) without waiting for the device (except for a border of
// more than kSchurDevMax rows, whose Schur complement is inverted on the host): a failed factorisation
// is latched in c->setup_flags and reported by setup_check.
rc_status cons_prepare(rc_ctx* c, const Curve& cv, Cons& k, const double* gamma, const double* w = nullptr);
// Waits for the stream, reports (and clears) the constraint set-up's latched failures.
rc_status setup_check(rc_ctx* c);
// With pop, the last launch also writes the operand of pop's next product,
// taken of out (of xacc when pfrom_x); returns whether it did.
bool cons_project(rc_ctx* c, const Curve& cv, Cons& k, const double* in, double* out, double* xacc = nullptr,
                  const LowpOp* pop = nullptr, bool pfrom_x = false);
void cons_values(rc_ctx* c, const double* gamma, double* phi);
rc_status cons_set_targets(rc_ctx* c, const double* gamma_ref, const double* x0_h, double total_len0,
                           const double* edge_len0);

void dense_free(Dense& d);
void mg_free(rc_ctx* c);

rc_status load_geometry(rc_ctx* c, const double* gamma);
rc_status prepare_solver(rc_ctx* c, const double* gamma, const rc_solve_opts& o);
rc_status solve_gradient(rc_ctx* c, const double* gamma, const double* rhs, double* out, rc_solve_opts& o,
                         int* iters, double* res, int* fell);
rc_status solve_prepared(rc_ctx* c, const double* rhs, double* out, const rc_solve_opts& o, int* iters, double* res);

struct LsResult {
  double tau = 0.0, E1 = 0.0, tau_max = 0.0;
  int backtracks = 0, proj_iters = 0, proj_solve_iters = 0;
};
rc_status line_search(rc_ctx* c, double* gamma, double E0, const double* dE, const double* g, const rc_ls_opts& ls,
                      const rc_solve_opts& so, LsResult* out);

rc_status learn_prepare_levels(rc_ctx* c, int n_min);
rc_status learn_levels_at(rc_ctx* c, const double* gamma, int n_min, bool features, float* R);
void learn_free(rc_ctx* c);

// batch.hip
rc_status batch_alloc(rc_ctx* c);
void batch_free(rc_ctx* c);
rc_status batch_edge_sums(rc_ctx* c, int slot, double* out);
rc_status batch_set_constraints(rc_ctx* c, const double* gamma_ref);
rc_status batch_apply(rc_ctx* c, const double* gamma, const double* X, double* Y, bool assembled);
rc_status batch_gradient(rc_ctx* c, const double* gamma, const double* dE, double* g, const rc_batch_opts& o);
rc_status batch_step(rc_ctx* c, double* gamma, const rc_batch_opts& o, double* stats_h);
void batch_invalidate_graph(rc_ctx* c);
rc_status batch_autotune(rc_ctx* c, const double* gamma, const char* cache, int* src_out, int* bpc_out,
                         double* ms_out);

}  // namespace rc
