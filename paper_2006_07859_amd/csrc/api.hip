// C ABI of librcurves: argument validation, context lifetime and the entry
// points declared in include/rcurves.h.  The solvers live in solver.hip.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>

#include "k_linalg.h"
#include "solver.h"

namespace rc {

const char* last_error();

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

template <typename T>
static rc_status dalloc(T** p, size_t n) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return RC_ERR_NOMEM;
  }
  return RC_OK;
}

}  // namespace rc

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace rc;

namespace {

rc_status check_ctx(const rc_ctx* c) {
  if (!c) {
    set_error("null context");
    return RC_ERR_ARG;
  }
  return RC_OK;
}

rc_status check_ptrs(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (!p) {
      set_error("null pointer argument");
      return RC_ERR_ARG;
    }
  return RC_OK;
}

// Entry points whose sums or solves assume one network reject batch contexts.
rc_status no_batch(const rc_ctx* c, const char* name) {
  if (c->curve.n_inst > 0) {
    set_error(std::string(name) + ": not available on a batch context (use the rc_batch_* calls)");
    return RC_ERR_UNSUPPORTED;
  }
  return RC_OK;
}

rc_solve_opts resolve(const rc_solve_opts* o) {
  rc_solve_opts d;
  rc_default_solve_opts(&d);
  if (o) d = *o;
  if (d.max_iter <= 0) d.max_iter = 500;
  if (!(d.tol > 0)) d.tol = 1e-6;
  if (d.mg_min_vertices <= 0) d.mg_min_vertices = 256;
  if (d.cheb_degree <= 0) d.cheb_degree = 2;
  if (d.lowp_min_vertices <= 0) d.lowp_min_vertices = 1 << 30;  // finest level only
  if (!(d.inner_tol > 0.0) || !(d.inner_tol < 1.0)) d.inner_tol = 0.0;
  if (d.fallback_after < 0) d.fallback_after = 0;
  return d;
}

rc_ls_opts resolve_ls(const rc_ls_opts* o) {
  rc_ls_opts d;
  rc_default_ls_opts(&d);
  if (o) d = *o;
  return d;
}

}  // namespace

extern "C" {

void rc_default_solve_opts(rc_solve_opts* o) {
  if (!o) return;
  o->solver = RC_SOLVE_PCG_MG;
  o->tol = 1e-6;
  o->max_iter = 200;
  o->replace_every = 0;
  o->mg_min_vertices = 256;
  o->cheb_degree = 2;
  o->op_f64 = 1;
  o->lowp = 0;
  o->lowp_band = 16;
  o->lowp_min_vertices = 4096;
  o->lowp_outer = 0;
  o->inner_tol = 0.0;
  o->fallback_after = 10;
  o->bct_theta = 0.0;
  o->bct_min_vertices = 32768;
}

void rc_default_ls_opts(rc_ls_opts* o) {
  if (!o) return;
  o->c_armijo = 0.01;
  o->shrink = 0.5;
  o->tau0 = 1.0;
  o->max_backtracks = 30;
  o->max_proj_iter = 10;
  o->proj_tol = 1e-10;
  o->proj_solve_tol = 1e-3;
  o->ccd = 0;
  o->bh_theta = 0.0;
  o->bh_refit = 0;
}

const char* rc_last_error(void) { return rc::last_error(); }

static rc_status create_ctx(int32_t nV, int32_t nE, const int32_t* edges_h, double alpha, double beta,
                            rc_dtype dtype, rc_stream stream, int32_t n_inst, const int32_t* voff_h,
                            rc_ctx** out) {
  set_error("");
  if (!out || !edges_h || nV <= 0 || nE <= 0) {
    set_error("rc_create: null pointer or empty curve");
    return RC_ERR_ARG;
  }
  *out = nullptr;
  if (dtype != RC_F32 && dtype != RC_F64) {
    set_error("rc_create: bad dtype");
    return RC_ERR_ARG;
  }
  if (!(alpha > 1.0) || !(beta >= alpha + 2.0) || !(beta < 2.0 * alpha + 1.0)) {
    set_error("rc_create: need alpha > 1 and alpha + 2 <= beta < 2 alpha + 1");
    return RC_ERR_PARAM_RANGE;
  }
  for (int i = 0; i < 2 * nE; ++i)
    if (edges_h[i] < 0 || edges_h[i] >= nV) {
      set_error("rc_create: edge endpoint out of range");
      return RC_ERR_ARG;
    }
  for (int I = 0; I < nE; ++I)
    if (edges_h[2 * I] == edges_h[2 * I + 1]) {
      set_error("rc_create: edge with equal endpoints");
      return RC_ERR_DEGENERATE;
    }
  std::unique_ptr<rc_ctx> c(new rc_ctx());
  c->nV = nV;
  c->nE = nE;
  c->alpha = alpha;
  c->beta = beta;
  c->dtype = dtype;
  c->stream = (hipStream_t)stream;
  RC_TRY(c->curve.init(nV, nE, edges_h));
  if (n_inst > 0) {
    RC_TRY(c->curve.set_instances(n_inst, voff_h));
    RC_TRY(batch_alloc(c.get()));
  } else if (c->curve.chain && alpha == 2.0 && dtype == RC_F32) {
    RC_TRY(c->curve.enable_vertex_pairs());
  }
  const size_t n3 = 3 * (size_t)nV;
  double** vecs[] = {&c->x,    &c->r,    &c->z,   &c->p,  &c->q,   &c->tmp, &c->tmp2,
                     &c->trial, &c->zmin, &c->inc, &c->dx, &c->dEs, &c->gs};
  for (double** v : vecs) RC_TRY(dalloc(v, n3));
  RC_TRY(dalloc(&c->diag, nV));
  RC_TRY(dalloc(&c->scal, 128));
  RC_TRY(dalloc(&c->red, (size_t)dot_scratch_size(kRedSets)));
  RC_TRY(dalloc(&c->phi, 2 * ((size_t)nE + 4)));
  c->phi_cap = (size_t)nE + 4;
  RC_TRY(dalloc(&c->status_dev, 1));
  RC_HIP(hipMemsetAsync(c->status_dev, 0, sizeof(unsigned), c->stream));
  RC_TRY(dalloc(&c->setup_flags, 1));
  RC_HIP(hipMemsetAsync(c->setup_flags, 0, sizeof(unsigned), c->stream));
  c->curve.status = c->status_dev;
  RC_HIP(hipMemsetAsync(c->x, 0, sizeof(double) * n3, c->stream));
  RC_TRY(sync(c.get()));
  *out = c.release();
  return RC_OK;
}

rc_status rc_create(int32_t nV, int32_t nE, const int32_t* edges_h, double alpha, double beta, rc_dtype dtype,
                    rc_stream stream, rc_ctx** out) {
  return create_ctx(nV, nE, edges_h, alpha, beta, dtype, stream, 0, nullptr, out);
}

rc_status rc_create_batch(int32_t n_inst, const int32_t* inst_vertex_off_h, int32_t n_vertices, int32_t n_edges,
                          const int32_t* edges_h, double alpha, double beta, rc_dtype dtype, rc_stream stream,
                          rc_ctx** out) {
  set_error("");
  if (n_inst < 1 || !inst_vertex_off_h) {
    set_error("rc_create_batch: need at least one instance and its vertex offsets");
    return RC_ERR_ARG;
  }
  return create_ctx(n_vertices, n_edges, edges_h, alpha, beta, dtype, stream, n_inst, inst_vertex_off_h, out);
}

rc_status rc_destroy(rc_ctx* c) {
  if (!c) return RC_OK;
  hipStreamSynchronize(c->stream);
  c->timer.clear();
  c->bvh.release();
  c->ccd.release();
  c->bct.release();
  c->bct_bvh.release();
  c->lowp.release();
  learn_free(c);
  batch_free(c);
  mg_free(c);
  dense_free(c->dense);
  cons_free(c->cons);
  c->curve.release();
  double* ps[] = {c->x,    c->r,    c->z,   c->p,   c->q,  c->tmp,  c->tmp2, c->diag, c->scal,
                  c->red,  c->trial, c->zmin, c->inc, c->phi, c->dx, c->dEs,  c->gs};
  for (double* p : ps)
    if (p) hipFree(p);
  if (c->status_dev) hipFree(c->status_dev);
  if (c->setup_flags) hipFree(c->setup_flags);
  delete c;
  return RC_OK;
}

// The RC_FLAG_* bit of a status returned by a solver call (0 for the others).
static unsigned flag_of(rc_status st) {
  switch (st) {
    case RC_ERR_NOT_CONVERGED: return RC_FLAG_NOT_CONVERGED;
    case RC_ERR_SINGULAR: return RC_FLAG_SINGULAR;
    case RC_ERR_PROJECTION: return RC_FLAG_PROJECTION;
    case RC_ERR_LINESEARCH: return RC_FLAG_LINESEARCH;
    default: return 0u;
  }
}

static rc_status latch_host(rc_ctx* c, rc_status st) {
  c->status_host |= flag_of(st);
  return st;
}

rc_status rc_sync_status(rc_ctx* c, rc_stats* out) {
  RC_TRY(check_ctx(c));
  unsigned dev = 0;
  RC_HIP(hipMemcpyAsync(&dev, c->status_dev, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  RC_HIP(hipMemsetAsync(c->status_dev, 0, sizeof(unsigned), c->stream));
  RC_HIP(hipStreamSynchronize(c->stream));
  const unsigned f = dev | c->status_host;
  c->status_host = 0;
  static const struct { unsigned bit; rc_status st; } order[] = {
      {RC_FLAG_INPUT_NONFINITE, RC_ERR_NONFINITE}, {RC_FLAG_ZERO_EDGE, RC_ERR_DEGENERATE},
      {RC_FLAG_PAIR_OVERFLOW, RC_ERR_DEGENERATE},  {RC_FLAG_RESULT_NONFINITE, RC_ERR_NONFINITE},
      {RC_FLAG_SINGULAR, RC_ERR_SINGULAR},         {RC_FLAG_NOT_CONVERGED, RC_ERR_NOT_CONVERGED},
      {RC_FLAG_PROJECTION, RC_ERR_PROJECTION},     {RC_FLAG_LINESEARCH, RC_ERR_LINESEARCH}};
  rc_status st = RC_OK;
  for (const auto& o : order)
    if (f & o.bit) {
      st = o.st;
      break;
    }
  if (out) {
    out->status = st;
    out->flags = f;
  }
  return st;
}

rc_status rc_use_vertex_pairs(rc_ctx* c, int32_t enable) {
  RC_TRY(check_ctx(c));
  if (!enable) {
    c->curve.vp = false;
    return RC_OK;
  }
  if (c->curve.n_inst > 0 || !c->curve.chain || c->alpha != 2.0 || c->dtype != RC_F32) {
    set_error("rc_use_vertex_pairs: needs an RC_F32 context with alpha = 2 on one network of vertex degree <= 2");
    return RC_ERR_UNSUPPORTED;
  }
  RC_HIP(hipStreamSynchronize(c->stream));
  return c->curve.enable_vertex_pairs();
}

rc_status rc_energy(rc_ctx* c, const double* gamma, double* energy) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, energy}));
  RC_TRY(launch_geometry(c->curve, gamma, c->dtype, c->stream));
  return launch_tpe(c->curve, c->alpha, c->beta, c->dtype, false, energy, nullptr, c->stream);
}

rc_status rc_differential(rc_ctx* c, const double* gamma, double* energy, double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, dE}));
  RC_TRY(launch_geometry(c->curve, gamma, c->dtype, c->stream));
  return launch_tpe(c->curve, c->alpha, c->beta, c->dtype, true, energy, dE, c->stream);
}

rc_status rc_sobolev_apply_prec(rc_ctx* c, const double* gamma, const double* X, double* Y, rc_dtype prec) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, X, Y}));
  if (prec != RC_F32 && prec != RC_F64) {
    set_error("bad precision");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_sobolev(c->curve, c->alpha, c->beta, prec, X, Y, nullptr, c->stream);
}

rc_status rc_sobolev_apply(rc_ctx* c, const double* gamma, const double* X, double* Y) {
  RC_TRY(check_ctx(c));
  return rc_sobolev_apply_prec(c, gamma, X, Y, c->dtype);
}

rc_status rc_sobolev_diag(rc_ctx* c, const double* gamma, double* diag) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, diag}));
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  RC_HIP(hipMemsetAsync(c->tmp, 0, sizeof(double) * 3 * c->nV, c->stream));
  return launch_sobolev(c->curve, c->alpha, c->beta, c->dtype, c->tmp, c->tmp2, diag, c->stream);
}

rc_status rc_assemble_dense(rc_ctx* c, const double* gamma, double* A) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_assemble_dense"));
  RC_TRY(check_ptrs({gamma, A}));
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_assemble_dense(c->curve, c->alpha, c->beta, A, c->stream);
}

rc_status rc_set_constraints(rc_ctx* c, uint32_t mask, const double* gamma_ref, const double* x0_h,
                             double total_len0, const double* edge_len0) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_constraints"));
  if (mask & ~7u) {
    set_error("unknown constraint flag");
    return RC_ERR_ARG;
  }
  if ((mask & RC_C_TOTAL_LENGTH) && (mask & RC_C_EDGE_LENGTH)) {
    set_error("total-length and edge-length constraints together are linearly dependent");
    return RC_ERR_ARG;
  }
  if (mask && !gamma_ref) {
    set_error("gamma_ref is required");
    return RC_ERR_ARG;
  }
  RC_TRY(sync(c));
  mg_free(c);  // the coarse levels carry constraints of the same kinds
  dense_free(c->dense);
  RC_TRY(cons_alloc(c, c->curve, c->cons, mask, c->pts, &c->surf, &c->tang));
  if (!c->pts.empty())
    RC_HIP(hipMemcpy(c->cons.ptx, c->pts_x.data(), sizeof(double) * c->pts_x.size(), hipMemcpyHostToDevice));
  if (mask == 0) return RC_OK;
  return cons_set_targets(c, gamma_ref, x0_h, total_len0, edge_len0);
}

namespace rc {
// Re-lays the finest level's constraint rows for the context's points and surface, keeping the
// targets of the other constraints.
static rc_status relay_constraints(rc_ctx* c) {
  RC_TRY(sync(c));
  Cons& k = c->cons;
  const uint32_t mask = k.mask;
  const double total0 = k.total0;
  double x0[3] = {0.0, 0.0, 0.0};
  std::vector<double> len0;
  if (k.geo) {
    RC_TRY(fetch(c, k.x0, x0, 3));
    len0.resize(c->nE);
    RC_TRY(fetch(c, k.len0, len0.data(), c->nE));
  }
  // Phi and its negation in the projection (2 k values)
  const size_t kmax = (size_t)c->nE + 4 + 3 * c->pts.size() + c->surf.verts.size() + 2 * c->tang.edges.size();
  if (kmax > c->phi_cap) {
    hipFree(c->phi);
    RC_TRY(dalloc(&c->phi, 2 * kmax));
    c->phi_cap = kmax;
  }
  mg_free(c);
  dense_free(c->dense);
  RC_TRY(cons_alloc(c, c->curve, k, mask, c->pts, &c->surf, &c->tang));
  k.total0 = total0;
  RC_HIP(hipMemcpy(k.x0, x0, sizeof(double) * 3, hipMemcpyHostToDevice));
  if (!len0.empty()) RC_HIP(hipMemcpy(k.len0, len0.data(), sizeof(double) * c->nE, hipMemcpyHostToDevice));
  if (!c->pts.empty())
    RC_HIP(hipMemcpy(k.ptx, c->pts_x.data(), sizeof(double) * c->pts_x.size(), hipMemcpyHostToDevice));
  return RC_OK;
}

// distinct indices in [0, nV), none of them in `other`
static bool valid_vertex_set(const std::vector<int>& v, int nV, const std::vector<int>& other) {
  std::vector<int> sorted = v;
  std::sort(sorted.begin(), sorted.end());
  if (!sorted.empty() && (sorted.front() < 0 || sorted.back() >= nV ||
                          std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()))
    return false;
  for (int u : other)
    if (std::binary_search(sorted.begin(), sorted.end(), u)) return false;
  return true;
}
}  // namespace rc

rc_status rc_set_point_constraints(rc_ctx* c, int32_t npt, const int32_t* vertices_h, const double* targets_h) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_point_constraints"));
  if (npt < 0 || npt > c->nV || (npt > 0 && (!vertices_h || !targets_h))) {
    set_error("point constraints: npt must lie in [0, nV], with host vertices and targets when positive");
    return RC_ERR_ARG;
  }
  std::vector<int> pts(vertices_h, vertices_h + npt);
  std::vector<double> px(targets_h, targets_h + 3 * (size_t)npt);
  if (!valid_vertex_set(pts, c->nV, c->surf.verts)) {
    set_error("point constraints: vertex out of range, given twice, or held on the surface");
    return RC_ERR_ARG;
  }
  for (double v : px)
    if (!std::isfinite(v)) {
      set_error("point constraints: non-finite target");
      return RC_ERR_ARG;
    }
  c->pts = pts;
  c->pts_x = px;
  return relay_constraints(c);
}

rc_status rc_set_surface_constraints(rc_ctx* c, int32_t kind, const double* params_h, int32_t n,
                                     const int32_t* vertices_h) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_surface_constraints"));
  if (n < 0 || n > c->nV || (n > 0 && (!vertices_h || !params_h)) ||
      (n > 0 && kind != RC_SURFACE_SPHERE && kind != RC_SURFACE_TORUS)) {
    set_error("surface constraints: n must lie in [0, nV], with a known kind, host parameters and vertices");
    return RC_ERR_ARG;
  }
  SurfSpec sp;
  if (n > 0) {
    sp.kind = kind;
    const int np_ = kind == RC_SURFACE_SPHERE ? 4 : 5;
    for (int q = 0; q < np_; ++q) {
      sp.par[q] = params_h[q];
      if (!std::isfinite(sp.par[q])) {
        set_error("surface constraints: non-finite parameter");
        return RC_ERR_ARG;
      }
    }
    const bool ok = kind == RC_SURFACE_SPHERE ? sp.par[3] > 0.0 : (sp.par[4] > 0.0 && sp.par[3] > sp.par[4]);
    if (!ok) {
      set_error("surface constraints: need r > 0 (sphere) or R > r > 0 (torus)");
      return RC_ERR_ARG;
    }
    sp.verts.assign(vertices_h, vertices_h + n);
    if (!valid_vertex_set(sp.verts, c->nV, c->pts)) {
      set_error("surface constraints: vertex out of range, given twice, or pinned");
      return RC_ERR_ARG;
    }
  }
  c->surf = sp;
  return relay_constraints(c);
}

int32_t rc_constraint_count(const rc_ctx* c) { return c ? c->cons.k : 0; }

rc_status rc_constraint_values(rc_ctx* c, const double* gamma, double* phi) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_constraint_values"));
  RC_TRY(check_ptrs({gamma, phi}));
  if (c->cons.k == 0) return RC_OK;
  cons_values(c, gamma, phi);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status rc_project(rc_ctx* c, const double* gamma, const double* X, double* Y) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_project"));
  RC_TRY(check_ptrs({gamma, X, Y}));
  RC_TRY(cons_prepare(c, c->curve, c->cons, gamma));
  RC_TRY(setup_check(c));
  cons_project(c, c->curve, c->cons, X, Y);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status rc_sobolev_gradient(rc_ctx* c, const double* gamma, const double* dE, double* g,
                              const rc_solve_opts* opts, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_sobolev_gradient"));
  RC_TRY(check_ptrs({gamma, dE, g}));
  rc_solve_opts o = resolve(opts);
  int iters = 0, fell = 0;
  double res = 0.0;
  rc_status st = latch_host(c, solve_gradient(c, gamma, dE, g, o, &iters, &res, &fell));
  if (stats) {
    stats->iterations = iters;
    stats->residual = res;
    stats->sweeps = c->last_sweeps;
    stats->status = st;
    stats->fallback = fell;
  }
  return st;
}

rc_status rc_line_search_step(rc_ctx* c, double* gamma, double energy0, const double* dE, const double* g,
                              const rc_ls_opts* ls, const rc_solve_opts* so, double* tau_h, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_line_search_step"));
  RC_TRY(check_ptrs({gamma, dE, g}));
  rc_solve_opts o = resolve(so);
  rc_ls_opts l = resolve_ls(ls);
  RC_TRY(prepare_solver(c, gamma, o));
  LsResult r;
  rc_status st = latch_host(c, line_search(c, gamma, energy0, dE, g, l, o, &r));
  if (tau_h) *tau_h = r.tau;
  if (stats) {
    stats->tau = r.tau;
    stats->energy_new = r.E1;
    stats->backtracks = r.backtracks;
    stats->proj_iters = r.proj_iters;
    stats->proj_solve_iterations = r.proj_solve_iters;
    stats->tau_max = r.tau_max;
    stats->status = st;
  }
  return st;
}

rc_status rc_bct_build(rc_ctx* c, const double* gamma, double theta, int32_t leaf_size) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_bct_build"));
  RC_TRY(check_ptrs({gamma}));
  if (!(theta > 0.0) || !std::isfinite(theta) || leaf_size < 1 || leaf_size > 32) {
    set_error("rc_bct_build: need theta > 0 and 1 <= leaf_size <= 32");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return build_bct(c->curve, c->bct_bvh, c->bct, theta, leaf_size, c->stream);
}

rc_status rc_bct_stats(rc_ctx* c, int64_t* stats_h) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({stats_h}));
  if (!c->bct.ready) {
    set_error("rc_bct_stats: no block cluster tree built");
    return RC_ERR_ARG;
  }
  stats_h[0] = c->bct.n_nodes;
  stats_h[1] = c->bct.n_far;
  stats_h[2] = c->bct.n_near;
  stats_h[3] = c->bct.near_pairs;
  return RC_OK;
}

rc_status rc_sobolev_apply_bct(rc_ctx* c, const double* gamma, const double* X, double* Y) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_sobolev_apply_bct"));
  RC_TRY(check_ptrs({gamma, X, Y}));
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_bct_apply(c->curve, c->bct_bvh, c->bct, c->alpha, c->beta, X, Y, c->stream);
}

rc_status rc_first_collision_time(rc_ctx* c, const double* gamma, const double* D, double horizon, double* t) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, D, t}));
  if (!(horizon > 0.0) || !std::isfinite(horizon)) {
    set_error("rc_first_collision_time: horizon must be positive and finite");
    return RC_ERR_ARG;
  }
  RC_TRY(c->ccd.ensure(c->nE));
  return launch_first_collision(c->curve, gamma, D, horizon, c->ccd, t, c->stream);
}

rc_status rc_step(rc_ctx* c, double* gamma, const rc_solve_opts* so, const rc_ls_opts* ls, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_step"));
  RC_TRY(check_ptrs({gamma}));
  rc_solve_opts o = resolve(so);
  rc_ls_opts l = resolve_ls(ls);
  if (!(l.bh_theta >= 0.0 && l.bh_theta < 0.5)) {
    set_error("rc_step: bh_theta must be 0 or lie in (0, 0.5)");
    return RC_ERR_ARG;
  }
  if (l.bh_theta > 0.0 && (c->curve.pen.on || c->curve.obstacle.on || c->curve.spot.on)) {
    set_error("rc_step: the Barnes-Hut evaluation (bh_theta > 0) carries no penalties or obstacle");
    return RC_ERR_UNSUPPORTED;
  }
  hipStream_t s = c->stream;
  // dE and g live in buffers that no solver routine touches
  double* dEb = c->dEs;
  double* gb = c->gs;
  rc_stats local{};
  rc_status st = RC_OK;
  hipEvent_t ev[4];
  for (hipEvent_t& e : ev) RC_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));  // timing only
  int nev = 0;
  RC_HIP(hipEventRecord(ev[nev++], s));
  do {
    if (l.bh_theta > 0.0) {
      st = launch_geometry(c->curve, gamma, RC_F32, s);
      if (st) break;
      st = launch_bh(c->curve, c->bvh, c->alpha, c->beta, l.bh_theta, kStepBhLeaf, c->scal + 8, dEb, s);
    } else {
      st = launch_geometry(c->curve, gamma, c->dtype, s);
      if (st) break;
      st = launch_tpe(c->curve, c->alpha, c->beta, c->dtype, true, c->scal + 8, dEb, s);
    }
    if (st) break;
    RC_HIP(hipEventRecord(ev[nev++], s));
    st = fetch(c, c->scal + 8, &local.energy, 1);
    if (st) break;
    if (!std::isfinite(local.energy)) {
      set_error("energy is not finite");
      st = RC_ERR_NONFINITE;
      break;
    }
    int iters = 0, fell = 0;
    double res = 0.0;
    st = solve_gradient(c, gamma, dEb, gb, o, &iters, &res, &fell);  // o becomes multigrid on a fallback
    local.iterations = iters;
    local.residual = res;
    local.sweeps = c->last_sweeps;
    local.fallback = fell;
    if (st) break;
    vec_dot(gb, gb, 3 * c->nV, c->red, c->scal, s);
    double gg;
    st = fetch(c, c->scal, &gg, 1);
    if (st) break;
    local.grad_norm = std::sqrt(gg);
    RC_HIP(hipEventRecord(ev[nev++], s));
    LsResult r;
    st = line_search(c, gamma, local.energy, dEb, gb, l, o, &r);
    local.tau = r.tau;
    local.energy_new = r.E1;
    local.backtracks = r.backtracks;
    local.proj_iters = r.proj_iters;
    local.proj_solve_iterations = r.proj_solve_iters;
    local.tau_max = r.tau_max;
    RC_HIP(hipEventRecord(ev[nev++], s));
  } while (false);
  hipStreamSynchronize(s);
  float ms = 0.f;
  if (nev > 1 && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) local.t_eval_ms = ms;
  if (nev > 2 && hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) local.t_solve_ms = ms;
  if (nev > 3 && hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) local.t_search_ms = ms;
  for (hipEvent_t e : ev) hipEventDestroy(e);
  local.status = st;
  latch_host(c, st);
  if (stats) *stats = local;
  return st;
}

}  // extern "C"

extern "C" rc_status rc_midpoint_differential(rc_ctx* c, const double* gamma, double* energy, double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_midpoint_differential"));
  RC_TRY(check_ptrs({gamma, dE}));
  RC_TRY(launch_geometry(c->curve, gamma, c->dtype, c->stream));
  return launch_midpoint(c->curve, c->alpha, c->beta, c->dtype, energy, dE, c->stream);
}

extern "C" rc_status rc_profile_enable(rc_ctx* c, int32_t enable) {
  RC_TRY(check_ctx(c));
  RC_HIP(hipStreamSynchronize(c->stream));
  c->timer.clear();
  c->timer.on = enable != 0;
  c->curve.timer = enable ? &c->timer : nullptr;
  return RC_OK;
}

extern "C" rc_status rc_profile_read(rc_ctx* c, int32_t which, double* total_ms, int32_t* launches) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({total_ms, launches}));
  if (which < 0 || which > 6) {
    set_error("rc_profile_read: which must be 0 (energy+differential pairs), 1 (FP32 operator pairs), 2 "
              "(assembled 16-bit product), 3 (assembled FP32 product), 4 (FP64 operator pairs), 5 (batch "
              "assembled product) or 6 (Barnes-Hut traversal)");
    return RC_ERR_ARG;
  }
  RC_HIP(hipStreamSynchronize(c->stream));
  const std::vector<hipEvent_t>& v =
      which == 0 ? c->timer.tpe : which == 1 ? c->timer.sob : which == 2 ? c->timer.lowp
                                : which == 3 ? c->timer.asm32 : which == 4 ? c->timer.sob64
                                : which == 5 ? c->timer.basm : c->timer.bh;
  double tot = 0.0;
  for (size_t i = 0; i + 1 < v.size(); i += 2) {
    float ms = 0.f;
    RC_HIP(hipEventElapsedTime(&ms, v[i], v[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int32_t)(v.size() / 2);
  return RC_OK;
}

extern "C" rc_status rc_bh_differential(rc_ctx* c, const double* gamma, double theta, int32_t leaf_size,
                                        double* energy, double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_bh_differential"));
  RC_TRY(check_ptrs({gamma, dE}));
  if (!(theta > 0.0) || !(theta < 0.5)) {
    set_error("rc_bh_differential: theta must lie in (0, 0.5) so that a target's own cluster is never admissible");
    return RC_ERR_ARG;
  }
  if (leaf_size < 1 || leaf_size > 256) {
    set_error("rc_bh_differential: leaf_size must lie in [1, 256]");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_bh(c->curve, c->bvh, c->alpha, c->beta, theta, leaf_size, energy, dE, c->stream);
}

extern "C" rc_status rc_bh_refit_differential(rc_ctx* c, const double* gamma, double theta, double* energy,
                                              double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_bh_refit_differential"));
  RC_TRY(check_ptrs({gamma, dE}));
  if (!(theta > 0.0) || !(theta < 0.5)) {
    set_error("rc_bh_refit_differential: theta must lie in (0, 0.5)");
    return RC_ERR_ARG;
  }
  if (c->bvh.n_nodes <= 0) {
    set_error("rc_bh_refit_differential: no Barnes-Hut tree built on this context yet");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_bh(c->curve, c->bvh, c->alpha, c->beta, theta, 0, energy, dE, c->stream, true);
}

extern "C" rc_status rc_bh_last_work(rc_ctx* c, int64_t* far_pairs, int64_t* near_pairs, int32_t* nodes,
                                     int32_t* depth) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({far_pairs, near_pairs, nodes, depth}));
  if (!c->bvh.work) {
    set_error("rc_bh_last_work: no Barnes-Hut evaluation yet");
    return RC_ERR_ARG;
  }
  unsigned long long w[2];
  RC_HIP(hipMemcpyAsync(w, c->bvh.work, sizeof(w), hipMemcpyDeviceToHost, c->stream));
  RC_HIP(hipStreamSynchronize(c->stream));
  *far_pairs = (int64_t)w[0];
  *near_pairs = (int64_t)w[1];
  *nodes = c->bvh.n_nodes;
  *depth = c->bvh.depth;
  return RC_OK;
}

extern "C" rc_status rc_lowp_assemble(rc_ctx* c, const double* gamma, int32_t fmt, int32_t band, int32_t with_f32) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_lowp_assemble"));
  RC_TRY(check_ptrs({gamma}));
  if (fmt != 1 && fmt != 2) {
    set_error("rc_lowp_assemble: fmt must be 1 (BF16) or 2 (FP16)");
    return RC_ERR_ARG;
  }
  if (band < 0 || band > kLowpMaxBand) {
    set_error("rc_lowp_assemble: band must lie in [0, 64]");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_assemble_lowp(c->curve, c->lowp, fmt, band, with_f32 != 0, c->alpha, c->beta, nullptr, c->stream);
}

extern "C" rc_status rc_lowp_apply(rc_ctx* c, const double* X, double* Y, int32_t f32) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({X, Y}));
  if (f32) return launch_lowp_apply32(c->lowp, X, Y, c->stream, &c->timer);
  return launch_lowp_apply(c->lowp, X, Y, c->stream, &c->timer);
}

// ---------------------------------------------------------------------------
// obstacle and batch entry points
// ---------------------------------------------------------------------------
extern "C" rc_status rc_set_obstacle(rc_ctx* c, const double* center_h, double radius, double weight) {
  RC_TRY(check_ctx(c));
  Obstacle& o = c->curve.obstacle;
  if (weight == 0.0) {
    o.on = false;
    return RC_OK;
  }
  RC_TRY(check_ptrs({center_h}));
  if (!(radius > 0.0) || !std::isfinite(weight) || !(weight > 0.0)) {
    set_error("rc_set_obstacle: need radius > 0 and weight > 0 (weight 0 removes the obstacle)");
    return RC_ERR_ARG;
  }
  o.on = true;
  o.c[0] = center_h[0];
  o.c[1] = center_h[1];
  o.c[2] = center_h[2];
  o.R = radius;
  o.p = c->beta - c->alpha;
  o.w = weight;
  return RC_OK;
}

extern "C" rc_status rc_set_penalties(rc_ctx* c, double w_length, double w_diff, double w_field,
                                     const double* field_h) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_penalties"));
  if (!std::isfinite(w_length) || !std::isfinite(w_diff) || !std::isfinite(w_field) || w_length < 0.0 ||
      w_diff < 0.0 || w_field < 0.0) {
    set_error("rc_set_penalties: weights must be finite and >= 0");
    return RC_ERR_ARG;
  }
  Penalties& p = c->curve.pen;
  double X[3] = {0.0, 0.0, 1.0};
  if (w_field > 0.0) {
    RC_TRY(check_ptrs({field_h}));
    const double n = std::sqrt(field_h[0] * field_h[0] + field_h[1] * field_h[1] + field_h[2] * field_h[2]);
    if (!(n > 0.0) || !std::isfinite(n)) {
      set_error("rc_set_penalties: the field direction must be a nonzero finite vector");
      return RC_ERR_ARG;
    }
    for (int k = 0; k < 3; ++k) X[k] = field_h[k] / n;
  }
  p.w_len = w_length;
  p.w_diff = w_diff;
  p.w_field = w_field;
  for (int k = 0; k < 3; ++k) p.X[k] = X[k];
  p.on = w_length > 0.0 || w_diff > 0.0 || w_field > 0.0;
  return RC_OK;
}

extern "C" rc_status rc_set_surface_potential(rc_ctx* c, int32_t nP, const double* P_h, int32_t nF, const int32_t* F_h,
                                              double weight, double theta) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_surface_potential"));
  if (!std::isfinite(weight) || weight < 0.0 || !(theta >= 0.0 && theta < 1.0)) {
    set_error("rc_set_surface_potential: weight must be finite and >= 0, theta in [0, 1)");
    return RC_ERR_ARG;
  }
  SurfacePotential& sp = c->curve.spot;
  if (weight == 0.0) {
    RC_TRY(sync(c));
    sp.release();
    return RC_OK;
  }
  if (nP < 3 || nF < 1 || !P_h || !F_h) {
    set_error("rc_set_surface_potential: need at least 3 vertices, 1 triangle and host arrays");
    return RC_ERR_ARG;
  }
  for (int64_t i = 0; i < 3 * (int64_t)nF; ++i)
    if (F_h[i] < 0 || F_h[i] >= nP) {
      set_error("rc_set_surface_potential: triangle vertex out of range");
      return RC_ERR_ARG;
    }
  for (int64_t i = 0; i < 3 * (int64_t)nP; ++i)
    if (!std::isfinite(P_h[i])) {
      set_error("rc_set_surface_potential: non-finite surface vertex");
      return RC_ERR_ARG;
    }
  RC_TRY(sync(c));
  RC_TRY(build_surface_potential(sp, P_h, nP, F_h, nF));
  sp.w = weight;
  sp.p = c->beta - c->alpha;
  sp.theta = theta;
  sp.on = true;
  return RC_OK;
}

extern "C" int32_t rc_batch_size(const rc_ctx* c) { return c ? c->curve.n_inst : 0; }

extern "C" rc_status rc_batch_energies(rc_ctx* c, const double* gamma, double* energies, double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, energies}));
  if (c->curve.n_inst == 0) {
    set_error("rc_batch_energies: not a batch context");
    return RC_ERR_ARG;
  }
  RC_TRY(launch_geometry(c->curve, gamma, c->dtype, c->stream));
  RC_TRY(launch_tpe(c->curve, c->alpha, c->beta, c->dtype, dE != nullptr, nullptr, dE, c->stream));
  return batch_edge_sums(c, 0, energies);
}

extern "C" rc_status rc_batch_tiling(rc_ctx* c, int32_t src_chunk, int32_t blocks_per_cu) {
  RC_TRY(check_ctx(c));
  if (c->curve.n_inst == 0) {
    set_error("rc_batch_tiling: not a batch context");
    return RC_ERR_ARG;
  }
  RC_HIP(hipStreamSynchronize(c->stream));
  batch_invalidate_graph(c);
  return c->curve.build_items(src_chunk, blocks_per_cu);
}

extern "C" rc_status rc_batch_autotune(rc_ctx* c, const double* gamma, const char* cache_path, int32_t* src_chunk,
                                       int32_t* blocks_per_cu, double* ms) {
  RC_TRY(check_ctx(c));
  if (c->curve.n_inst == 0) {
    set_error("rc_batch_autotune: not a batch context");
    return RC_ERR_ARG;
  }
  RC_TRY(check_ptrs({gamma, src_chunk, blocks_per_cu, ms}));
  int a = 0, b = 0;
  double t = 0.0;
  RC_TRY(batch_autotune(c, gamma, cache_path, &a, &b, &t));
  *src_chunk = a;
  *blocks_per_cu = b;
  *ms = t;
  return RC_OK;
}

extern "C" void rc_default_batch_opts(rc_batch_opts* o) {
  if (!o) return;
  o->tol = 1e-4;
  o->max_iter = 60;
  o->ls_rounds = 4;
  o->proj_iters = 2;
  o->proj_max_iter = 5;
  o->proj_tol = 1e-2;
  o->accept_tol = 1e-6;
  o->c_armijo = 0.01;
  o->tau0 = 1.0;
  o->graph = 0;
  o->check_every = 5;
  o->coarse = 1;
  o->op_assembled = 1;
  o->refine = 0;
  o->inner_tol = 1e-4;
}

static rc_status batch_ctx(rc_ctx* c, const char* name) {
  RC_TRY(check_ctx(c));
  if (c->curve.n_inst == 0) {
    set_error(std::string(name) + ": not a batch context");
    return RC_ERR_ARG;
  }
  return RC_OK;
}

static rc_status batch_opts(const rc_batch_opts* in, rc_batch_opts* o) {
  rc_default_batch_opts(o);
  if (in) *o = *in;
  if (!(o->tol > 0) || o->max_iter < 1 || o->ls_rounds < 1 || o->proj_iters < 0 || o->proj_max_iter < 1 ||
      !(o->proj_tol > 0) || !(o->accept_tol > 0) || !(o->c_armijo > 0) || !(o->tau0 > 0) || o->check_every < 0 ||
      (o->coarse != 0 && o->coarse != 1) || (o->op_assembled != 0 && o->op_assembled != 1) || o->refine < 0 ||
      o->refine > 20 || !(o->inner_tol > 0) || !(o->inner_tol < 1)) {
    set_error("batch options out of range");
    return RC_ERR_ARG;
  }
  if (o->max_iter > 10000 || o->ls_rounds > 60 || o->proj_iters > 20 || o->proj_max_iter > 10000) {
    set_error("batch options: trip counts too large");
    return RC_ERR_ARG;
  }
  return RC_OK;
}

extern "C" rc_status rc_batch_set_constraints(rc_ctx* c, const double* gamma_ref) {
  RC_TRY(batch_ctx(c, "rc_batch_set_constraints"));
  RC_TRY(check_ptrs({gamma_ref}));
  return batch_set_constraints(c, gamma_ref);
}

extern "C" rc_status rc_batch_gradient(rc_ctx* c, const double* gamma, const double* dE, double* g,
                                       const rc_batch_opts* opts) {
  RC_TRY(batch_ctx(c, "rc_batch_gradient"));
  RC_TRY(check_ptrs({gamma, dE, g}));
  rc_batch_opts o;
  RC_TRY(batch_opts(opts, &o));
  return batch_gradient(c, gamma, dE, g, o);
}

extern "C" rc_status rc_batch_step(rc_ctx* c, double* gamma, const rc_batch_opts* opts, double* stats_h) {
  RC_TRY(batch_ctx(c, "rc_batch_step"));
  RC_TRY(check_ptrs({gamma}));
  rc_batch_opts o;
  RC_TRY(batch_opts(opts, &o));
  return batch_step(c, gamma, o, stats_h);
}

extern "C" rc_status rc_batch_sobolev_apply(rc_ctx* c, const double* gamma, const double* X, double* Y,
                                            int32_t assembled) {
  RC_TRY(batch_ctx(c, "rc_batch_sobolev_apply"));
  RC_TRY(check_ptrs({gamma, X, Y}));
  if (assembled != 0 && assembled != 1) {
    set_error("rc_batch_sobolev_apply: assembled must be 0 or 1");
    return RC_ERR_ARG;
  }
  return batch_apply(c, gamma, X, Y, assembled != 0);
}

extern "C" rc_status rc_batch_pcg_state(rc_ctx* c, double* iters_h, double* res_h) {
  RC_TRY(batch_ctx(c, "rc_batch_pcg_state"));
  RC_TRY(check_ptrs({iters_h, res_h}));
  const int n = c->curve.n_inst;
  std::vector<double> sc((size_t)kBatchScal * n);
  RC_HIP(hipMemcpyAsync(sc.data(), c->batch.sc, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, c->stream));
  RC_HIP(hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) {
    iters_h[i] = sc[(size_t)i * kBatchScal + 8];
    res_h[i] = sc[(size_t)i * kBatchScal + 6];
  }
  return RC_OK;
}

// ---------------------------------------------------------------------------
// learned multilevel preconditioner
// ---------------------------------------------------------------------------
extern "C" int32_t rc_mlp_n_params(void) { return kMlpParams; }

extern "C" rc_status rc_mlp_create(const float* theta_h, rc_stream stream, rc_mlp** out) {
  RC_TRY(check_ptrs({out}));
  *out = nullptr;
  auto* m = new (std::nothrow) rc_mlp();
  if (!m) {
    set_error("out of host memory");
    return RC_ERR_NOMEM;
  }
  rc_status st = m->m.init(theta_h, (hipStream_t)stream);
  if (st != RC_OK) {
    m->m.release();
    delete m;
    return st;
  }
  *out = m;
  return RC_OK;
}

extern "C" rc_status rc_mlp_destroy(rc_mlp* m) {
  if (!m) return RC_OK;
  hipStreamSynchronize(m->m.stream);
  m->m.release();
  delete m;
  return RC_OK;
}

static rc_status check_mlp(const rc_mlp* m) {
  if (!m) {
    set_error("null MLP");
    return RC_ERR_ARG;
  }
  return RC_OK;
}

extern "C" rc_status rc_mlp_get(rc_mlp* m, float* theta_h) {
  RC_TRY(check_mlp(m));
  RC_TRY(check_ptrs({theta_h}));
  RC_HIP(hipStreamSynchronize(m->m.stream));
  RC_HIP(hipMemcpy(theta_h, m->m.theta, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return RC_OK;
}

extern "C" rc_status rc_mlp_set(rc_mlp* m, const float* theta_h) {
  RC_TRY(check_mlp(m));
  RC_TRY(check_ptrs({theta_h}));
  RC_HIP(hipStreamSynchronize(m->m.stream));
  return m->m.set(theta_h);
}

extern "C" rc_status rc_mlp_forward(rc_mlp* m, const float* X, int32_t N, float* Y) {
  RC_TRY(check_mlp(m));
  if (N < 0) {
    set_error("rc_mlp_forward: N < 0");
    return RC_ERR_ARG;
  }
  if (N == 0) return RC_OK;
  RC_TRY(check_ptrs({X, Y}));
  return mlp_forward(m->m, X, N, Y, false, m->m.stream);
}

extern "C" rc_status rc_mlp_backward(rc_mlp* m, const float* X, int32_t N, const float* dY, float* grad) {
  RC_TRY(check_mlp(m));
  RC_TRY(check_ptrs({X, dY, grad}));
  if (N <= 0) {
    set_error("rc_mlp_backward: N must be positive");
    return RC_ERR_ARG;
  }
  RC_TRY(m->m.ensure_rows(N));  // allocates the output row buffer Y before it is passed on
  RC_TRY(mlp_forward(m->m, X, N, m->m.Y, true, m->m.stream));
  return mlp_backward(m->m, X, N, dY, grad, m->m.stream);
}

extern "C" rc_status rc_mlp_adam(rc_mlp* m, const float* grad, float lr) {
  RC_TRY(check_mlp(m));
  RC_TRY(check_ptrs({grad}));
  if (!(lr > 0.f)) {
    set_error("rc_mlp_adam: lr must be positive");
    return RC_ERR_ARG;
  }
  return mlp_adam(m->m, grad, lr, m->m.stream);
}

extern "C" rc_status rc_learned_attach(rc_ctx* c, rc_mlp* m) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_learned_attach"));
  c->mlp = m;
  return RC_OK;
}

extern "C" rc_status rc_learned_levels(rc_ctx* c, int32_t n_min, int32_t* sizes_h, int32_t max_levels,
                                       int32_t* levels) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_learned_levels"));
  RC_TRY(check_ptrs({levels}));
  RC_TRY(learn_prepare_levels(c, n_min));
  const int nl = (int)c->learn_off.size() - 1;
  *levels = nl;
  for (int l = 0; sizes_h && l < nl && l < max_levels; ++l) sizes_h[l] = c->learn_off[l + 1] - c->learn_off[l];
  return RC_OK;
}

extern "C" rc_status rc_learned_features(rc_ctx* c, const double* gamma, int32_t n_min, float* X, double* diag) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_learned_features"));
  RC_TRY(check_ptrs({gamma, X}));
  RC_TRY(learn_levels_at(c, gamma, n_min, true, nullptr));
  const int N = c->learn_N;
  RC_HIP(hipMemcpyAsync(X, c->learn_X, sizeof(float) * kMlpIn * N, hipMemcpyDeviceToDevice, c->stream));
  if (diag) RC_HIP(hipMemcpyAsync(diag, c->learn_diag, sizeof(double) * N, hipMemcpyDeviceToDevice, c->stream));
  return RC_OK;
}

extern "C" rc_status rc_learned_targets(rc_ctx* c, const double* gamma, int32_t n_min, float* R) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_learned_targets"));
  RC_TRY(check_ptrs({gamma, R}));
  return learn_levels_at(c, gamma, n_min, false, R);
}

extern "C" rc_status rc_mlp_fit_step(rc_mlp* m, const float* X, const float* R, int32_t N, float lr, double* loss_h,
                                     float* grad) {
  RC_TRY(check_mlp(m));
  RC_TRY(check_ptrs({X, R, loss_h}));
  if (N <= 0 || !(lr >= 0.f)) {
    set_error("rc_mlp_fit_step: N must be positive and lr >= 0");
    return RC_ERR_ARG;
  }
  double* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(double)) != hipSuccess) {
    set_error("rc_mlp_fit_step: allocation failed");
    return RC_ERR_NOMEM;
  }
  rc_status st = mlp_fit_step(m->m, X, R, N, lr, d, grad, m->m.stream);
  if (st == RC_OK && hipMemcpyAsync(loss_h, d, sizeof(double), hipMemcpyDeviceToHost, m->m.stream) != hipSuccess) {
    set_error("rc_mlp_fit_step: copy of the loss failed");
    st = RC_ERR_HIP;
  }
  if (hipStreamSynchronize(m->m.stream) != hipSuccess && st == RC_OK) {
    set_error("rc_mlp_fit_step: stream synchronisation failed");
    st = RC_ERR_HIP;
  }
  hipFree(d);
  return st;
}

rc_status rc_set_tangent_constraints(rc_ctx* c, int32_t n, const int32_t* edges_h, const double* dirs_h) {
  RC_TRY(check_ctx(c));
  RC_TRY(no_batch(c, "rc_set_tangent_constraints"));
  if (n < 0 || n > c->nE || (n > 0 && (!edges_h || !dirs_h))) {
    set_error("tangent constraints: n must lie in [0, nE], with host edges and directions when positive");
    return RC_ERR_ARG;
  }
  TangentSpec t;
  t.edges.assign(edges_h, edges_h + n);
  if (!valid_vertex_set(t.edges, c->nE, {})) {
    set_error("tangent constraints: edge out of range or given twice");
    return RC_ERR_ARG;
  }
  for (int j = 0; j < n; ++j) {
    double X[3] = {dirs_h[3 * j], dirs_h[3 * j + 1], dirs_h[3 * j + 2]};
    const double len = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    if (!(std::isfinite(len) && len > 0.0)) {
      set_error("tangent constraints: a direction is zero or not finite");
      return RC_ERR_ARG;
    }
    for (double& x : X) x /= len;
    // u = X x e_m / |X x e_m| with e_m the axis of the smallest |X_m| (the first on ties), v = X x u
    int m = 0;
    for (int q = 1; q < 3; ++q)
      if (std::fabs(X[q]) < std::fabs(X[m])) m = q;
    double em[3] = {0.0, 0.0, 0.0};
    em[m] = 1.0;
    double u[3] = {X[1] * em[2] - X[2] * em[1], X[2] * em[0] - X[0] * em[2], X[0] * em[1] - X[1] * em[0]};
    const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (double& x : u) x /= un;
    const double v[3] = {X[1] * u[2] - X[2] * u[1], X[2] * u[0] - X[0] * u[2], X[0] * u[1] - X[1] * u[0]};
    t.basis.insert(t.basis.end(), {u[0], u[1], u[2], v[0], v[1], v[2]});
  }
  c->tang = t;
  return relay_constraints(c);
}
