// C ABI of librcurves and the host-side orchestration of the solvers.
//
// The host drives the iterative loops (PCG, projection, line search) and
// reads back only the scalars that decide control flow; every vector
// operation runs in the kernels of k_pairs.hip and k_linalg.hip.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "k_linalg.h"
#include "rc_internal.h"

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

// ---------------------------------------------------------------------------
// constraint state
// ---------------------------------------------------------------------------
struct Cons {
  uint32_t mask = 0;
  int bary = 0, total = 0, edge = 0;
  int nb = 0, np = 0, ncut = 0, k = 0;  // border rows, path rows, cut edges, total rows
  double total0 = 0.0;
  std::vector<int> h_path_edge, h_path_prev, h_cut_edge, h_edge_path_row;
  int *path_edge = nullptr, *path_prev = nullptr, *cut_edge = nullptr, *edge_path_row = nullptr;
  double *x0 = nullptr, *len0 = nullptr, *ones = nullptr;
  double *geo = nullptr, *geo_eval = nullptr, *vals = nullptr;
  double *rows = nullptr, *ta = nullptr, *td = nullptr, *tc = nullptr;
  double *Kpb = nullptr, *Z = nullptr, *Sinv = nullptr, *tri_scratch = nullptr;
  double *wp = nullptr, *yp = nullptr, *wb = nullptr, *yb = nullptr, *dots = nullptr, *rhs = nullptr;
  double* small = nullptr;
  bool prepared = false;
};

// multigrid level (level 0 is the context's own curve)
struct Level {
  Curve curve;
  std::vector<int> h_fine_of;   // coarse vertex -> fine vertex index
  int* fine_of = nullptr;
  int2* prolong = nullptr;      // fine vertex -> (coarse a, coarse b), value = (x_a + x_b)/2
  int *restr_off = nullptr, *restr_idx = nullptr;  // coarse -> fine list (weights 1 or 1/2 via prolong)
  double* gamma = nullptr;      // this level's vertex positions [nV][3]
};

struct MGLevelState {
  double *diag = nullptr, *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *pw = nullptr;
  double lmax = 0.0;
};

}  // namespace rc

using namespace rc;

struct rc_ctx {
  int nV = 0, nE = 0;
  double alpha = 0, beta = 0;
  rc_dtype dtype = RC_F64;
  hipStream_t stream = nullptr;
  Curve curve;
  Cons cons;
  // solver vectors [3 nV]
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *tmp = nullptr, *tmp2 = nullptr;
  double *diag = nullptr, *scal = nullptr, *red = nullptr, *trial = nullptr, *zmin = nullptr, *inc = nullptr;
  double *phi = nullptr, *dx = nullptr, *dEs = nullptr, *gs = nullptr;
  // multigrid
  std::vector<std::unique_ptr<Level>> levels;  // levels[0] unused placeholder (uses curve)
  std::vector<MGLevelState> mg;
  double *coarse_inv = nullptr;
  int coarse_n = 0;
  bool mg_built = false, mg_prepared = false;
  int mg_min = 0, cheb_deg = 0;
  // dense direct path
  double *Ad = nullptr, *Cd = nullptr, *CtC = nullptr, *H = nullptr, *W = nullptr, *Sd = nullptr, *Sdinv = nullptr,
         *dtmp = nullptr;
  int* dinfo = nullptr;
  bool dense_prepared = false;
  int last_iters = 0, last_restarts = 0;
  double last_res = 0.0;
};

namespace rc {

// ---------------------------------------------------------------------------
// small host helpers
// ---------------------------------------------------------------------------
static rc_status sync(rc_ctx* c) {
  RC_HIP(hipStreamSynchronize(c->stream));
  return RC_OK;
}

static rc_status fetch(rc_ctx* c, const double* dev, double* host, int n) {
  RC_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

// Gauss-Jordan inverse with partial pivoting (small border systems).
static bool invert_small(std::vector<double>& A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (!(std::fabs(A[piv * n + col]) > 0.0)) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(A[col * n + j], A[piv * n + j]);
        std::swap(I[col * n + j], I[piv * n + j]);
      }
    const double d = 1.0 / A[col * n + col];
    for (int j = 0; j < n; ++j) {
      A[col * n + j] *= d;
      I[col * n + j] *= d;
    }
    for (int r = 0; r < n; ++r)
      if (r != col) {
        const double f = A[r * n + col];
        if (f == 0.0) continue;
        for (int j = 0; j < n; ++j) {
          A[r * n + j] -= f * A[col * n + j];
          I[r * n + j] -= f * I[col * n + j];
        }
      }
  }
  A = I;
  return true;
}

// ---------------------------------------------------------------------------
// constraints
// ---------------------------------------------------------------------------
static void cons_free(Cons& k) {
  void* ptrs[] = {k.path_edge, k.path_prev, k.cut_edge, k.edge_path_row, k.x0, k.len0, k.ones, k.geo,
                  k.geo_eval, k.vals, k.rows, k.ta, k.td, k.tc, k.Kpb, k.Z, k.Sinv, k.tri_scratch,
                  k.wp, k.yp, k.wb, k.yb, k.dots, k.rhs, k.small};
  for (void* p : ptrs)
    if (p) hipFree(p);
  k = Cons();
}

// Prepare C(gamma), the tridiagonal path block, the border Schur complement.
static rc_status cons_prepare(rc_ctx* c, const double* gamma) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nV = c->nV, nE = c->nE;
  cons_geometry(gamma, c->curve.edges, nE, k.geo, s);
  cons_border_rows(k.geo, c->curve.inc_off, c->curve.inc, c->curve.edges, k.x0, nV, k.bary, k.total,
                   k.cut_edge, k.ncut, k.rows, k.nb, s);
  const int nb = k.nb, np = k.np;
  std::vector<double> S(nb * nb, 0.0);
  if (nb > 0) {
    // Kbb: Gram matrix of the border rows
    for (int r = 0; r < nb; ++r)
      vec_dots(k.rows, 3 * nV, k.rows + (size_t)r * 3 * nV, 0, 3 * nV, nb, c->red, k.dots + r * nb, s);
    if (np > 0) {
      cons_path_coeffs(k.geo, c->curve.edges, k.path_edge, k.path_prev, np, k.ta, k.td, k.tc, s);
      cons_path_apply(k.geo, c->curve.edges, k.path_edge, np, k.rows, nV, nb, k.Kpb, s);
      for (int r = 0; r < nb; ++r)
        tridiag_solve(k.ta, k.td, k.tc, k.Kpb + (size_t)r * np, k.Z + (size_t)r * np, np, k.tri_scratch, s);
      for (int r = 0; r < nb; ++r)
        vec_dots(k.Kpb, np, k.Z + (size_t)r * np, 0, np, nb, c->red, k.small + r * nb, s);
    }
    std::vector<double> kbb(nb * nb), kz(nb * nb, 0.0);
    RC_TRY(fetch(c, k.dots, kbb.data(), nb * nb));
    if (np > 0) RC_TRY(fetch(c, k.small, kz.data(), nb * nb));
    for (int i = 0; i < nb * nb; ++i) S[i] = kbb[i] - kz[i];
    if (!invert_small(S, nb)) {
      set_error("constraint Schur complement is singular (dependent constraints?)");
      return RC_ERR_SINGULAR;
    }
    RC_HIP(hipMemcpyAsync(k.Sinv, S.data(), sizeof(double) * nb * nb, hipMemcpyHostToDevice, s));
  } else if (np > 0) {
    cons_path_coeffs(k.geo, c->curve.edges, k.path_edge, k.path_prev, np, k.ta, k.td, k.tc, s);
  }
  RC_TRY(sync(c));
  k.prepared = true;
  return RC_OK;
}

// Given (wp, wb) on device, solve C C^T y = w in place: yp, yb.
static void cons_solve_K(rc_ctx* c) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  if (k.np > 0) tridiag_solve(k.ta, k.td, k.tc, k.wp, k.yp, k.np, k.tri_scratch, s);
  if (k.nb > 0) {
    if (k.np > 0) vec_dots(k.Kpb, k.np, k.yp, 0, k.np, k.nb, c->red, k.dots, s);
    else hipMemsetAsync(k.dots, 0, sizeof(double) * k.nb, s);
    cons_border_solve(k.Sinv, k.wb, k.dots, k.rhs, k.nb, k.yb, s);
    cons_sub_Zy(k.Z, k.yb, k.nb, k.np, k.yp, s);
  }
}

// out = P in (in may equal out).  No-op copy when there are no constraints.
static void cons_project(rc_ctx* c, const double* in, double* out) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nV = c->nV;
  if (k.k == 0) {
    if (in != out) vec_copy(in, out, 3 * nV, s);
    return;
  }
  cons_path_apply(k.geo, c->curve.edges, k.path_edge, k.np, in, nV, 1, k.wp, s);
  if (k.nb > 0) vec_dots(k.rows, 3 * nV, in, 0, 3 * nV, k.nb, c->red, k.wb, s);
  cons_solve_K(c);
  cons_apply_CT(k.geo, c->curve.inc_off, c->curve.inc, k.edge_path_row, k.yp, k.rows, k.yb, k.nb, nV, in, out, s);
}

// Map an external-order right-hand side b (bary, total, edges) to (wp, wb).
__global__ void k_map_rhs(const double* __restrict__ b, int bary, int total, const int* __restrict__ path_edge,
                          int np, const int* __restrict__ cut_edge, int ncut, double* __restrict__ wp,
                          double* __restrict__ wb, double sign) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nd = 3 * bary + total;
  if (i < np) wp[i] = sign * b[nd + path_edge[i]];
  if (i < nd) wb[i] = sign * b[i];
  if (i < ncut) wb[nd + i] = sign * b[nd + cut_edge[i]];
}

// z = C^T (C C^T)^-1 b for an external-order b (device, k values).
static void cons_min_norm(rc_ctx* c, const double* b, double* z) {
  Cons& k = c->cons;
  const int n = std::max(k.np, std::max(k.nb, 1));
  hipLaunchKernelGGL(k_map_rhs, dim3(cdiv(n, 256)), dim3(256), 0, c->stream, b, k.bary, k.total, k.path_edge,
                     k.np, k.cut_edge, k.ncut, k.wp, k.wb, -1.0);
  cons_solve_K(c);
  // apply_CT computes in - C^T y with in = null: -C^T y = C^T K^-1 b
  cons_apply_CT(k.geo, c->curve.inc_off, c->curve.inc, k.edge_path_row, k.yp, k.rows, k.yb, k.nb, c->nV, nullptr,
                z, c->stream);
}

__global__ void k_phi_border(const double* __restrict__ sm, int bary, int total, double total0,
                             double* __restrict__ phi) {
  int o = 0;
  if (bary) {
    phi[0] = sm[0];
    phi[1] = sm[1];
    phi[2] = sm[2];
    o = 3;
  }
  if (total) phi[o] = total0 - sm[3];
}

__global__ void k_negate(const double* __restrict__ in, double* __restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -in[i];
}

// Phi(gamma) in external order into phi (device, k values).
static void cons_values(rc_ctx* c, const double* gamma, double* phi) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nE = c->nE;
  cons_geometry(gamma, c->curve.edges, nE, k.geo_eval, s);
  const int nd = 3 * k.bary + k.total;
  cons_phi_edge(k.geo_eval, k.x0, nE, k.len0, k.vals, k.edge ? phi + nd : nullptr, s);
  if (nd > 0) {
    vec_dots(k.vals, nE, k.ones, 0, nE, 4, c->red, k.small, s);
    // barycenter rows: sum l (x - x0) = small[0..2]; total length: L0 - small[3]
    hipLaunchKernelGGL(k_phi_border, dim3(1), dim3(1), 0, s, k.small, k.bary, k.total, k.total0, phi);
  }
}

// ---------------------------------------------------------------------------
// operator application on the finest level
// ---------------------------------------------------------------------------
static rc_status load_geometry(rc_ctx* c, const double* gamma) {
  return launch_geometry(c->curve, gamma, RC_F32, c->stream);  // both precisions
}

static rc_status apply_A(rc_ctx* c, const Curve& cv, const double* X, double* Y, rc_dtype prec) {
  return launch_sobolev(cv, c->alpha, c->beta, prec, X, Y, nullptr, c->stream);
}

// ---------------------------------------------------------------------------
// multigrid
// ---------------------------------------------------------------------------
__global__ void k_gather_coarse(const double* __restrict__ fine, const int* __restrict__ fine_of, int nc,
                                double* __restrict__ coarse) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int f = fine_of[i];
  coarse[3 * i] = fine[3 * f];
  coarse[3 * i + 1] = fine[3 * f + 1];
  coarse[3 * i + 2] = fine[3 * f + 2];
}

// x_fine += J x_coarse: fine v gets (x_a + x_b)/2 (a = b for kept vertices)
__global__ void k_prolong_add(const int2* __restrict__ pr, int nf, const double* __restrict__ xc,
                              double* __restrict__ xf) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nf) return;
  int2 ab = pr[v];
  for (int k = 0; k < 3; ++k) xf[3 * v + k] += 0.5 * (xc[3 * ab.x + k] + xc[3 * ab.y + k]);
}

// b_coarse = J^T r_fine
__global__ void k_restrict(const int* __restrict__ off, const int* __restrict__ idx, const int2* __restrict__ pr,
                           int nc, const double* __restrict__ rf, double* __restrict__ bc) {
  int cidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (cidx >= nc) return;
  double s[3] = {0, 0, 0};
  for (int k = off[cidx]; k < off[cidx + 1]; ++k) {
    int v = idx[k];
    int2 ab = pr[v];
    double w = 0.5 * ((ab.x == cidx) + (ab.y == cidx));
    for (int d = 0; d < 3; ++d) s[d] += w * rf[3 * v + d];
  }
  for (int d = 0; d < 3; ++d) bc[3 * cidx + d] = s[d];
}

// Chebyshev helpers: d = D^-1 r / theta ; x += d ; etc.
__global__ void k_cheb_init(const double* __restrict__ r, const double* __restrict__ dg, double inv_theta, int nV,
                            double* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * nV) d[i] = inv_theta * r[i] / dg[i / 3];
}

__global__ void k_cheb_update(const double* __restrict__ r, const double* __restrict__ dg, double c1, double c2,
                              int nV, double* __restrict__ d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * nV) d[i] = c1 * d[i] + c2 * r[i] / dg[i / 3];
}

__global__ void k_add_ones_outer(double* __restrict__ A, int n, double rho) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) A[i] += rho;
}

__global__ void k_identity(double* __restrict__ A, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) A[i] = (i / n == i % n) ? 1.0 : 0.0;
}

__global__ void k_fill_pattern(double* __restrict__ x, int n, unsigned seed) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned h = (unsigned)i * 2654435761u ^ seed;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  x[i] = (double)(h & 0xffffff) / 16777216.0 - 0.5;
}

static const Curve& level_curve(rc_ctx* c, int l) { return l == 0 ? c->curve : c->levels[l]->curve; }

static rc_status mg_build(rc_ctx* c) {
  if (c->mg_built) return RC_OK;
  if (!c->curve.chain) {
    set_error("multigrid needs every vertex to have degree <= 2");
    return RC_ERR_UNSUPPORTED;
  }
  c->levels.clear();
  c->levels.emplace_back(nullptr);
  const Curve* fine = &c->curve;
  while (fine->nV > c->mg_min) {
    std::vector<Chain> chs = chains_of(*fine);
    // coarse vertices: even chain positions; path ends stay
    std::vector<int> coarse_id(fine->nV, -1);
    std::vector<int> fine_of;
    std::vector<int> cedges;
    std::vector<int2> prolong(fine->nV, make_int2(-1, -1));
    bool ok = true;
    for (const Chain& ch : chs) {
      const int m = (int)ch.verts.size();
      if (ch.loop && m < 12) { ok = false; break; }
      std::vector<int> keep;
      for (int i = 0; i < m; ++i)
        if (i % 2 == 0 || (!ch.loop && i == m - 1)) keep.push_back(i);
      for (int i : keep) {
        coarse_id[ch.verts[i]] = (int)fine_of.size();
        fine_of.push_back(ch.verts[i]);
      }
      const int nk = (int)keep.size();
      for (int q = 0; q + 1 < nk || (ch.loop && q < nk); ++q) {
        int a = coarse_id[ch.verts[keep[q]]], b = coarse_id[ch.verts[keep[(q + 1) % nk]]];
        cedges.push_back(a);
        cedges.push_back(b);
      }
      for (int q = 0; q < nk; ++q) {
        const int i0 = keep[q];
        const int i1 = (q + 1 < nk) ? keep[q + 1] : (ch.loop ? keep[0] + m : -1);
        prolong[ch.verts[i0]] = make_int2(coarse_id[ch.verts[i0]], coarse_id[ch.verts[i0]]);
        if (i1 < 0) continue;
        for (int i = i0 + 1; i < i1; ++i)
          prolong[ch.verts[i % m]] = make_int2(coarse_id[ch.verts[i0]], coarse_id[ch.verts[i1 % m]]);
      }
    }
    for (int v = 0; v < fine->nV; ++v)
      if (prolong[v].x < 0) ok = false;  // isolated vertices are not coarsened
    if (!ok || fine_of.size() == (size_t)fine->nV) break;
    auto L = std::make_unique<Level>();
    const int nc = (int)fine_of.size();
    RC_TRY(L->curve.init(nc, (int)cedges.size() / 2, cedges.data()));
    L->h_fine_of = fine_of;
    RC_TRY(dalloc(&L->fine_of, nc));
    RC_TRY(dalloc(&L->prolong, fine->nV));
    RC_TRY(dalloc(&L->gamma, 3 * (size_t)nc));
    RC_HIP(hipMemcpy(L->fine_of, fine_of.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(L->prolong, prolong.data(), sizeof(int2) * fine->nV, hipMemcpyHostToDevice));
    std::vector<int> off(nc + 1, 0), idx;
    std::vector<std::vector<int>> lists(nc);
    for (int v = 0; v < fine->nV; ++v) {
      lists[prolong[v].x].push_back(v);
      if (prolong[v].y != prolong[v].x) lists[prolong[v].y].push_back(v);
    }
    for (int i = 0; i < nc; ++i) {
      off[i + 1] = off[i] + (int)lists[i].size();
      idx.insert(idx.end(), lists[i].begin(), lists[i].end());
    }
    RC_TRY(dalloc(&L->restr_off, nc + 1));
    RC_TRY(dalloc(&L->restr_idx, idx.size()));
    RC_HIP(hipMemcpy(L->restr_off, off.data(), sizeof(int) * (nc + 1), hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(L->restr_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
    c->levels.push_back(std::move(L));
    fine = &c->levels.back()->curve;
  }
  const int nl = (int)c->levels.size();
  c->mg.assign(nl, MGLevelState());
  for (int l = 0; l < nl; ++l) {
    const int n = level_curve(c, l).nV;
    MGLevelState& st = c->mg[l];
    RC_TRY(dalloc(&st.diag, n));
    RC_TRY(dalloc(&st.x, 3 * (size_t)n));
    RC_TRY(dalloc(&st.b, 3 * (size_t)n));
    RC_TRY(dalloc(&st.r, 3 * (size_t)n));
    RC_TRY(dalloc(&st.d, 3 * (size_t)n));
    RC_TRY(dalloc(&st.t, 3 * (size_t)n));
    RC_TRY(dalloc(&st.pw, 3 * (size_t)n));
    hipLaunchKernelGGL(k_fill_pattern, dim3(cdiv(3 * n, 256)), dim3(256), 0, c->stream, st.pw, 3 * n, 12345u + l);
  }
  c->coarse_n = level_curve(c, nl - 1).nV;
  RC_TRY(dalloc(&c->coarse_inv, (size_t)c->coarse_n * c->coarse_n));
  c->mg_built = true;
  return RC_OK;
}

static rc_status mg_prepare(rc_ctx* c, const double* gamma) {
  RC_TRY(mg_build(c));
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  const double* g = gamma;
  for (int l = 1; l < nl; ++l) {
    Level& L = *c->levels[l];
    hipLaunchKernelGGL(k_gather_coarse, dim3(cdiv(L.curve.nV, 256)), dim3(256), 0, s, g, L.fine_of, L.curve.nV,
                       L.gamma);
    g = L.gamma;
    RC_TRY(launch_geometry(L.curve, L.gamma, RC_F32, s));
  }
  const rc_dtype prec = c->dtype;
  for (int l = 0; l < nl - 1; ++l) {
    const Curve& cv = level_curve(c, l);
    MGLevelState& st = c->mg[l];
    const int n = cv.nV;
    // diagonal (any input vector; the output Y is scratch)
    RC_TRY(launch_sobolev(cv, c->alpha, c->beta, prec, st.pw, st.t, st.diag, s));
    // lambda_max of D^-1 A by power iteration, warm-started from the
    // previous call's vector (the geometry changes little between steps)
    double nrm = 0.0;
    for (int it = 0; it < 8; ++it) {
      RC_TRY(launch_sobolev(cv, c->alpha, c->beta, prec, st.pw, st.t, nullptr, s));
      vec_scale_diag_inv(st.t, st.diag, st.d, n, s);
      vec_dot(st.d, st.d, 3 * n, c->red, c->scal, s);
      double h;
      RC_TRY(fetch(c, c->scal, &h, 1));
      nrm = std::sqrt(h);
      if (!(nrm > 0)) {
        set_error("multigrid setup: zero operator");
        return RC_ERR_SINGULAR;
      }
      vec_axpby(1.0 / nrm, st.d, 0.0, st.pw, 3 * n, s);
    }
    st.lmax = 1.1 * nrm;
  }
  // coarsest: dense FP64 (A_c + rho 1 1^T)^-1
  {
    const Curve& cv = level_curve(c, nl - 1);
    const int n = cv.nV;
    RC_TRY(launch_geometry(cv, nl == 1 ? gamma : c->levels[nl - 1]->gamma, RC_F32, s));
    double* Ac = c->coarse_inv;
    RC_TRY(launch_assemble_dense(cv, c->alpha, c->beta, Ac, s));
    // rho = trace / n^2
    std::vector<double> diag(n);
    std::vector<double> Ah((size_t)n * n);
    RC_HIP(hipMemcpyAsync(Ah.data(), Ac, sizeof(double) * n * n, hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += Ah[(size_t)i * n + i];
    hipLaunchKernelGGL(k_add_ones_outer, dim3(cdiv(n * n, 256)), dim3(256), 0, s, Ac, n, tr / ((double)n * n));
    dense_cholesky(Ac, n, c->dinfo, s);
    int info = 0;
    RC_HIP(hipMemcpyAsync(&info, c->dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    if (info != 0) {
      set_error("multigrid coarse factorisation failed");
      return RC_ERR_SINGULAR;
    }
    // explicit inverse: solve with the identity
    double* Inv;
    RC_TRY(dalloc(&Inv, (size_t)n * n));
    hipLaunchKernelGGL(k_identity, dim3(cdiv(n * n, 256)), dim3(256), 0, s, Inv, n);
    dense_chol_solve(Ac, Inv, n, n, s);
    RC_HIP(hipMemcpyAsync(Ac, Inv, sizeof(double) * n * n, hipMemcpyDeviceToDevice, s));
    RC_TRY(sync(c));
    hipFree(Inv);
  }
  c->mg_prepared = true;
  return RC_OK;
}

// Chebyshev smoothing of A_l x = b on level l (3 components), deg steps.
// x_zero: x starts at 0 (no initial product).
static rc_status cheb_smooth(rc_ctx* c, int l, double* x, const double* b, bool x_zero) {
  const Curve& cv = level_curve(c, l);
  MGLevelState& st = c->mg[l];
  hipStream_t s = c->stream;
  const int n = cv.nV, n3 = 3 * n;
  const double lmax = st.lmax, lmin = 0.2 * lmax;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (x_zero) {
    vec_copy(b, st.r, n3, s);
    hipMemsetAsync(x, 0, sizeof(double) * n3, s);
  } else {
    RC_TRY(apply_A(c, cv, x, st.r, c->dtype));
    vec_axpby(1.0, b, -1.0, st.r, n3, s);
  }
  hipLaunchKernelGGL(k_cheb_init, dim3(cdiv(n3, 256)), dim3(256), 0, s, st.r, st.diag, 1.0 / theta, n, st.d);
  const int deg = c->cheb_deg;
  for (int k = 0; k < deg; ++k) {
    vec_axpby(1.0, st.d, 1.0, x, n3, s);
    if (k == deg - 1) break;
    RC_TRY(apply_A(c, cv, st.d, st.t, c->dtype));
    vec_axpby(-1.0, st.t, 1.0, st.r, n3, s);
    const double rn = 1.0 / (2.0 * sigma - rho);
    hipLaunchKernelGGL(k_cheb_update, dim3(cdiv(n3, 256)), dim3(256), 0, s, st.r, st.diag, rn * rho, 2.0 * rn / delta,
                       n, st.d);
    rho = rn;
  }
  return RC_OK;
}

static rc_status vcycle(rc_ctx* c, int l, const double* b, double* x) {
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  if (l == nl - 1) {
    dense_gemm(c->coarse_inv, b, x, c->coarse_n, 3, c->coarse_n, 0.0, false, s);
    return RC_OK;
  }
  const Curve& cv = level_curve(c, l);
  MGLevelState& st = c->mg[l];
  const int n3 = 3 * cv.nV;
  RC_TRY(cheb_smooth(c, l, x, b, true));
  RC_TRY(apply_A(c, cv, x, st.t, c->dtype));
  vec_axpby(1.0, b, -1.0, st.t, n3, s);  // t = b - A x
  Level& C = *c->levels[l + 1];
  MGLevelState& sc = c->mg[l + 1];
  hipLaunchKernelGGL(k_restrict, dim3(cdiv(C.curve.nV, 256)), dim3(256), 0, s, C.restr_off, C.restr_idx, C.prolong,
                     C.curve.nV, st.t, sc.b);
  RC_TRY(vcycle(c, l + 1, sc.b, sc.x));
  hipLaunchKernelGGL(k_prolong_add, dim3(cdiv(cv.nV, 256)), dim3(256), 0, s, C.prolong, cv.nV, sc.x, x);
  RC_TRY(cheb_smooth(c, l, x, b, false));
  return RC_OK;
}

// ---------------------------------------------------------------------------
// projected PCG:  P Abar P y = P b, y in range(P)
// ---------------------------------------------------------------------------
static rc_status precondition(rc_ctx* c, int kind, const double* r, double* z) {
  if (kind == RC_SOLVE_PCG_MG) {
    MGLevelState& st = c->mg[0];
    vec_copy(r, st.b, 3 * c->nV, c->stream);
    RC_TRY(vcycle(c, 0, st.b, z));
  } else {
    vec_scale_diag_inv(r, c->diag, z, c->nV, c->stream);
  }
  cons_project(c, z, z);
  return RC_OK;
}

static rc_status pcg_solve(rc_ctx* c, const double* b, double* x, const rc_solve_opts& o, int* iters_out,
                           double* res_out) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV;
  const rc_dtype op = o.op_f64 ? RC_F64 : c->dtype;
  double* r = c->r;
  double* z = c->z;
  double* p = c->p;
  double* q = c->q;
  cons_project(c, b, c->tmp2);  // P b
  vec_dot(c->tmp2, c->tmp2, n3, c->red, c->scal, s);
  double bb;
  RC_TRY(fetch(c, c->scal, &bb, 1));
  const double bn = std::sqrt(bb);
  hipMemsetAsync(x, 0, sizeof(double) * n3, s);
  if (!(bn > 0)) {
    *iters_out = 0;
    *res_out = 0.0;
    return RC_OK;
  }
  vec_copy(c->tmp2, r, n3, s);
  int it = 0;
  double res = 1.0;
  bool converged = false;
  while (it < o.max_iter && !converged) {
    RC_TRY(precondition(c, o.solver, r, z));
    vec_copy(z, p, n3, s);
    vec_dot(r, z, n3, c->red, c->scal, s);
    double rz;
    RC_TRY(fetch(c, c->scal, &rz, 1));
    int since = 0;
    while (it < o.max_iter) {
      RC_TRY(apply_A(c, c->curve, p, q, op));
      cons_project(c, q, q);
      vec_dot(p, q, n3, c->red, c->scal, s);
      double pq;
      RC_TRY(fetch(c, c->scal, &pq, 1));
      if (!(pq > 0)) break;
      const double al = rz / pq;
      vec_axpby(al, p, 1.0, x, n3, s);
      vec_axpby(-al, q, 1.0, r, n3, s);
      ++it;
      ++since;
      vec_dot(r, r, n3, c->red, c->scal, s);
      double rr;
      RC_TRY(fetch(c, c->scal, &rr, 1));
      res = std::sqrt(rr) / bn;
      const bool check = res < o.tol || (o.replace_every > 0 && since >= o.replace_every);
      if (check) {
        // FP64 true residual r = P (b - Abar x)
        RC_TRY(apply_A(c, c->curve, x, c->tmp, RC_F64));
        vec_copy(b, r, n3, s);
        vec_axpby(-1.0, c->tmp, 1.0, r, n3, s);
        cons_project(c, r, r);
        vec_dot(r, r, n3, c->red, c->scal, s);
        RC_TRY(fetch(c, c->scal, &rr, 1));
        res = std::sqrt(rr) / bn;
        if (res < o.tol) converged = true;
        break;  // restart the recurrence from the true residual
      }
      RC_TRY(precondition(c, o.solver, r, z));
      vec_dot(r, z, n3, c->red, c->scal, s);
      double rzn;
      RC_TRY(fetch(c, c->scal, &rzn, 1));
      vec_axpby(1.0, z, rzn / rz, p, n3, s);
      rz = rzn;
    }
    if (since == 0) break;
  }
  *iters_out = it;
  *res_out = res;
  if (!converged) {
    set_error("projected PCG did not reach the tolerance");
    return RC_ERR_NOT_CONVERGED;
  }
  return RC_OK;
}

// ---------------------------------------------------------------------------
// dense direct path (eq. GradientSaddlePointProblem): H = Abar + C^T C,
// W = H^-1 C^T, S = C W; g = H^-1 dE - W S^-1 W^T dE;  x = -W S^-1 Phi
// ---------------------------------------------------------------------------
static rc_status dense_prepare(rc_ctx* c, const double* gamma) {
  hipStream_t s = c->stream;
  const int nV = c->nV, n = 3 * nV, k = c->cons.k;
  if (nV > 2048) {
    set_error("dense solver limited to 2048 vertices");
    return RC_ERR_UNSUPPORTED;
  }
  if (!c->Ad) {
    RC_TRY(dalloc(&c->Ad, (size_t)nV * nV));
    RC_TRY(dalloc(&c->H, (size_t)n * n));
    RC_TRY(dalloc(&c->CtC, (size_t)n * n));
  }
  if (c->Cd) {
    hipFree(c->Cd);
    hipFree(c->W);
    hipFree(c->Sd);
    hipFree(c->Sdinv);
    hipFree(c->dtmp);
  }
  RC_TRY(dalloc(&c->Cd, (size_t)std::max(k, 1) * n));
  RC_TRY(dalloc(&c->W, (size_t)n * std::max(k, 1)));
  RC_TRY(dalloc(&c->Sd, (size_t)std::max(k * k, 1)));
  RC_TRY(dalloc(&c->Sdinv, (size_t)std::max(k * k, 1)));
  RC_TRY(dalloc(&c->dtmp, (size_t)std::max(k, 1) + n));
  RC_TRY(load_geometry(c, gamma));
  RC_TRY(launch_assemble_dense(c->curve, c->alpha, c->beta, c->Ad, s));
  if (k > 0) {
    // dense C in external order: border rows first (bary, total), then edges
    Cons& K = c->cons;
    const int nd = 3 * K.bary + K.total;
    RC_HIP(hipMemsetAsync(c->Cd, 0, sizeof(double) * (size_t)k * n, s));
    if (nd > 0) RC_HIP(hipMemcpyAsync(c->Cd, K.rows, sizeof(double) * (size_t)nd * n, hipMemcpyDeviceToDevice, s));
    if (K.edge) dense_C_edges(K.geo, c->curve.edges, c->nE, nd, nV, c->Cd, s);
    dense_gemm(c->Cd, c->Cd, c->CtC, n, n, k, 0.0, true, s);
  } else {
    RC_HIP(hipMemsetAsync(c->CtC, 0, sizeof(double) * (size_t)n * n, s));
  }
  dense_build_H(c->Ad, c->CtC, nV, c->H, s);
  dense_cholesky(c->H, n, c->dinfo, s);
  int info = 0;
  RC_HIP(hipMemcpyAsync(&info, c->dinfo, sizeof(int), hipMemcpyDeviceToHost, s));
  RC_TRY(sync(c));
  if (info != 0) {
    set_error("Cholesky of Abar + C^T C failed: Abar is not definite on null(C)");
    return RC_ERR_SINGULAR;
  }
  if (k > 0) {
    // W = H^-1 C^T  (C^T as n x k: transpose via gemm with the identity)
    double* Ik;
    RC_TRY(dalloc(&Ik, (size_t)k * k));
    hipLaunchKernelGGL(k_identity, dim3(cdiv(k * k, 256)), dim3(256), 0, s, Ik, k);
    dense_gemm(c->Cd, Ik, c->W, n, k, k, 0.0, true, s);
    dense_chol_solve(c->H, c->W, n, k, s);
    dense_gemm(c->Cd, c->W, c->Sd, k, k, n, 0.0, false, s);
    std::vector<double> S((size_t)k * k);
    RC_HIP(hipMemcpyAsync(S.data(), c->Sd, sizeof(double) * k * k, hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    hipFree(Ik);
    if (!invert_small(S, k)) {
      set_error("constraint Schur complement is singular");
      return RC_ERR_SINGULAR;
    }
    RC_HIP(hipMemcpyAsync(c->Sdinv, S.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, s));
  }
  RC_TRY(sync(c));
  c->dense_prepared = true;
  return RC_OK;
}

static rc_status dense_gradient(rc_ctx* c, const double* dE, double* g) {
  hipStream_t s = c->stream;
  const int n = 3 * c->nV, k = c->cons.k;
  vec_copy(dE, g, n, s);
  dense_chol_solve(c->H, g, n, 1, s);  // u = H^-1 dE
  if (k > 0) {
    double* t1 = c->dtmp;  // k
    double* t2 = c->dtmp + k;
    dense_gemm(c->Cd, g, t1, k, 1, n, 0.0, false, s);     // C u
    dense_gemm(c->Sdinv, t1, t2, k, 1, k, 0.0, false, s);  // lambda
    dense_gemm(c->W, t2, c->tmp, n, 1, k, 0.0, false, s);  // W lambda
    vec_axpby(-1.0, c->tmp, 1.0, g, n, s);
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

rc_solve_opts resolve(const rc_solve_opts* o) {
  rc_solve_opts d;
  rc_default_solve_opts(&d);
  if (o) d = *o;
  if (d.max_iter <= 0) d.max_iter = 500;
  if (!(d.tol > 0)) d.tol = 1e-6;
  if (d.mg_min_vertices <= 0) d.mg_min_vertices = 512;
  if (d.cheb_degree <= 0) d.cheb_degree = 2;
  return d;
}

rc_ls_opts resolve_ls(const rc_ls_opts* o) {
  rc_ls_opts d;
  rc_default_ls_opts(&d);
  if (o) d = *o;
  return d;
}

// Everything a gradient solve and the projections at gamma need.
rc_status prepare_solver(rc_ctx* c, const double* gamma, const rc_solve_opts& o) {
  RC_TRY(load_geometry(c, gamma));
  if (c->cons.k > 0) RC_TRY(cons_prepare(c, gamma));
  if (o.solver == RC_SOLVE_DENSE) return dense_prepare(c, gamma);
  if (o.solver == RC_SOLVE_PCG_MG) {
    if (c->mg_min != o.mg_min_vertices) {
      c->mg_built = false;
      c->mg_min = o.mg_min_vertices;
    }
    c->cheb_deg = o.cheb_degree;
    RC_TRY(mg_prepare(c, gamma));
    RC_TRY(load_geometry(c, gamma));
  } else {
    RC_TRY(launch_sobolev(c->curve, c->alpha, c->beta, c->dtype, c->x, c->tmp, c->diag, c->stream));
  }
  return RC_OK;
}

// Gradient solve at the prepared gamma.
rc_status solve_prepared(rc_ctx* c, const double* rhs, double* out, const rc_solve_opts& o, int* iters,
                         double* res) {
  if (o.solver == RC_SOLVE_DENSE) {
    RC_TRY(dense_gradient(c, rhs, out));
    *iters = 0;
    *res = 0.0;
    return sync(c);
  }
  return pcg_solve(c, rhs, out, o, iters, res);
}

// Projection increment x for the constraint violation phi (external order):
// eq. ConstraintSaddlePointProblem, via eq. SaddleSolutionTransformation on
// the PCG paths.
rc_status projection_increment(rc_ctx* c, const double* phi, double* x, const rc_solve_opts& o, int* iters) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV, k = c->cons.k;
  *iters = 0;
  if (o.solver == RC_SOLVE_DENSE) {
    double* t1 = c->dtmp;
    dense_gemm(c->Sdinv, phi, t1, k, 1, k, 0.0, false, s);
    dense_gemm(c->W, t1, x, n3, 1, k, 0.0, false, s);
    vec_axpby(0.0, x, -1.0, x, n3, s);  // x = -W S^-1 phi
    return RC_OK;
  }
  // z = C^T (C C^T)^-1 (-phi): the minimum-norm correction; then x = z - y with
  // y solving the projected system for the right-hand side Abar z
  hipLaunchKernelGGL(k_negate, dim3(cdiv(k, 256)), dim3(256), 0, s, phi, c->phi + k, k);
  cons_min_norm(c, c->phi + k, c->zmin);
  RC_TRY(apply_A(c, c->curve, c->zmin, c->inc, RC_F64));
  double res = 0.0;
  rc_status st = pcg_solve(c, c->inc, c->x, o, iters, &res);
  if (st != RC_OK && st != RC_ERR_NOT_CONVERGED) return st;
  vec_copy(c->zmin, x, n3, s);
  vec_axpby(-1.0, c->x, 1.0, x, n3, s);
  return RC_OK;
}

struct LsResult {
  double tau = 0.0, E1 = 0.0;
  int backtracks = 0, proj_iters = 0, proj_solve_iters = 0;
};

rc_status line_search(rc_ctx* c, double* gamma, double E0, const double* dE, const double* g, const rc_ls_opts& ls,
                      const rc_solve_opts& so, LsResult* out) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV, k = c->cons.k;
  // scal[16] keeps |g|^2 for the trial points; the solvers use scal[0..15]
  vec_dot(g, g, n3, c->red, c->scal + 16, s);
  vec_dot(dE, g, n3, c->red, c->scal + 17, s);
  double h[2];
  RC_TRY(fetch(c, c->scal + 16, h, 2));
  if (!(h[0] > 0)) {
    set_error("zero gradient");
    return RC_ERR_LINESEARCH;
  }
  const double slope = h[1] / std::sqrt(h[0]);
  // per-row projection tolerances (relative to the mean edge length at gamma)
  std::vector<double> phi_h(std::max(k, 1));
  double lbar = 0.0, Ltot = 0.0;
  if (k > 0) {
    cons_values(c, gamma, c->phi);
    RC_TRY(sync(c));
  }
  {
    // mean edge length from the FP64 geometry of gamma
    std::vector<double> ga(4 * (size_t)c->nE);
    RC_TRY(load_geometry(c, gamma));
    RC_HIP(hipMemcpyAsync(ga.data(), c->curve.gd.a, sizeof(double) * 4 * c->nE, hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    for (int I = 0; I < c->nE; ++I) Ltot += ga[4 * I + 3];
    lbar = Ltot / std::max(1, c->nE);
  }
  const Cons& K = c->cons;
  const int nd = 3 * K.bary + K.total;
  double tau = ls.tau0;
  for (int bt = 0; bt <= ls.max_backtracks; ++bt) {
    vec_trial(gamma, g, c->scal + 16, tau, c->trial, n3, s);
    bool ok = (k == 0);
    int it = 0;
    for (; k > 0 && it <= ls.max_proj_iter; ++it) {
      cons_values(c, c->trial, c->phi);
      RC_TRY(fetch(c, c->phi, phi_h.data(), k));
      bool done = true;
      for (int i = 0; i < k; ++i) {
        double tol = ls.proj_tol * lbar;
        if (K.bary && i < 3) tol *= Ltot;
        if (!std::isfinite(phi_h[i]) || std::fabs(phi_h[i]) > tol) done = false;
      }
      (void)nd;
      if (done) {
        ok = true;
        break;
      }
      if (it == ls.max_proj_iter) break;
      int pit = 0;
      RC_TRY(load_geometry(c, gamma));
      RC_TRY(projection_increment(c, c->phi, c->dx, so, &pit));
      out->proj_solve_iters += pit;
      vec_axpby(1.0, c->dx, 1.0, c->trial, n3, s);
    }
    if (ok) {
      RC_TRY(load_geometry(c, c->trial));
      RC_TRY(launch_tpe(c->curve, c->alpha, c->beta, c->dtype, false, c->scal + 18, nullptr, s));
      double E1;
      RC_TRY(fetch(c, c->scal + 18, &E1, 1));
      if (std::isfinite(E1) && E1 <= E0 - ls.c_armijo * tau * slope) {
        vec_copy(c->trial, gamma, n3, s);
        RC_TRY(sync(c));
        out->tau = tau;
        out->E1 = E1;
        out->backtracks = bt;
        out->proj_iters = it;
        return RC_OK;
      }
    }
    tau *= ls.shrink;
  }
  set_error("line search found no admissible step");
  out->backtracks = ls.max_backtracks;
  return RC_ERR_LINESEARCH;
}

}  // namespace

extern "C" {

void rc_default_solve_opts(rc_solve_opts* o) {
  if (!o) return;
  o->solver = RC_SOLVE_PCG_MG;
  o->tol = 1e-6;
  o->max_iter = 500;
  o->replace_every = 0;
  o->mg_min_vertices = 512;
  o->cheb_degree = 2;
  o->op_f64 = 0;
}

void rc_default_ls_opts(rc_ls_opts* o) {
  if (!o) return;
  o->c_armijo = 0.01;
  o->shrink = 0.5;
  o->tau0 = 1.0;
  o->max_backtracks = 30;
  o->max_proj_iter = 10;
  o->proj_tol = 1e-10;
}

const char* rc_last_error(void) { return rc::last_error(); }

rc_status rc_create(int32_t nV, int32_t nE, const int32_t* edges_h, double alpha, double beta, rc_dtype dtype,
                    rc_stream stream, rc_ctx** out) {
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
  const size_t n3 = 3 * (size_t)nV;
  double** vecs[] = {&c->x,    &c->r,    &c->z,   &c->p,  &c->q,   &c->tmp, &c->tmp2,
                     &c->trial, &c->zmin, &c->inc, &c->dx, &c->dEs, &c->gs};
  for (double** v : vecs) RC_TRY(dalloc(v, n3));
  RC_TRY(dalloc(&c->diag, nV));
  RC_TRY(dalloc(&c->scal, 64));
  RC_TRY(dalloc(&c->red, (size_t)dot_scratch_size(128)));
  RC_TRY(dalloc(&c->phi, 2 * ((size_t)nE + 4)));
  RC_TRY(dalloc(&c->dinfo, 1));
  RC_HIP(hipMemsetAsync(c->x, 0, sizeof(double) * n3, c->stream));
  RC_TRY(sync(c.get()));
  *out = c.release();
  return RC_OK;
}

rc_status rc_destroy(rc_ctx* c) {
  if (!c) return RC_OK;
  hipStreamSynchronize(c->stream);
  c->curve.release();
  cons_free(c->cons);
  for (auto& L : c->levels)
    if (L) {
      L->curve.release();
      hipFree(L->fine_of);
      hipFree(L->prolong);
      hipFree(L->restr_off);
      hipFree(L->restr_idx);
      hipFree(L->gamma);
    }
  for (auto& st : c->mg) {
    double* ps[] = {st.diag, st.x, st.b, st.r, st.d, st.t, st.pw};
    for (double* p : ps) hipFree(p);
  }
  double* ps[] = {c->x, c->r, c->z, c->p, c->q, c->tmp, c->tmp2, c->diag, c->scal, c->red, c->trial,
                  c->zmin, c->inc, c->phi, c->dx, c->dEs, c->gs, c->coarse_inv, c->Ad, c->Cd, c->CtC, c->H, c->W, c->Sd,
                  c->Sdinv, c->dtmp};
  for (double* p : ps)
    if (p) hipFree(p);
  if (c->dinfo) hipFree(c->dinfo);
  delete c;
  return RC_OK;
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
  RC_TRY(check_ptrs({gamma, A}));
  RC_TRY(launch_geometry(c->curve, gamma, RC_F32, c->stream));
  return launch_assemble_dense(c->curve, c->alpha, c->beta, A, c->stream);
}

rc_status rc_set_constraints(rc_ctx* c, uint32_t mask, const double* gamma_ref, const double* x0_h,
                             double total_len0, const double* edge_len0) {
  RC_TRY(check_ctx(c));
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
  if ((mask & RC_C_EDGE_LENGTH) && !c->curve.chain) {
    set_error("edge-length constraints need every vertex to have degree <= 2");
    return RC_ERR_UNSUPPORTED;
  }
  RC_TRY(sync(c));
  cons_free(c->cons);
  Cons& k = c->cons;
  k.mask = mask;
  k.bary = (mask & RC_C_BARYCENTER) ? 1 : 0;
  k.total = (mask & RC_C_TOTAL_LENGTH) ? 1 : 0;
  k.edge = (mask & RC_C_EDGE_LENGTH) ? 1 : 0;
  const int nV = c->nV, nE = c->nE;
  k.h_edge_path_row.assign(nE, -1);
  if (k.edge) {
    for (const Chain& ch : chains_of(c->curve)) {
      const int m = (int)ch.edges.size();
      for (int q = 0; q < m; ++q) {
        if (ch.loop && q == 0) {
          k.h_cut_edge.push_back(ch.edges[0]);
          continue;
        }
        k.h_edge_path_row[ch.edges[q]] = (int)k.h_path_edge.size();
        const bool has_prev = ch.loop ? q > 1 : q > 0;
        k.h_path_prev.push_back(has_prev ? 1 : 0);
        k.h_path_edge.push_back(ch.edges[q]);
      }
    }
  }
  k.np = (int)k.h_path_edge.size();
  k.ncut = (int)k.h_cut_edge.size();
  k.nb = 3 * k.bary + k.total + k.ncut;
  k.k = 3 * k.bary + k.total + (k.edge ? nE : 0);
  if (k.nb > 120) {
    set_error("too many loops for edge-length constraints (at most 120 border rows)");
    return RC_ERR_UNSUPPORTED;
  }
  RC_TRY(dalloc(&k.path_edge, k.np));
  RC_TRY(dalloc(&k.path_prev, k.np));
  RC_TRY(dalloc(&k.cut_edge, k.ncut));
  RC_TRY(dalloc(&k.edge_path_row, nE));
  if (k.np) {
    RC_HIP(hipMemcpy(k.path_edge, k.h_path_edge.data(), sizeof(int) * k.np, hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(k.path_prev, k.h_path_prev.data(), sizeof(int) * k.np, hipMemcpyHostToDevice));
  }
  if (k.ncut) RC_HIP(hipMemcpy(k.cut_edge, k.h_cut_edge.data(), sizeof(int) * k.ncut, hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(k.edge_path_row, k.h_edge_path_row.data(), sizeof(int) * nE, hipMemcpyHostToDevice));
  RC_TRY(dalloc(&k.x0, 3));
  RC_TRY(dalloc(&k.len0, nE));
  RC_TRY(dalloc(&k.ones, nE));
  RC_TRY(dalloc(&k.geo, 8 * (size_t)nE));
  RC_TRY(dalloc(&k.geo_eval, 8 * (size_t)nE));
  RC_TRY(dalloc(&k.vals, 4 * (size_t)nE));
  RC_TRY(dalloc(&k.rows, (size_t)std::max(k.nb, 1) * 3 * nV));
  RC_TRY(dalloc(&k.ta, k.np));
  RC_TRY(dalloc(&k.td, k.np));
  RC_TRY(dalloc(&k.tc, k.np));
  RC_TRY(dalloc(&k.Kpb, (size_t)std::max(k.nb, 1) * std::max(k.np, 1)));
  RC_TRY(dalloc(&k.Z, (size_t)std::max(k.nb, 1) * std::max(k.np, 1)));
  RC_TRY(dalloc(&k.Sinv, (size_t)std::max(k.nb * k.nb, 1)));
  RC_TRY(dalloc(&k.tri_scratch, 4 * (size_t)std::max(k.np, 1)));
  RC_TRY(dalloc(&k.wp, k.np));
  RC_TRY(dalloc(&k.yp, k.np));
  RC_TRY(dalloc(&k.wb, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.yb, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.rhs, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.dots, (size_t)std::max(k.nb * k.nb, 4)));
  RC_TRY(dalloc(&k.small, (size_t)std::max(k.nb * k.nb, 8)));
  std::vector<double> ones(nE, 1.0);
  RC_HIP(hipMemcpy(k.ones, ones.data(), sizeof(double) * nE, hipMemcpyHostToDevice));
  if (mask == 0) return RC_OK;
  // reference values from gamma_ref
  hipStream_t s = c->stream;
  cons_geometry(gamma_ref, c->curve.edges, nE, k.geo_eval, s);
  RC_HIP(hipMemsetAsync(k.x0, 0, sizeof(double) * 3, s));
  cons_phi_edge(k.geo_eval, k.x0, nE, k.ones, k.vals, nullptr, s);
  vec_dots(k.vals, nE, k.ones, 0, nE, 4, c->red, k.small, s);
  double sums[4];
  RC_TRY(fetch(c, k.small, sums, 4));
  double x0[3] = {sums[0] / sums[3], sums[1] / sums[3], sums[2] / sums[3]};
  if (x0_h) std::memcpy(x0, x0_h, sizeof(x0));
  RC_HIP(hipMemcpy(k.x0, x0, sizeof(double) * 3, hipMemcpyHostToDevice));
  k.total0 = total_len0 >= 0 ? total_len0 : sums[3];
  if (edge_len0) {
    RC_HIP(hipMemcpyAsync(k.len0, edge_len0, sizeof(double) * nE, hipMemcpyDeviceToDevice, s));
  } else {
    // l0 = current lengths: column 3 of vals holds l_I
    RC_HIP(hipMemcpyAsync(k.len0, k.vals + 3 * (size_t)nE, sizeof(double) * nE, hipMemcpyDeviceToDevice, s));
  }
  RC_TRY(sync(c));
  c->mg_prepared = false;
  c->dense_prepared = false;
  return RC_OK;
}

int32_t rc_constraint_count(const rc_ctx* c) { return c ? c->cons.k : 0; }

rc_status rc_constraint_values(rc_ctx* c, const double* gamma, double* phi) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, phi}));
  if (c->cons.k == 0) return RC_OK;
  cons_values(c, gamma, phi);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status rc_project(rc_ctx* c, const double* gamma, const double* X, double* Y) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, X, Y}));
  if (c->cons.k > 0) RC_TRY(cons_prepare(c, gamma));
  cons_project(c, X, Y);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status rc_sobolev_gradient(rc_ctx* c, const double* gamma, const double* dE, double* g,
                              const rc_solve_opts* opts, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, dE, g}));
  rc_solve_opts o = resolve(opts);
  RC_TRY(prepare_solver(c, gamma, o));
  int iters = 0;
  double res = 0.0;
  rc_status st = solve_prepared(c, dE, g, o, &iters, &res);
  if (stats) {
    stats->iterations = iters;
    stats->residual = res;
    stats->status = st;
  }
  return st;
}

rc_status rc_line_search_step(rc_ctx* c, double* gamma, double energy0, const double* dE, const double* g,
                              const rc_ls_opts* ls, const rc_solve_opts* so, double* tau_h, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, dE, g}));
  rc_solve_opts o = resolve(so);
  rc_ls_opts l = resolve_ls(ls);
  RC_TRY(prepare_solver(c, gamma, o));
  LsResult r;
  rc_status st = line_search(c, gamma, energy0, dE, g, l, o, &r);
  if (tau_h) *tau_h = r.tau;
  if (stats) {
    stats->tau = r.tau;
    stats->energy_new = r.E1;
    stats->backtracks = r.backtracks;
    stats->proj_iters = r.proj_iters;
    stats->proj_solve_iterations = r.proj_solve_iters;
    stats->status = st;
  }
  return st;
}

rc_status rc_step(rc_ctx* c, double* gamma, const rc_solve_opts* so, const rc_ls_opts* ls, rc_stats* stats) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma}));
  rc_solve_opts o = resolve(so);
  rc_ls_opts l = resolve_ls(ls);
  hipStream_t s = c->stream;
  // dE and g live in buffers that no solver routine touches
  double* dEb = c->dEs;
  double* gb = c->gs;
  rc_stats local{};
  rc_status st = RC_OK;
  do {
    st = launch_geometry(c->curve, gamma, c->dtype, s);
    if (st) break;
    st = launch_tpe(c->curve, c->alpha, c->beta, c->dtype, true, c->scal + 8, dEb, s);
    if (st) break;
    st = fetch(c, c->scal + 8, &local.energy, 1);
    if (st) break;
    if (!std::isfinite(local.energy)) {
      set_error("energy is not finite");
      st = RC_ERR_NONFINITE;
      break;
    }
    st = prepare_solver(c, gamma, o);
    if (st) break;
    int iters = 0;
    double res = 0.0;
    st = solve_prepared(c, dEb, gb, o, &iters, &res);
    local.iterations = iters;
    local.residual = res;
    if (st) break;
    vec_dot(gb, gb, 3 * c->nV, c->red, c->scal, s);
    double gg;
    st = fetch(c, c->scal, &gg, 1);
    if (st) break;
    local.grad_norm = std::sqrt(gg);
    LsResult r;
    st = line_search(c, gamma, local.energy, dEb, gb, l, o, &r);
    local.tau = r.tau;
    local.energy_new = r.E1;
    local.backtracks = r.backtracks;
    local.proj_iters = r.proj_iters;
    local.proj_solve_iterations = r.proj_solve_iters;
  } while (false);
  local.status = st;
  if (stats) *stats = local;
  return st;
}

}  // extern "C"

extern "C" rc_status rc_midpoint_differential(rc_ctx* c, const double* gamma, double* energy, double* dE) {
  RC_TRY(check_ctx(c));
  RC_TRY(check_ptrs({gamma, dE}));
  RC_TRY(launch_geometry(c->curve, gamma, c->dtype, c->stream));
  return launch_midpoint(c->curve, c->alpha, c->beta, c->dtype, energy, dE, c->stream);
}
