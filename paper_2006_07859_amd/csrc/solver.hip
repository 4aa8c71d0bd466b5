// Host orchestration of the constrained Sobolev solve (paper Sec. 4.3-4.4,
// App. B.3): constraint projection, dense saddle factorisation, projected
// multigrid-preconditioned CG, constraint projection of trial steps and the
// backtracking line search.
//
// The host drives the loops and reads back only the scalars that decide
// control flow; every vector operation runs in the kernels of k_pairs.hip and
// k_linalg.hip.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "k_linalg.h"
#include "solver.h"

namespace rc {

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

template <typename T>
static void dfree(T*& p) {
  if (p) hipFree(p);
  p = nullptr;
}

rc_status sync(rc_ctx* c) {
  RC_HIP(hipStreamSynchronize(c->stream));
  return RC_OK;
}

rc_status fetch(rc_ctx* c, const double* dev, double* host, int n) {
  RC_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  return sync(c);
}

bool trace_on() {
  static int on = -1;
  if (on < 0) {
    const char* v = getenv("RC_TRACE");
    on = (v && v[0] == '1') ? 1 : 0;
  }
  return on == 1;
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
// small kernels
// ---------------------------------------------------------------------------
// b in external order (barycenter and total length [nbt], points, surface, tangents [2 ntg] from
// ext_tg, edges from nd) -> path rows wp and border rows wb (barycenter, total length, tangents,
// cut edges)
__global__ void k_map_rhs(const double* __restrict__ b, int nbt, int ext_tg, int ntg, int nd,
                          const int* __restrict__ path_edge, int np, const int* __restrict__ cut_edge, int ncut,
                          double* __restrict__ wp, double* __restrict__ wb, double sign) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) wp[i] = sign * b[nd + path_edge[i]];
  if (i < nbt) wb[i] = sign * b[i];
  if (i < 2 * ntg) wb[nbt + i] = sign * b[ext_tg + i];
  if (i < ncut) wb[nbt + 2 * ntg + i] = sign * b[nd + cut_edge[i]];
}

// tangent rows of Phi: (u . T_I, v . T_I) from row0 (geo: the edges' T at slots 1..3)
__global__ void k_phi_tangent(const double* __restrict__ geo, const int* __restrict__ tg,
                              const double* __restrict__ tgb, int ntg, int row0, double* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ntg) return;
  const double* t = geo + 8 * (size_t)tg[i / 2] + 1;
  const double* b = tgb + 6 * (i / 2) + 3 * (i % 2);
  phi[row0 + i] = b[0] * t[0] + b[1] * t[1] + b[2] * t[2];
}

// The implicit surface of a surface constraint by value (kernel argument).
struct SurfPar {
  int kind;
  double p[5];
};

static SurfPar surf_par(const Cons& k) {
  SurfPar q;
  q.kind = k.surf.kind;
  for (int j = 0; j < 5; ++j) q.p[j] = k.surf.par[j];
  return q;
}

// f(x) and grad f(x): the signed distance of a sphere (|x - c| - r) or of a torus about the z
// axis through c (sqrt((rho - R)^2 + (z - c_z)^2) - r, rho the distance from the axis)
__device__ __forceinline__ double surf_eval(const SurfPar& q, const double* x, double* gr) {
  const double d0 = x[0] - q.p[0], d1 = x[1] - q.p[1], d2 = x[2] - q.p[2];
  if (q.kind == RC_SURFACE_SPHERE) {
    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    gr[0] = d0 / r;
    gr[1] = d1 / r;
    gr[2] = d2 / r;
    return r - q.p[3];
  }
  const double rho = sqrt(d0 * d0 + d1 * d1);
  const double a = rho - q.p[3];
  const double qq = sqrt(a * a + d2 * d2);
  gr[0] = a / qq * d0 / rho;
  gr[1] = a / qq * d1 / rho;
  gr[2] = d2 / qq;
  return qq - q.p[4];
}

// grad f at the held vertices, and their unit normals in the per-vertex array
__global__ void k_surface_prepare(const double* __restrict__ gamma, const int* __restrict__ sf, int nsf,
                                  SurfPar q, double* __restrict__ sgrad, double* __restrict__ nrm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsf) return;
  const int v = sf[j];
  double gr[3];
  surf_eval(q, gamma + 3 * (size_t)v, gr);
  const double inv = 1.0 / sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
  for (int c = 0; c < 3; ++c) {
    sgrad[3 * j + c] = gr[c];
    nrm[3 * (size_t)v + c] = gr[c] * inv;
  }
}

// surface rows of Phi: f(gamma_i) from row0
__global__ void k_phi_surface(const double* __restrict__ gamma, const int* __restrict__ sf, int nsf, SurfPar q,
                              int row0, double* __restrict__ phi) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsf) return;
  double gr[3];
  phi[row0 + j] = surf_eval(q, gamma + 3 * (size_t)sf[j], gr);
}

// surface rows of the dense C: grad f(gamma_i)^T at vertex i, from row0
__global__ void k_dense_C_surface(const double* __restrict__ sgrad, const int* __restrict__ sf, int nsf, int row0,
                                  int nV, double* __restrict__ Cd) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nsf) return;
  for (int c = 0; c < 3; ++c) Cd[(size_t)(row0 + j) * 3 * nV + 3 * sf[j] + c] = sgrad[3 * j + c];
}

// The eliminated rows' part v of a particular solution of C z = b (z zero on entry): v_p = b_p at a
// pinned vertex (its three point rows), v_i = b_i grad f / |grad f|^2 at a held vertex (its
// surface row), so that those rows hold for v + F u whatever u.
__global__ void k_particular(const double* __restrict__ b, int nbt, const int* __restrict__ pt, int npt,
                             const int* __restrict__ sf, const double* __restrict__ sgrad, int nsf,
                             double* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * npt) z[3 * (size_t)pt[i / 3] + i % 3] = b[nbt + i];
  if (i < nsf) {
    const double* gr = sgrad + 3 * i;
    const double s = b[nbt + 3 * npt + i] / (gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
    for (int c = 0; c < 3; ++c) z[3 * (size_t)sf[i] + c] = s * gr[c];
  }
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

// point rows of Phi (Sec. 7.1): gamma_i - x_i, three per pinned vertex from row0
__global__ void k_phi_points(const double* __restrict__ gamma, const int* __restrict__ pt,
                             const double* __restrict__ ptx, int npt, int row0, double* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * npt) return;
  phi[row0 + i] = gamma[3 * (size_t)pt[i / 3] + i % 3] - ptx[i];
}

__global__ void k_gather_coarse(const double* __restrict__ fine, const int* __restrict__ fine_of, int nc,
                                double* __restrict__ coarse) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  int f = fine_of[i];
  coarse[3 * i] = fine[3 * f];
  coarse[3 * i + 1] = fine[3 * f + 1];
  coarse[3 * i + 2] = fine[3 * f + 2];
}

// xf = J xc: fine v gets (x_a + x_b)/2 (a = b for kept vertices)
__global__ void k_prolong(const int2* __restrict__ pr, int nf, const double* __restrict__ xc, double* __restrict__ xf) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nf) return;
  int2 ab = pr[v];
  for (int k = 0; k < 3; ++k) xf[3 * v + k] = 0.5 * (xc[3 * ab.x + k] + xc[3 * ab.y + k]);
}

// bc = J^T rf
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

__global__ void k_add_const(double* __restrict__ A, int n, double rho) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) A[i] += rho;
}


__global__ void k_negate(const double* __restrict__ in, double* __restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -in[i];
}

__global__ void k_fill_u32(unsigned* __restrict__ x, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_fill(double* __restrict__ x, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
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

// ---------------------------------------------------------------------------
// constraints of one level
// ---------------------------------------------------------------------------
void cons_free(Cons& k) {
  int* ip[] = {k.path_edge, k.path_prev, k.cut_edge, k.edge_path_row, k.pt, k.sf, k.tg};
  for (int* p : ip)
    if (p) hipFree(p);
  double* dp[] = {k.x0, k.len0, k.ones, k.geo, k.geo_eval, k.vals, k.rows, k.ta, k.td, k.tc, k.Kpb, k.Z, k.Sinv,
                  k.tri_scratch, k.wp, k.yp, k.wb, k.yb, k.dots, k.rhs, k.small, k.part, k.sp_VW, k.sp_Rt, k.sp_g,
                  k.sp_U, k.sp_tmp, k.ptx, k.free, k.weff, k.sgrad, k.nrm, k.tgb};
  for (double* p : dp)
    if (p) hipFree(p);
  if (k.prow) hipFree(k.prow);
  if (k.pvert) hipFree(k.pvert);
  if (k.rowsW) hipFree(k.rowsW);
  k = Cons();
}

rc_status cons_alloc(rc_ctx* c, const Curve& cv, Cons& k, uint32_t mask, const std::vector<int>& pts,
                     const SurfSpec* surf, const TangentSpec* tang) {
  (void)c;
  cons_free(k);
  k.mask = mask;
  k.h_pt = pts;
  k.npt = (int)pts.size();
  if (surf && surf->kind && !surf->verts.empty()) k.surf = *surf;
  k.nsf = (int)k.surf.verts.size();
  if (tang) k.tang = *tang;
  k.ntg = (int)k.tang.edges.size();
  k.elim = k.npt > 0 || k.nsf > 0;
  k.bary = (mask & RC_C_BARYCENTER) ? 1 : 0;
  k.total = (mask & RC_C_TOTAL_LENGTH) ? 1 : 0;
  k.edge = (mask & RC_C_EDGE_LENGTH) ? 1 : 0;
  const int nV = cv.nV, nE = cv.nE;
  k.h_edge_path_row.assign(nE, -1);
  if (k.edge) {
    // with junctions (vertices of degree >= 3) every edge at a junction is a border row; the
    // other edges form paths and loops whose rows stay tridiagonal
    std::vector<char> keep;
    if (!cv.chain) {
      keep.assign(nE, 1);
      for (int v = 0; v < nV; ++v)
        if (cv.h_inc_off[v + 1] - cv.h_inc_off[v] >= 3)
          for (int q = cv.h_inc_off[v]; q < cv.h_inc_off[v + 1]; ++q) keep[cv.h_inc[q] >> 1] = 0;
      for (int I = 0; I < nE; ++I)
        if (!keep[I]) k.h_cut_edge.push_back(I);
    }
    for (const Chain& ch : chains_of(cv, cv.chain ? nullptr : &keep)) {
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
  k.nbt = 3 * k.bary + k.total;
  k.ext_tg = k.nbt + 3 * k.npt + k.nsf;
  k.nd = k.ext_tg + 2 * k.ntg;
  k.nb = k.nbt + 2 * k.ntg + k.ncut;
  k.k = k.nd + (k.edge ? nE : 0);
  if (k.nb > 120) {
    set_error("too many rows in the projector's dense block (at most 120: 3 + 1 for barycenter and total length, "
              "2 per tangent constraint, and with edge-length constraints 1 per loop and 1 per edge at a vertex of "
              "degree >= 3)");
    return RC_ERR_UNSUPPORTED;
  }
  if (k.elim) {
    RC_TRY(dalloc(&k.free, nV));
    RC_TRY(dalloc(&k.weff, nV));
    std::vector<double> fr(nV, 1.0);
    for (int v : pts) fr[v] = 0.0;
    RC_HIP(hipMemcpy(k.free, fr.data(), sizeof(double) * nV, hipMemcpyHostToDevice));
  }
  if (k.npt) {
    RC_TRY(dalloc(&k.pt, k.npt));
    RC_TRY(dalloc(&k.ptx, 3 * (size_t)k.npt));
    RC_HIP(hipMemcpy(k.pt, pts.data(), sizeof(int) * k.npt, hipMemcpyHostToDevice));
    RC_HIP(hipMemset(k.ptx, 0, sizeof(double) * 3 * k.npt));
  }
  if (k.ntg) {
    RC_TRY(dalloc(&k.tg, k.ntg));
    RC_TRY(dalloc(&k.tgb, 6 * (size_t)k.ntg));
    RC_HIP(hipMemcpy(k.tg, k.tang.edges.data(), sizeof(int) * k.ntg, hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(k.tgb, k.tang.basis.data(), sizeof(double) * 6 * k.ntg, hipMemcpyHostToDevice));
  }
  if (k.nsf) {
    RC_TRY(dalloc(&k.sf, k.nsf));
    RC_TRY(dalloc(&k.sgrad, 3 * (size_t)k.nsf));
    RC_TRY(dalloc(&k.nrm, 3 * (size_t)nV));
    RC_HIP(hipMemcpy(k.sf, k.surf.verts.data(), sizeof(int) * k.nsf, hipMemcpyHostToDevice));
    RC_HIP(hipMemset(k.nrm, 0, sizeof(double) * 3 * nV));
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
  RC_TRY(dalloc(&k.tri_scratch, 2 * (size_t)std::max(k.np, 1) + 2));  // l and 1/u of the path block, info
  RC_TRY(dalloc(&k.wp, k.np));
  RC_TRY(dalloc(&k.yp, k.np));
  RC_TRY(dalloc(&k.wb, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.yb, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.rhs, std::max(k.nb, 1)));
  RC_TRY(dalloc(&k.dots, (size_t)std::max(k.nb * k.nb, 4)));
  RC_TRY(dalloc(&k.small, (size_t)std::max(k.nb * k.nb, 8)));
  k.tri = tri_blocks(k.np);
  if (k.tri.B > kSpMaxB) {
    set_error("edge-length constraints: too many path rows for the block-partitioned solve");
    return RC_ERR_UNSUPPORTED;
  }
  const size_t nbc = std::max(k.nb, 1), npc = std::max(k.np, 1);
  RC_TRY(dalloc(&k.part, (size_t)std::max(k.tri.B, 64) * 2 * kProjMaxBorder));
  RC_TRY(dalloc(&k.sp_VW, 2 * npc));
  RC_TRY(dalloc(&k.sp_Rt, std::max((size_t)k.tri.nr * k.tri.nr, (size_t)1)));
  RC_TRY(dalloc(&k.sp_g, nbc * npc));
  RC_TRY(dalloc(&k.sp_U, nbc * std::max(k.tri.nr, 1)));
  RC_TRY(dalloc(&k.sp_tmp, 2 * npc));
  if (cv.max_degree <= 2) {
    RC_HIP(hipMalloc(&k.prow, sizeof(ProjRow) * std::max(k.np, 1)));
    RC_HIP(hipMalloc(&k.pvert, sizeof(ProjVert) * std::max(nV, 1)));
  }
  std::vector<double> ones(nE, 1.0);
  RC_HIP(hipMemcpy(k.ones, ones.data(), sizeof(double) * nE, hipMemcpyHostToDevice));
  RC_HIP(hipMemset(k.x0, 0, sizeof(double) * 3));
  return RC_OK;
}

// Targets of the finest level's constraints (x0, L0, l0) from gamma_ref.
rc_status cons_set_targets(rc_ctx* c, const double* gamma_ref, const double* x0_h, double total_len0,
                           const double* edge_len0) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nE = c->nE;
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
  if (edge_len0)
    RC_HIP(hipMemcpyAsync(k.len0, edge_len0, sizeof(double) * nE, hipMemcpyDeviceToDevice, s));
  else  // l0 = current lengths: column 3 of vals holds l_I
    RC_HIP(hipMemcpyAsync(k.len0, k.vals + 3 * (size_t)nE, sizeof(double) * nE, hipMemcpyDeviceToDevice, s));
  return sync(c);
}

// The path block's factors as a block-partitioned tridiagonal system.
static TriSys path_sys(const Cons& k) {
  TriSys T;
  T.L = k.tri;
  T.lo = k.tri_scratch;
  T.uinv = k.tri_scratch + k.np;
  T.c = k.tc;
  T.V = k.sp_VW;
  T.W = k.sp_VW + k.np;
  T.Rt = k.sp_Rt;
  return T;
}

// C(gamma), the tridiagonal path block and the border Schur complement, of
// C C^T, or of C W C^T with W = diag(w) per vertex when w is given (times the
// free mask when vertices are pinned).
rc_status cons_prepare(rc_ctx* c, const Curve& cv, Cons& k, const double* gamma, const double* w) {
  if (k.k == 0) return RC_OK;
  hipStream_t s = c->stream;
  const int nV = cv.nV, nE = cv.nE;
  if (k.elim) {
    free_weights(w, k.free, nV, k.weff, s);
    w = k.weff;
  }
  if (k.nsf)
    hipLaunchKernelGGL(k_surface_prepare, dim3(cdiv(k.nsf, 64)), dim3(64), 0, s, gamma, k.sf, k.nsf, surf_par(k),
                       k.sgrad, k.nrm);
  cons_geometry(gamma, cv.edges, nE, k.geo, s);
  cons_border_rows(k.geo, cv.inc_off, cv.inc, cv.edges, k.x0, nV, k.bary, k.total, k.tg, k.tgb, k.ntg, k.cut_edge,
                   k.ncut, k.rows, k.nb, s);
  const int nb = k.nb, np = k.np;
  double* lo = k.tri_scratch;
  double* uinv = k.tri_scratch + np;
  int* tinfo = (int*)(k.tri_scratch + 2 * np);
  if (np > 0) {
    cons_path_coeffs(k.geo, cv.edges, k.path_edge, k.path_prev, np, w, k.nrm, k.ta, k.td, k.tc, s);
    tri_prepare(k.ta, k.td, k.tc, k.tri, lo, uinv, k.sp_VW, k.sp_Rt, k.sp_tmp, tinfo, s);
    flag_if_nonzero(tinfo, c->setup_flags, kSetupGram, s);
  }
  if (k.prow)
    cons_project_pack(k.geo, cv.edges, k.path_edge, np, cv.inc_off, cv.inc, k.edge_path_row, nV, k.prow, k.pvert, s);
  if (nb > 0) {
    const double* rows2 = k.rows;  // W rows
    if (w) {
      if (!k.rowsW) RC_TRY(dalloc(&k.rowsW, (size_t)nb * 3 * nV));
      cons_scale_rows(k.rows, w, k.nrm, nV, nb, k.rowsW, s);
      rows2 = k.rowsW;
    }
    // the Gram products in one pair of launches each while the scratch holds nb^2 partial sets
    const bool gram = nb * nb <= kRedSets;
    if (gram) vec_gram(k.rows, 3 * nV, rows2, 3 * nV, 3 * nV, nb, nb, c->red, k.dots, s);
    else
      for (int r = 0; r < nb; ++r)
        vec_dots(k.rows, 3 * nV, rows2 + (size_t)r * 3 * nV, 0, 3 * nV, nb, c->red, k.dots + r * nb, s);
    if (np > 0) {
      cons_path_apply(k.geo, cv.edges, k.path_edge, np, rows2, nV, nb, k.Kpb, s);
      tri_solve(path_sys(k), k.Kpb, np, k.Z, np, nb, k.sp_g, k.sp_U, s);
      if (gram) vec_gram(k.Kpb, np, k.Z, np, np, nb, nb, c->red, k.small, s);
      else
        for (int r = 0; r < nb; ++r)
          vec_dots(k.Kpb, np, k.Z + (size_t)r * np, 0, np, nb, c->red, k.small + r * nb, s);
    }
    // a border row that vanishes on the free vertices (a cut edge with both ends pinned) is zero
    // in S: a unit diagonal gives it a zero multiplier
    if (nb <= kSchurDevMax) {
      schur_inverse_device(k.dots, np > 0 ? k.small : nullptr, nb, k.elim, k.Sinv, c->setup_flags, kSetupSchur, s);
      return RC_OK;
    }
    std::vector<double> S(nb * nb), kz(nb * nb, 0.0);
    RC_TRY(fetch(c, k.dots, S.data(), nb * nb));
    if (np > 0) RC_TRY(fetch(c, k.small, kz.data(), nb * nb));
    for (int i = 0; i < nb * nb; ++i) S[i] -= kz[i];
    if (k.elim)
      for (int i = 0; i < nb; ++i)
        if (S[i * nb + i] == 0.0) S[i * nb + i] = 1.0;
    if (!invert_small(S, nb)) {
      set_error("constraint Schur complement is singular (dependent constraints?)");
      return RC_ERR_SINGULAR;
    }
    RC_HIP(hipMemcpyAsync(k.Sinv, S.data(), sizeof(double) * nb * nb, hipMemcpyHostToDevice, s));
    return sync(c);  // S is read by the copy
  }
  return RC_OK;
}

rc_status setup_check(rc_ctx* c) {
  unsigned f = 0;
  RC_HIP(hipMemcpyAsync(&f, c->setup_flags, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, c->setup_flags, 1, 0u);
  RC_TRY(sync(c));
  if (f & kSetupGram) {
    set_error("edge-length constraint Gram matrix is not positive definite");
    return RC_ERR_SINGULAR;
  }
  if (f & kSetupSchur) {
    set_error("constraint Schur complement is singular (dependent constraints?)");
    return RC_ERR_SINGULAR;
  }
  return RC_OK;
}

// (wp, wb) -> (yp, yb) = (C C^T)^-1 w
static void cons_solve_K(rc_ctx* c, Cons& k) {
  hipStream_t s = c->stream;
  if (k.np > 0) tri_solve(path_sys(k), k.wp, k.np, k.yp, k.np, 1, k.sp_g, k.sp_U, s);
  if (k.nb > 0) {
    if (k.np > 0) vec_dots(k.Kpb, k.np, k.yp, 0, k.np, k.nb, c->red, k.dots, s);
    else hipMemsetAsync(k.dots, 0, sizeof(double) * k.nb, s);
    cons_border_solve(k.Sinv, k.wb, k.dots, k.rhs, k.nb, k.yb, s);
    cons_sub_Zy(k.Z, k.yb, k.nb, k.np, k.yp, s);
  }
}

// The three-launch projector's data for one level's constraints.
static ProjData proj_data(const Curve& cv, Cons& k) {
  ProjData d;
  d.np = k.np;
  d.nb = k.nb;
  d.nV = cv.nV;
  d.geo = k.geo;
  d.edges = cv.edges;
  d.path_edge = k.path_edge;
  d.rows = k.rows;
  d.Z = k.Z;
  d.Sinv = k.Sinv;
  d.tri = k.tri;
  d.lo = k.tri_scratch;
  d.uinv = k.tri_scratch + k.np;
  d.tc = k.tc;
  d.V = k.sp_VW;
  d.W = k.sp_VW + k.np;
  d.Rt = k.sp_Rt;
  d.inc_off = cv.inc_off;
  d.inc = cv.inc;
  d.edge_path_row = k.edge_path_row;
  d.prow = k.prow;
  d.pvert = k.pvert;
  d.part = k.part;
  d.g = k.sp_g;
  d.U = k.sp_U;
  d.yb = k.yb;
  return d;
}

// Points a projection's last launch at the operand of pop's next product.
static void set_prep(ProjData& d, const LowpOp* pop, bool pfrom_x) {
  if (!pop) return;
  d.pp = pop->pbuf;
  d.pcref = pop->cref;
  d.psqd = pop->sqd;
  d.prep_x = pfrom_x;
}

// out = beta prev + scale M in with M = W - W C^T (C W C^T)^-1 C W, W = diag(w):
// kw holds the factors of C W C^T (cons_prepare with w); nb <= kProjMaxBorder.
// With xacc, also xacc = out (xset) or xacc += out.  With pop, also the
// operand of pop's next product (of out, or of xacc when pfrom_x).
static void cons_project_w(rc_ctx* c, const Curve& cv, Cons& kw, const double* w, const double* in, double* out,
                           double scale, double beta, const double* prev, double* xacc = nullptr,
                           bool xset = false, const LowpOp* pop = nullptr, bool pfrom_x = false) {
  ProjData d = proj_data(cv, kw);
  set_prep(d, pop, pfrom_x);
  d.w = kw.elim ? kw.weff : w;  // (w times the free mask with pinned vertices, as prepared)
  d.nrm = kw.nrm;
  d.scale = scale;
  d.beta = beta;
  d.prev = prev;
  d.xacc = xacc;
  d.xset = xset;
  cons_project_fused(d, in, out, c->stream);
}

// out = P in with P = I - C^T (C C^T)^-1 C (in may equal out), the orthogonal
// projector onto null(C); with pinned vertices and surface constraints
// P = F - F C^T (C F C^T)^-1 C F (F_v = 0 at a pinned vertex, I - n_v n_v^T on
// a surface, I elsewhere), onto null(C) with the pinned entries zero and the
// held vertices' entries tangent to the surface.  With xacc, also xacc += out.
bool cons_project(rc_ctx* c, const Curve& cv, Cons& k, const double* in, double* out, double* xacc,
                  const LowpOp* pop, bool pfrom_x) {
  hipStream_t s = c->stream;
  const int nV = cv.nV;
  if (k.k == 0) {
    if (in != out) vec_copy(in, out, 3 * nV, s);
    if (xacc) vec_axpby(1.0, out, 1.0, xacc, 3 * nV, s);
    return false;
  }
  if (k.nb <= kProjMaxBorder) {
    ProjData d = proj_data(cv, k);
    d.w = k.elim ? k.weff : nullptr;
    d.nrm = k.nrm;
    d.xacc = xacc;
    set_prep(d, pop, pfrom_x);
    cons_project_fused(d, in, out, s);
    return pop != nullptr;
  }
  if (k.elim) {  // F in, then F (F in - C^T y) with y from C F in
    if (in != out) vec_copy(in, out, 3 * nV, s);
    mask_vertices(out, k.weff, k.nrm, nV, s);
    in = out;
  }
  cons_path_apply(k.geo, cv.edges, k.path_edge, k.np, in, nV, 1, k.wp, s);
  if (k.nb > 0) vec_dots(k.rows, 3 * nV, in, 0, 3 * nV, k.nb, c->red, k.wb, s);
  cons_solve_K(c, k);
  cons_apply_CT(k.geo, cv.inc_off, cv.inc, k.edge_path_row, k.yp, k.rows, k.yb, k.nb, nV, in, out, s);
  if (k.elim) mask_vertices(out, k.weff, k.nrm, nV, s);
  if (xacc) vec_axpby(1.0, out, 1.0, xacc, 3 * nV, s);
  return false;
}

// A particular solution z of C z = b for an external-order b (finest level):
// z = C^T (C C^T)^-1 b, the minimum-norm one, without eliminated rows; with
// point and surface rows z = v + F C^T (C F C^T)^-1 (b_C - C v), v their part
// (k_particular), which satisfies every row.  scratch: [3 nV].
static void cons_min_norm(rc_ctx* c, const double* b, double* z, double* scratch) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nV = c->nV, n3 = 3 * nV;
  const int n = std::max(k.np, std::max(k.nb, 1));
  hipLaunchKernelGGL(k_map_rhs, dim3(cdiv(n, 256)), dim3(256), 0, s, b, k.nbt, k.ext_tg, k.ntg, k.nd, k.path_edge,
                     k.np, k.cut_edge, k.ncut, k.wp, k.wb, -1.0);
  if (k.elim) {  // (wp, wb) = -(b_C - C v)
    hipLaunchKernelGGL(k_fill, dim3(cdiv(n3, 256)), dim3(256), 0, s, z, n3, 0.0);
    hipLaunchKernelGGL(k_particular, dim3(cdiv(std::max(3 * k.npt, k.nsf), 64)), dim3(64), 0, s, b, k.nbt, k.pt,
                       k.npt, k.sf, k.sgrad, k.nsf, z);
    if (k.np > 0) {
      cons_path_apply(k.geo, c->curve.edges, k.path_edge, k.np, z, nV, 1, k.yp, s);
      vec_axpby(1.0, k.yp, 1.0, k.wp, k.np, s);
    }
    if (k.nb > 0) {
      vec_dots(k.rows, n3, z, 0, n3, k.nb, c->red, k.yb, s);
      vec_axpby(1.0, k.yb, 1.0, k.wb, k.nb, s);
    }
  }
  cons_solve_K(c, k);
  // apply_CT computes in - C^T y with in = null: -C^T y, and y = K^-1 (-b)
  double* u = k.elim ? scratch : z;
  cons_apply_CT(k.geo, c->curve.inc_off, c->curve.inc, k.edge_path_row, k.yp, k.rows, k.yb, k.nb, nV, nullptr, u,
                s);
  if (k.elim) {
    mask_vertices(u, k.weff, k.nrm, nV, s);
    vec_axpby(1.0, u, 1.0, z, n3, s);
  }
}

// Phi(gamma) in external order (barycenter, total length, points, surface, tangents, edges).
void cons_values(rc_ctx* c, const double* gamma, double* phi) {
  Cons& k = c->cons;
  hipStream_t s = c->stream;
  const int nE = c->nE;
  cons_geometry(gamma, c->curve.edges, nE, k.geo_eval, s);
  const int nbt = 3 * k.bary + k.total;
  cons_phi_edge(k.geo_eval, k.x0, nE, k.len0, k.vals, k.edge ? phi + k.nd : nullptr, s);
  if (nbt > 0) {
    vec_dots(k.vals, nE, k.ones, 0, nE, 4, c->red, k.small, s);
    hipLaunchKernelGGL(k_phi_border, dim3(1), dim3(1), 0, s, k.small, k.bary, k.total, k.total0, phi);
  }
  if (k.npt > 0)
    hipLaunchKernelGGL(k_phi_points, dim3(cdiv(3 * k.npt, 64)), dim3(64), 0, s, gamma, k.pt, k.ptx, k.npt, nbt, phi);
  if (k.nsf > 0)
    hipLaunchKernelGGL(k_phi_surface, dim3(cdiv(k.nsf, 64)), dim3(64), 0, s, gamma, k.sf, k.nsf, surf_par(k),
                       nbt + 3 * k.npt, phi);
  if (k.ntg > 0)
    hipLaunchKernelGGL(k_phi_tangent, dim3(cdiv(2 * k.ntg, 64)), dim3(64), 0, s, k.geo_eval, k.tg, k.tgb, k.ntg,
                       k.ext_tg, phi);
}

// ---------------------------------------------------------------------------
// dense saddle on one level
// ---------------------------------------------------------------------------
void dense_free(Dense& d) {
  dfree(d.A);
  dfree(d.Cd);
  dfree(d.CtC);
  dfree(d.H);
  dfree(d.W);
  dfree(d.S);
  dfree(d.Sinv);
  dfree(d.gjm);
  dfree(d.gjo);
  dfree(d.gjc);
  dfree(d.t1);
  dfree(d.t2);
  dfree(d.t3);
  dfree(d.X);
  dfree(d.info);
  d = Dense();
}

static rc_status dense_prepare(rc_ctx* c, const Curve& cv, Cons& k, Dense& d, const double* gamma) {
  hipStream_t s = c->stream;
  const int nV = cv.nV, n = 3 * nV, kk = k.k;
  if (nV > 2048) {
    set_error("dense solver limited to 2048 vertices");
    return RC_ERR_UNSUPPORTED;
  }
  if (d.nV != nV || d.k != kk) {
    dense_free(d);
    d.nV = nV;
    d.k = kk;
    RC_TRY(dalloc(&d.A, (size_t)nV * nV));
    RC_TRY(dalloc(&d.CtC, (size_t)n * n));
    RC_TRY(dalloc(&d.Cd, (size_t)std::max(kk, 1) * n));
    RC_TRY(dalloc(&d.W, (size_t)n * std::max(kk, 1)));
    RC_TRY(dalloc(&d.S, (size_t)std::max(kk * kk, 1)));
    RC_TRY(dalloc(&d.Sinv, (size_t)std::max(kk * kk, 1)));
    RC_TRY(dalloc(&d.t1, (size_t)std::max(kk, 1)));
    RC_TRY(dalloc(&d.t2, (size_t)std::max(kk, 1)));
    RC_TRY(dalloc(&d.t3, (size_t)n));
    RC_TRY(dalloc(&d.X, (size_t)n * n));
    RC_TRY(dalloc(&d.info, 2));
    RC_TRY(dalloc(&d.gjm, 4));
    RC_TRY(dalloc(&d.gjo, 1));
    RC_TRY(dalloc(&d.gjc, (size_t)32 * std::max(n, kk) + 1024));
  }
  RC_TRY(launch_geometry(cv, gamma, RC_F32, s));
  RC_TRY(launch_assemble_dense(cv, c->alpha, c->beta, d.A, s));
  if (kk > 0) {
    // dense C in external order: the border rows of barycenter and total length, the point
    // rows, the surface rows, the tangent rows of the border, then the edge rows
    RC_HIP(hipMemsetAsync(d.Cd, 0, sizeof(double) * (size_t)kk * n, s));
    if (k.nbt > 0)
      RC_HIP(hipMemcpyAsync(d.Cd, k.rows, sizeof(double) * (size_t)k.nbt * n, hipMemcpyDeviceToDevice, s));
    dense_C_points(k.pt, k.npt, k.nbt, nV, d.Cd, s);
    if (k.nsf)
      hipLaunchKernelGGL(k_dense_C_surface, dim3(cdiv(k.nsf, 64)), dim3(64), 0, s, k.sgrad, k.sf, k.nsf,
                         k.nbt + 3 * k.npt, nV, d.Cd);
    if (k.ntg)  // the tangent rows of the border, after the surface rows
      RC_HIP(hipMemcpyAsync(d.Cd + (size_t)k.ext_tg * n, k.rows + (size_t)k.nbt * n,
                            sizeof(double) * (size_t)2 * k.ntg * n, hipMemcpyDeviceToDevice, s));
    if (k.edge) dense_C_edges(k.geo, cv.edges, cv.nE, k.nd, nV, k.free, d.Cd, s);
    dense_gemm(d.Cd, d.Cd, d.CtC, n, n, kk, 0.0, true, s);
  } else {
    // no constraint: regularise the constant null space with rho 1 1^T per component
    std::vector<double> Ah((size_t)nV * nV);
    RC_HIP(hipMemcpyAsync(Ah.data(), d.A, sizeof(double) * nV * nV, hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    double tr = 0;
    for (int i = 0; i < nV; ++i) tr += Ah[(size_t)i * nV + i];
    hipLaunchKernelGGL(k_add_const, dim3(cdiv(nV * nV, 256)), dim3(256), 0, s, d.A, nV, tr / ((double)nV * nV));
    RC_HIP(hipMemsetAsync(d.CtC, 0, sizeof(double) * (size_t)n * n, s));
  }
  // X = H^-1 (H built in X, inverted in place), then X -= W S^-1 W^T
  dense_build_H(d.A, d.CtC, nV, d.X, s);
  gj_invert_spd(d.X, n, d.gjm, d.gjo, d.gjc, d.info, s);
  if (kk > 0) {
    dense_gemm(d.X, d.Cd, d.W, n, kk, n, 0.0, false, s, true);  // W = H^-1 C^T
    dense_gemm(d.Cd, d.W, d.Sinv, kk, kk, n, 0.0, false, s);    // S = C H^-1 C^T (SPD)
    if (k.elim) unit_zero_diag(d.Sinv, kk, s);  // the zero rows of edges with both ends pinned
    gj_invert_spd(d.Sinv, kk, d.gjm, d.gjo, d.gjc, d.info + 1, s);
    // X += (-W S^-1) W^T, with -W S^-1 staged in CtC (no longer needed)
    dense_gemm(d.W, d.Sinv, d.CtC, n, kk, kk, 0.0, false, s);
    vec_axpby(0.0, d.CtC, -1.0, d.CtC, n * kk, s);
    dense_gemm(d.CtC, d.W, d.X, n, n, kk, 1.0, false, s, true);
  }
  int info[2] = {0, 0};
  RC_HIP(hipMemcpyAsync(info, d.info, sizeof(int) * (kk > 0 ? 2 : 1), hipMemcpyDeviceToHost, s));
  RC_TRY(sync(c));
  if (info[0] != 0) {
    set_error("Cholesky of Abar + C^T C failed: Abar is not definite on null(C)");
    return RC_ERR_SINGULAR;
  }
  if (info[1] != 0) {
    set_error("constraint Schur complement is singular");
    return RC_ERR_SINGULAR;
  }
  return RC_OK;
}

// x = H^-1 b - W S^-1 W^T b: the saddle solution with right-hand side (b, 0).
static void dense_solve(rc_ctx* c, Dense& d, const double* b, double* x) {
  dense_gemv(d.X, b, x, 3 * d.nV, c->stream);
}

// x = -W S^-1 phi: the saddle solution with right-hand side (0, -phi).
static void dense_increment(rc_ctx* c, Dense& d, const double* phi, double* x) {
  hipStream_t s = c->stream;
  const int n = 3 * d.nV, k = d.k;
  dense_gemm(d.Sinv, phi, d.t1, k, 1, k, 0.0, false, s);
  dense_gemm(d.W, d.t1, x, n, 1, k, 0.0, false, s);
  vec_axpby(0.0, x, -1.0, x, n, s);
}

// ---------------------------------------------------------------------------
// projected multigrid (App. B.3.1-B.3.3): every level carries its own
// constraints and projector, smooths P A P with projected Chebyshev-Jacobi,
// and the coarsest level solves its saddle problem densely.
// ---------------------------------------------------------------------------
static const Curve& level_curve(rc_ctx* c, int l) { return l == 0 ? c->curve : c->levels[l]->curve; }
static Cons& level_cons(rc_ctx* c, int l) { return l == 0 ? c->cons : c->levels[l]->cons; }
static Cons& level_cons_w(rc_ctx* c, int l) { return l == 0 ? c->cons_w : c->levels[l]->cons_w; }

// w = 1 / d per vertex
__global__ void k_recip(const double* __restrict__ d, int n, double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = 1.0 / d[i];
}

rc_status load_geometry(rc_ctx* c, const double* gamma) { return launch_geometry(c->curve, gamma, RC_F32, c->stream); }

void mg_free(rc_ctx* c) {
  for (auto& L : c->levels)
    if (L) {
      L->curve.release();
      cons_free(L->cons);
      cons_free(L->cons_w);
      dfree(L->fine_of);
      dfree(L->prolong);
      dfree(L->restr_off);
      dfree(L->restr_idx);
      dfree(L->gamma);
      L->lowp.release();
      L->bvh.release();
      L->bct.release();
    }
  c->levels.clear();
  cons_free(c->cons_w);
  for (auto& st : c->mg) {
    dfree(st.diag);
    dfree(st.w);
    dfree(st.x);
    dfree(st.b);
    dfree(st.r);
    dfree(st.d);
    dfree(st.t);
    dfree(st.pw);
  }
  c->mg.clear();
  dense_free(c->coarse);
  c->mg_built = false;
}

static rc_status mg_build(rc_ctx* c) {
  if (c->mg_built) return RC_OK;
  mg_free(c);
  c->levels.emplace_back(nullptr);
  const Curve* fine = &c->curve;
  std::vector<int> fine_pts = c->cons.h_pt;
  SurfSpec fine_surf = c->cons.surf;
  while (fine->nV > c->mg_min) {
    // loops and open paths; with junctions, the arcs between vertices of degree != 2
    std::vector<Chain> chs = arcs_of(*fine);
    // black/white coarsening: keep even chain positions, and both ends of open paths and arcs
    // (a junction is kept once, whatever the number of its arcs); an arc of at most 3 edges keeps
    // all its vertices (coarsened, two arcs between the same junctions could become one edge)
    std::vector<int> coarse_id(fine->nV, -1), fine_of, cedges;
    std::vector<int2> prolong(fine->nV, make_int2(-1, -1));
    bool ok = true;
    for (const Chain& ch : chs) {
      const int m = (int)ch.verts.size();
      const bool closed_arc = !ch.loop && ch.verts.front() == ch.verts.back();
      if ((ch.loop && m < 12) || (closed_arc && m < 13)) {
        ok = false;
        break;
      }
      std::vector<int> keep;
      for (int i = 0; i < m; ++i)
        if (i % 2 == 0 || (!ch.loop && (i == m - 1 || m < 5))) keep.push_back(i);
      for (int i : keep) {
        if (coarse_id[ch.verts[i]] >= 0) continue;
        coarse_id[ch.verts[i]] = (int)fine_of.size();
        fine_of.push_back(ch.verts[i]);
      }
      const int nk = (int)keep.size();
      for (int q = 0; q + 1 < nk || (ch.loop && q < nk); ++q) {
        cedges.push_back(coarse_id[ch.verts[keep[q]]]);
        cedges.push_back(coarse_id[ch.verts[keep[(q + 1) % nk]]]);
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
    for (int v = 0; ok && v < fine->nV; ++v)
      if (prolong[v].x < 0) ok = false;  // isolated vertices are not coarsened
    if (!ok || fine_of.size() == (size_t)fine->nV) break;
    std::vector<int> coarse_pts;
    for (int v : fine_pts)
      for (int q : {prolong[v].x, prolong[v].y})
        if (std::find(coarse_pts.begin(), coarse_pts.end(), q) == coarse_pts.end()) coarse_pts.push_back(q);
    if (4 * coarse_pts.size() > fine_of.size()) break;  // keep most of a level free
    auto L = std::make_unique<Level>();
    const int nc = (int)fine_of.size();
    RC_TRY(L->curve.init(nc, (int)cedges.size() / 2, cedges.data()));
    RC_TRY(dalloc(&L->fine_of, nc));
    RC_TRY(dalloc(&L->prolong, fine->nV));
    RC_TRY(dalloc(&L->gamma, 3 * (size_t)nc));
    RC_HIP(hipMemcpy(L->fine_of, fine_of.data(), sizeof(int) * nc, hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(L->prolong, prolong.data(), sizeof(int2) * fine->nV, hipMemcpyHostToDevice));
    std::vector<std::vector<int>> lists(nc);
    for (int v = 0; v < fine->nV; ++v) {
      lists[prolong[v].x].push_back(v);
      if (prolong[v].y != prolong[v].x) lists[prolong[v].y].push_back(v);
    }
    std::vector<int> off(nc + 1, 0), idx;
    for (int i = 0; i < nc; ++i) {
      off[i + 1] = off[i] + (int)lists[i].size();
      idx.insert(idx.end(), lists[i].begin(), lists[i].end());
    }
    RC_TRY(dalloc(&L->restr_off, nc + 1));
    RC_TRY(dalloc(&L->restr_idx, idx.size()));
    RC_HIP(hipMemcpy(L->restr_off, off.data(), sizeof(int) * (nc + 1), hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(L->restr_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
    // the level's own constraints (same kinds as the finest level); a pinned vertex pins the
    // coarse vertices it interpolates from, so that every prolonged correction vanishes on it
    // a held vertex that the coarsening keeps stays on the surface
    SurfSpec csurf = fine_surf;
    csurf.verts.clear();
    for (int v : fine_surf.verts)
      if (coarse_id[v] >= 0) csurf.verts.push_back(coarse_id[v]);
    RC_TRY(cons_alloc(c, L->curve, L->cons, c->cons.mask, coarse_pts, &csurf));
    fine_pts = coarse_pts;
    fine_surf = csurf;
    if (c->cons.bary)
      RC_HIP(hipMemcpy(L->cons.x0, c->cons.x0, sizeof(double) * 3, hipMemcpyDeviceToDevice));
    c->levels.push_back(std::move(L));
    fine = &c->levels.back()->curve;
  }
  const int nl = (int)c->levels.size();
  c->mg.assign(nl, MGLevelState());
  for (int l = 0; l < nl; ++l) {
    const int n = level_curve(c, l).nV;
    MGLevelState& st = c->mg[l];
    RC_TRY(dalloc(&st.diag, n));
    RC_TRY(dalloc(&st.w, n));
    double** bufs[] = {&st.x, &st.b, &st.r, &st.d, &st.t, &st.pw};
    for (double** b : bufs) RC_TRY(dalloc(b, 3 * (size_t)n));
    hipLaunchKernelGGL(k_fill_pattern, dim3(cdiv(3 * n, 256)), dim3(256), 0, c->stream, st.pw, 3 * n, 12345u + l);
  }
  c->mg_built = true;
  return RC_OK;
}

// After a failed set-up: the power iterations start cold again from their initial vectors (a set-up at
// a non-finite curve leaves non-finite iterates behind, which would seed the next call's warm start).
static void mg_reset_power(rc_ctx* c) {
  if (!c->mg_built) return;
  for (size_t l = 0; l < c->mg.size(); ++l) {
    MGLevelState& st = c->mg[l];
    const int n = level_curve(c, (int)l).nV;
    hipLaunchKernelGGL(k_fill_pattern, dim3(cdiv(3 * n, 256)), dim3(256), 0, c->stream, st.pw, 3 * n,
                       12345u + (unsigned)l);
    st.lmax = 0.0;
  }
}

// A X on a level: the block-cluster-tree product when the level has a tree
// (FP64 sums whatever prec), else the matrix-free operator in precision prec.
static rc_status apply_A(rc_ctx* c, const Curve& cv, const double* X, double* Y, rc_dtype prec) {
  if (cv.hbct) return launch_bct_apply(cv, *cv.hbvh, *cv.hbct, c->alpha, c->beta, X, Y, c->stream);
  return launch_sobolev(cv, c->alpha, c->beta, prec, X, Y, nullptr, c->stream);
}

static LowpOp& level_lowp(rc_ctx* c, int l) { return l == 0 ? c->lowp : c->levels[l]->lowp; }

// The operator of level l inside PCG and the smoothers: the assembled 16-bit
// block when the precision path covers the level, else the matrix-free
// operator in the context's precision.
static rc_status apply_level(rc_ctx* c, int l, const double* X, double* Y) {
  if (l < c->lowp_levels) return launch_lowp_apply(level_lowp(c, l), X, Y, c->stream, l == 0 ? &c->timer : nullptr);
  return apply_A(c, level_curve(c, l), X, Y, c->dtype);
}

// Learned smoother diagonals: the network's ratio prediction times this margin.
constexpr double kLearnedMargin = 1.05;

// scal[kPwSlot0 ..] holds the power iterations' squared norms, two per level (the context's scalar
// buffer has 128 slots; the solvers use the first 20)
constexpr int kPwSlot0 = 64, kPwSlots = 64;

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
  }
  for (int l = 0; l < nl; ++l) {
    Curve& cv = const_cast<Curve&>(level_curve(c, l));
    const double* gl = l == 0 ? gamma : c->levels[l]->gamma;
    RC_TRY(launch_geometry(cv, gl, RC_F32, s));
    // hierarchical operator: a block cluster tree of the level at its curve (not on the
    // coarsest level, whose dense saddle is assembled exactly)
    cv.hbvh = nullptr;
    cv.hbct = nullptr;
    if (c->bct_theta > 0.0 && l < nl - 1 && cv.nV >= c->bct_min_v) {
      Bvh& bv = l == 0 ? c->bct_bvh : c->levels[l]->bvh;
      Bct& bt = l == 0 ? c->bct : c->levels[l]->bct;
      RC_TRY(build_bct(cv, bv, bt, c->bct_theta, 32, s));
      cv.hbvh = &bv;
      cv.hbct = &bt;
    }
  }
  const rc_dtype prec = c->dtype;
  // the smoothers' weighted projector needs every smoothed level's border in the fused projector
  c->mg_weighted = c->cons.k > 0;
  for (int l = 0; l < nl - 1; ++l)
    c->mg_weighted = c->mg_weighted && level_cons(c, l).nb <= kProjMaxBorder && level_cons(c, l).k > 0;
  for (int l = 0; l < nl - 1; ++l) {
    const Curve& cv = level_curve(c, l);
    MGLevelState& st = c->mg[l];
    if (l < c->lowp_levels)
      RC_TRY(launch_assemble_lowp(cv, level_lowp(c, l), c->lowp_fmt, c->lowp_band, l == 0 && c->lowp_outer == 1,
                                  c->alpha, c->beta, st.diag, s));
    else if (cv.hbct)
      RC_TRY(launch_bct_apply(cv, *cv.hbvh, *cv.hbct, c->alpha, c->beta, st.pw, st.t, s, st.diag));
    else
      RC_TRY(launch_sobolev(cv, c->alpha, c->beta, prec, st.pw, st.t, st.diag, s));
    if (c->mg_learned)
      RC_TRY(launch_level_features(cv, l == 0 ? gamma : c->levels[l]->gamma, st.diag, c->learn_scratch,
                                   c->learn_X + (size_t)kMlpIn * c->learn_off[l], s));
  }
  if (c->mg_learned) {
    // the smoothers' diagonals D_v = margin (1 + y_v) diag_v from the network's ratio predictions
    const int rows = c->learn_off[nl - 1];
    RC_TRY(mlp_forward(c->mlp->m, c->learn_X, rows, c->learn_Y, false, s));
    for (int l = 0; l < nl - 1; ++l)
      RC_TRY(launch_learned_diag(c->learn_Y + c->learn_off[l], level_curve(c, l).nV, kLearnedMargin, c->mg[l].diag,
                                 s));
  }
  // every level's constraint factors: many small launches, enqueued while the device runs the
  // operators' assembly above (none of them waits for the device)
  for (int l = 0; l < nl; ++l)
    RC_TRY(cons_prepare(c, level_curve(c, l), level_cons(c, l), l == 0 ? gamma : c->levels[l]->gamma));
  std::vector<int> pw_levels;  // the levels whose smoother interval comes from power iteration
  for (int l = 0; l < nl - 1; ++l) {
    const Curve& cv = level_curve(c, l);
    Cons& K = level_cons(c, l);
    MGLevelState& st = c->mg[l];
    const int n = cv.nV;
    if (c->mg_weighted) {  // factors of C W C^T, W = D^-1
      Cons& Kw = level_cons_w(c, l);
      if (Kw.mask != K.mask || Kw.h_pt != K.h_pt || Kw.surf != K.surf || Kw.tang != K.tang || !Kw.geo)
        RC_TRY(cons_alloc(c, cv, Kw, K.mask, K.h_pt, &K.surf, &K.tang));
      RC_HIP(hipMemcpyAsync(Kw.x0, K.x0, sizeof(double) * 3, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_recip, dim3(cdiv(n, 256)), dim3(256), 0, s, st.diag, n, st.w);
      RC_TRY(cons_prepare(c, cv, Kw, l == 0 ? gamma : c->levels[l]->gamma, st.w));
    }
    if (c->mg_learned) {
      // the learned diagonal places the top of the spectrum of D^-1 A at 1 / margin, and the
      // projected operators' spectra lie inside that of D^-1 A
      st.lmax = 1.0;
      continue;
    }
    if (c->mg_cg) continue;  // the CG smoother needs no spectral interval
    pw_levels.push_back(l);
  }
  // lambda_max of the smoother's preconditioned operator (P D^-1 P A P, or M A with the weighted
  // projector M) by power iteration, warm-started from the last call's vector: at most 12
  // iterations, stopping once the estimate moves by less than 1 % after at least 3 (warm start) or 8
  // (first call) of them.  The iterate is normalised on the device, and the levels' estimates of
  // their last two iterations are read together once per pass (a level's first pass runs its
  // minimum count).
  const int npw = (int)pw_levels.size();
  if (2 * npw > kPwSlots) {
    set_error("multigrid setup: too many levels");
    return RC_ERR_UNSUPPORTED;
  }
  auto power_step = [&](int q, int it) -> rc_status {  // one iteration on level pw_levels[q]
    const int l = pw_levels[q];
    const Curve& cv = level_curve(c, l);
    Cons& K = level_cons(c, l);
    MGLevelState& st = c->mg[l];
    const int n = cv.nV;
    if (c->mg_weighted) {
      RC_TRY(apply_level(c, l, st.pw, st.t));
      cons_project_w(c, cv, level_cons_w(c, l), st.w, st.t, st.d, 1.0, 0.0, nullptr);
    } else {
      cons_project(c, cv, K, st.pw, st.pw);
      RC_TRY(apply_level(c, l, st.pw, st.t));
      cons_project(c, cv, K, st.t, st.t);
      vec_scale_diag_inv(st.t, st.diag, st.d, n, s);
      cons_project(c, cv, K, st.d, st.d);
    }
    double* sq = c->scal + kPwSlot0 + 2 * q + (it & 1);
    vec_dot(st.d, st.d, 3 * n, c->red, sq, s);
    vec_scale_rsqrt(st.d, sq, st.pw, 3 * n, s);
    return RC_OK;
  };
  std::vector<int> its(npw, 0);
  std::vector<char> done(npw, 0);
  std::vector<double> h(2 * std::max(npw, 1));
  for (int pass = 0; npw > 0; ++pass) {
    for (int q = 0; q < npw; ++q) {
      if (done[q]) continue;
      const int count = pass == 0 ? (c->mg[pw_levels[q]].lmax > 0.0 ? 3 : 8) : 1;
      for (int k = 0; k < count; ++k) RC_TRY(power_step(q, its[q]++));
    }
    RC_TRY(fetch(c, c->scal + kPwSlot0, h.data(), 2 * npw));
    bool all = true;
    for (int q = 0; q < npw; ++q) {
      if (done[q]) continue;
      const int it = its[q] - 1;  // the last iteration
      const double nrm = std::sqrt(h[2 * q + (it & 1)]), prev = std::sqrt(h[2 * q + ((it + 1) & 1)]);
      if (!(nrm > 0)) {
        set_error("multigrid setup: zero operator");
        return RC_ERR_SINGULAR;
      }
      if (std::fabs(nrm - prev) < 0.01 * nrm || its[q] >= 12) {
        done[q] = 1;
        MGLevelState& st = c->mg[pw_levels[q]];
        st.lmax = 1.1 * nrm;
        if (trace_on())
          fprintf(stderr, "[rc mg] level %d n %d lmax %.6e (%d iterations)\n", pw_levels[q],
                  level_curve(c, pw_levels[q]).nV, nrm, its[q]);
      } else {
        all = false;
      }
    }
    if (all) break;
  }
  RC_TRY(dense_prepare(c, level_curve(c, nl - 1), level_cons(c, nl - 1), c->coarse,
                       nl == 1 ? gamma : c->levels[nl - 1]->gamma));
  return RC_OK;
}

// Projected Chebyshev smoothing of P A_l P x = b (b in range(P)) on level l.
// Chebyshev smoothing of A x = b at level l.  x_prepped: the 16-bit operand
// of the level already holds x (written by the launch that produced it);
// prep_after: the caller's next product is of x, so the last projection writes
// its operand, and *prepped_out tells whether it did.
static rc_status cheb_smooth(rc_ctx* c, int l, double* x, const double* b, bool x_zero, bool x_prepped = false,
                             bool prep_after = false, bool* prepped_out = nullptr) {
  if (prepped_out) *prepped_out = false;
  const Curve& cv = level_curve(c, l);
  Cons& K = level_cons(c, l);
  MGLevelState& st = c->mg[l];
  hipStream_t s = c->stream;
  const int n = cv.nV, n3 = 3 * n;
  const double lmax = st.lmax, lmin = 0.2 * lmax;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (c->mg_weighted) {
    // weighted projector M = W - W C^T (C W C^T)^-1 C W (W = D^-1): M annihilates
    // range(C^T), so the residuals need no projection and each step takes one M.
    // r = base - A X is formed by the product's finish (the 16-bit block) and
    // x += d by the projector's last launch.
    Cons& Kw = level_cons_w(c, l);
    // the 16-bit block of the level; its operand is written by the projection
    // before each product (of d, or of x for the caller's next product)
    const LowpOp* lop = l < c->lowp_levels ? &level_lowp(c, l) : nullptr;
    const int deg = c->cheb_deg;
    auto residual = [&](const double* X, const double* base, bool prepped) -> rc_status {  // r = base - A X
      if (lop) return launch_lowp_apply(*lop, X, st.r, s, l == 0 ? &c->timer : nullptr, base, -1.0, prepped);
      RC_TRY(apply_level(c, l, X, st.t));
      if (base != st.r) vec_copy(base, st.r, n3, s);
      vec_axpby(-1.0, st.t, 1.0, st.r, n3, s);
      return RC_OK;
    };
    // the operand the k-th projection (k = 0 .. deg - 1) writes: d when a residual of d follows, else x
    auto prep_op = [&](int k) -> const LowpOp* { return (k + 1 < deg || prep_after) ? lop : nullptr; };
    if (x_zero) {  // d = M b / theta, x = d
      cons_project_w(c, cv, Kw, st.w, b, st.d, 1.0 / theta, 0.0, nullptr, x, true, prep_op(0), deg == 1);
      if (deg > 1) RC_TRY(residual(st.d, b, lop != nullptr));
    } else {  // r = b - A x, d = M r / theta, x += d
      RC_TRY(residual(x, b, x_prepped && lop != nullptr));
      cons_project_w(c, cv, Kw, st.w, st.r, st.d, 1.0 / theta, 0.0, nullptr, x, false, prep_op(0), deg == 1);
      if (deg > 1) RC_TRY(residual(st.d, st.r, lop != nullptr));
    }
    for (int k = 1; k < deg; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      // d = c1 d + c2 M r, x += d
      cons_project_w(c, cv, Kw, st.w, st.r, st.d, 2.0 * rn / delta, rn * rho, st.d, x, false, prep_op(k),
                     k + 1 == deg);
      rho = rn;
      if (k + 1 < deg) RC_TRY(residual(st.d, st.r, lop != nullptr));
    }
    if (prepped_out) *prepped_out = prep_after && lop != nullptr;
    return RC_OK;
  }
  if (x_zero) {
    vec_copy(b, st.r, n3, s);
    hipMemsetAsync(x, 0, sizeof(double) * n3, s);
  } else {
    RC_TRY(apply_level(c, l, x, st.r));
    vec_axpby(1.0, b, -1.0, st.r, n3, s);
    cons_project(c, cv, K, st.r, st.r);
  }
  hipLaunchKernelGGL(k_cheb_init, dim3(cdiv(n3, 256)), dim3(256), 0, s, st.r, st.diag, 1.0 / theta, n, st.d);
  cons_project(c, cv, K, st.d, st.d);
  const int deg = c->cheb_deg;
  for (int k = 0; k < deg; ++k) {
    vec_axpby(1.0, st.d, 1.0, x, n3, s);
    if (k == deg - 1) break;
    RC_TRY(apply_level(c, l, st.d, st.t));
    cons_project(c, cv, K, st.t, st.t);
    vec_axpby(-1.0, st.t, 1.0, st.r, n3, s);
    const double rn = 1.0 / (2.0 * sigma - rho);
    // d = c1 d + c2 P D^-1 r (d is already in range(P))
    hipLaunchKernelGGL(k_cheb_update, dim3(cdiv(n3, 256)), dim3(256), 0, s, st.r, st.diag, rn * rho,
                       2.0 * rn / delta, n, st.d);
    cons_project(c, cv, K, st.d, st.d);
    rho = rn;
  }
  return RC_OK;
}

static rc_status vcycle(rc_ctx* c, int l, const double* b, double* x) {
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  if (l == nl - 1) {
    dense_solve(c, c->coarse, b, x);
    return RC_OK;
  }
  const Curve& cv = level_curve(c, l);
  Cons& K = level_cons(c, l);
  MGLevelState& st = c->mg[l];
  const int n3 = 3 * cv.nV;
  const bool lp = l < c->lowp_levels;
  bool prepped = false;
  RC_TRY(cheb_smooth(c, l, x, b, true, false, lp, &prepped));
  if (lp) {  // t = b - A x
    RC_TRY(launch_lowp_apply(level_lowp(c, l), x, st.t, s, l == 0 ? &c->timer : nullptr, b, -1.0, prepped));
  } else {
    RC_TRY(apply_level(c, l, x, st.t));
    vec_axpby(1.0, b, -1.0, st.t, n3, s);
  }
  cons_project(c, cv, K, st.t, st.t);
  Level& C = *c->levels[l + 1];
  MGLevelState& sc = c->mg[l + 1];
  hipLaunchKernelGGL(k_restrict, dim3(cdiv(C.curve.nV, 256)), dim3(256), 0, s, C.restr_off, C.restr_idx, C.prolong,
                     C.curve.nV, st.t, sc.b);
  // With the weighted smoother every use of the coarse right-hand side (M b, M (b - A x), the
  // Euclidean P of the coarse residual, and the coarsest level's saddle solve X b) annihilates
  // range(C^T) of the coarse level, so projecting it first would not change the V-cycle.
  if (!c->mg_weighted) cons_project(c, C.curve, C.cons, sc.b, sc.b);
  RC_TRY(vcycle(c, l + 1, sc.b, sc.x));
  hipLaunchKernelGGL(k_prolong, dim3(cdiv(cv.nV, 256)), dim3(256), 0, s, C.prolong, cv.nV, sc.x, st.t);
  // x += P J x_c (writing the operand of the smoother's first product, A x)
  const bool xp = cons_project(c, cv, K, st.t, st.t, x, (lp && c->mg_weighted) ? &level_lowp(c, l) : nullptr, true);
  RC_TRY(cheb_smooth(c, l, x, b, false, xp));
  return RC_OK;
}

// ---------------------------------------------------------------------------
// projected PCG:  P Abar P y = P b, y in range(P)   (App. B.3.3)
// ---------------------------------------------------------------------------
static rc_status precondition(rc_ctx* c, int kind, const double* r, double* z) {
  if (kind == RC_SOLVE_PCG_MG || kind == RC_SOLVE_PCG_LEARNED) {
    MGLevelState& st = c->mg[0];
    return vcycle(c, 0, r, z);  // the V-cycle only reads its right-hand side
  }
  vec_scale_diag_inv(r, c->diag, z, c->nV, c->stream);
  cons_project(c, c->curve, c->cons, z, z);
  return RC_OK;
}

// x += a p, r -= a q with a = rz / pq read on the device (a = 0 when pq <= 0)
__global__ void k_pcg_xr(const double* __restrict__ rz, const double* __restrict__ pq, const double* __restrict__ p,
                         const double* __restrict__ q, double* __restrict__ x, double* __restrict__ r, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = pq[0] > 0.0 ? rz[0] / pq[0] : 0.0;
  x[i] += a * p[i];
  r[i] -= a * q[i];
}

// p = z + (rz_new / rz_old) p
__global__ void k_pcg_p(const double* __restrict__ rz_new, const double* __restrict__ rz_old,
                        const double* __restrict__ z, double* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = z[i] + (rz_new[0] / rz_old[0]) * p[i];
}

// With an absolute reference (rc_ctx::pcg_ref) the relative tolerance is capped at this: every solve
// still removes most of its right-hand side's rough part, to which the tangent-point energy is most
// sensitive at fine resolutions
constexpr double kPcgRefMaxTol = 0.02;

static rc_status pcg_solve(rc_ctx* c, const double* b, double* x, const rc_solve_opts& o, int* iters_out,
                           double* res_out) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV;
  const rc_dtype op = o.op_f64 ? RC_F64 : c->dtype;
  const bool lowp = c->lowp_levels > 0;
  double *r = c->r, *z = c->z, *p = c->p, *q = c->q;
  // Krylov operator: the assembled FP32 block (lowp_outer 1), the finest 16-bit
  // block (lowp_outer 2, internal: loose projection-increment solves only), or
  // the matrix-free operator in precision op
  auto apply_op = [&](const double* X, double* Y) -> rc_status {
    if (lowp && c->lowp_outer == 1 && o.lowp_outer == 1) return launch_lowp_apply32(c->lowp, X, Y, s, &c->timer);
    if (lowp && o.lowp_outer == 2) return launch_lowp_apply(c->lowp, X, Y, s, nullptr);
    return apply_A(c, c->curve, X, Y, op);
  };
  c->last_sweeps = 0;
  cons_project(c, c->curve, c->cons, b, c->tmp2);  // P b
  vec_dot(c->tmp2, c->tmp2, n3, c->red, c->scal, s);
  double bb;
  RC_TRY(fetch(c, c->scal, &bb, 1));
  const double bn = std::sqrt(bb);
  c->last_bnorm = bn;
  hipMemsetAsync(x, 0, sizeof(double) * n3, s);
  *iters_out = 0;
  *res_out = 0.0;
  if (!(bn > 0)) return RC_OK;
  const double tol = c->pcg_ref > bn ? std::min(kPcgRefMaxTol, o.tol * c->pcg_ref / bn) : o.tol;
  vec_copy(c->tmp2, r, n3, s);
  int it = 0;
  double res = 1.0, res_sweep = 1.0;  // residual at the start of the current sweep
  bool converged = false;
  const bool watch = o.fallback_after > 0 && o.solver == RC_SOLVE_PCG_LEARNED;
  int growing = 0;  // consecutive iterations with a growing recurrence residual
  // with an inexact Krylov operator (FP32 block or FP32 pairs) a sweep ends
  // early when its recurrence residual stalls at the operator's floor (less
  // than halved over 5 iterations): the next sweep restarts from the FP64
  // true residual
  const bool inexact = (lowp && c->lowp_outer == 1 && o.lowp_outer == 1) || op != RC_F64;
  double window[6];
  // the recurrence scalars stay on the device (scal[5] = p.q, scal[6] = r.r, r.z alternating in
  // scal[10], scal[11]); the host reads p.q and r.r once per iteration for the stopping tests
  double* const sc = c->scal;
  int par = 0;
  while (it < o.max_iter && !converged) {
    RC_TRY(precondition(c, o.solver, r, z));
    vec_copy(z, p, n3, s);
    vec_dot(r, z, n3, c->red, sc + 10 + par, s);
    int since = 0;
    while (it < o.max_iter) {
      RC_TRY(apply_op(p, q));
      cons_project(c, c->curve, c->cons, q, q);
      vec_dot(p, q, n3, c->red, sc + 5, s);
      hipLaunchKernelGGL(k_pcg_xr, dim3(cdiv(n3, 256)), dim3(256), 0, s, (const double*)(sc + 10 + par),
                         (const double*)(sc + 5), (const double*)p, (const double*)q, x, r, n3);
      vec_dot(r, r, n3, c->red, sc + 6, s);
      double h[2];
      RC_TRY(fetch(c, sc + 5, h, 2));
      const double pq = h[0], rr = h[1];
      if (!(pq > 0)) {  // x and r were left unchanged
        if (trace_on()) fprintf(stderr, "[rc pcg] it %d breakdown p.q = %.3e\n", it, pq);
        break;
      }
      ++it;
      ++since;
      const double res_prev = res;
      res = std::sqrt(rr) / bn;
      if (trace_on()) fprintf(stderr, "[rc pcg] it %d rec-res %.3e\n", it, res);
      const bool stalled = inexact && since > 5 && res > 0.5 * window[(since - 5) % 6];
      window[since % 6] = res;
      growing = res > res_prev ? growing + 1 : 0;
      if (watch && growing >= o.fallback_after) {
        *iters_out = it;
        *res_out = res;
        set_error("projected PCG: the residual kept growing");
        return RC_ERR_NOT_CONVERGED;
      }
      if (res < std::max(tol, o.inner_tol * res_sweep) || (o.replace_every > 0 && since >= o.replace_every) ||
          stalled) {
        // true residual r = P (b - Abar x) (FP64); restart the recurrence from it
        // a loose solve (tol >= 1e-4) checks with its own operator
        if (tol >= 1e-4) RC_TRY(apply_op(x, c->tmp));
        else RC_TRY(apply_A(c, c->curve, x, c->tmp, RC_F64));
        vec_copy(b, r, n3, s);
        vec_axpby(-1.0, c->tmp, 1.0, r, n3, s);
        cons_project(c, c->curve, c->cons, r, r);
        vec_dot(r, r, n3, c->red, c->scal, s);
        double rt;
        RC_TRY(fetch(c, c->scal, &rt, 1));
        res = std::sqrt(rt) / bn;
        res_sweep = res;
        ++c->last_sweeps;
        if (trace_on()) fprintf(stderr, "[rc pcg] it %d TRUE-res %.3e\n", it, res);
        if (res < tol) converged = true;
        break;
      }
      RC_TRY(precondition(c, o.solver, r, z));
      vec_dot(r, z, n3, c->red, sc + 10 + (par ^ 1), s);
      hipLaunchKernelGGL(k_pcg_p, dim3(cdiv(n3, 256)), dim3(256), 0, s, (const double*)(sc + 10 + (par ^ 1)),
                         (const double*)(sc + 10 + par), (const double*)z, p, n3);
      par ^= 1;
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
// entry points used by the C ABI
// ---------------------------------------------------------------------------
static rc_status prepare_solver_body(rc_ctx* c, const double* gamma, const rc_solve_opts& o) {
  if (o.solver < RC_SOLVE_DENSE || o.solver > RC_SOLVE_MG_FMG || o.solver == 3) {
    set_error("solve options: unknown solver kind");
    return RC_ERR_ARG;
  }
  if (o.lowp < 0 || o.lowp > 2) {
    set_error("solve options: lowp must be 0 (off), 1 (BF16) or 2 (FP16)");
    return RC_ERR_ARG;
  }
  if (o.lowp_outer < 0 || o.lowp_outer > 1) {
    set_error("solve options: lowp_outer must be 0 (matrix-free) or 1 (assembled FP32)");
    return RC_ERR_ARG;
  }
  c->lowp_levels = 0;
  if (o.bct_theta < 0.0 ||
      (o.bct_theta > 0.0 &&
       (o.lowp || (o.solver != RC_SOLVE_PCG_MG && o.solver != RC_SOLVE_PCG_LEARNED && o.solver != RC_SOLVE_MG_FMG)))) {
    set_error("solve options: the block-cluster-tree operator (bct_theta > 0) serves the multigrid solver "
              "without the precision path");
    return RC_ERR_ARG;
  }
  c->bct_theta = o.bct_theta;
  c->bct_min_v = std::max(1, o.bct_min_vertices);
  c->curve.hbvh = nullptr;
  c->curve.hbct = nullptr;
  for (auto& L : c->levels)
    if (L) {
      L->curve.hbvh = nullptr;
      L->curve.hbct = nullptr;
    }
  RC_TRY(load_geometry(c, gamma));
  const bool multigrid =
      o.solver == RC_SOLVE_PCG_MG || o.solver == RC_SOLVE_PCG_LEARNED || o.solver == RC_SOLVE_MG_FMG;
  if (!multigrid) RC_TRY(cons_prepare(c, c->curve, c->cons, gamma));  // (the multigrid set-up does every level)
  if (o.solver == RC_SOLVE_DENSE) return dense_prepare(c, c->curve, c->cons, c->dense, gamma);
  c->lowp_fmt = o.lowp;
  c->lowp_band = o.lowp_band;
  c->lowp_outer = o.lowp_outer;
  c->mg_learned = false;
  c->mg_cg = o.solver == RC_SOLVE_MG_FMG;
  if (o.solver == RC_SOLVE_PCG_LEARNED) {
    if (!c->mlp) {
      set_error("learned smoother: no MLP attached (rc_learned_attach)");
      return RC_ERR_ARG;
    }
    RC_TRY(learn_prepare_levels(c, o.mg_min_vertices));
    c->mg_learned = true;
  }
  if (o.solver == RC_SOLVE_PCG_MG || o.solver == RC_SOLVE_PCG_LEARNED || o.solver == RC_SOLVE_MG_FMG) {
    if (c->mg_min != o.mg_min_vertices) {
      mg_free(c);
      c->mg_min = o.mg_min_vertices;
    }
    c->cheb_deg = o.cheb_degree;
    RC_TRY(mg_build(c));
    // the precision path covers the finest level and every smoothed level
    // with at least lowp_min_vertices vertices
    const int nl = (int)c->levels.size();
    int nlow = 0;
    if (o.lowp) {
      nlow = 1;
      while (nlow < nl - 1 && level_curve(c, nlow).nV >= o.lowp_min_vertices) ++nlow;
    }
    c->lowp_levels = nlow;
    RC_TRY(mg_prepare(c, gamma));
    RC_TRY(load_geometry(c, gamma));
    // a single-level hierarchy has no smoothed level: assemble the finest block here
    if (o.lowp && nl == 1)
      RC_TRY(launch_assemble_lowp(c->curve, c->lowp, o.lowp, o.lowp_band, o.lowp_outer == 1, c->alpha, c->beta,
                                  nullptr, c->stream));
    return RC_OK;
  }
  if (o.lowp) {
    RC_TRY(launch_assemble_lowp(c->curve, c->lowp, o.lowp, o.lowp_band, o.lowp_outer == 1, c->alpha, c->beta,
                                c->diag, c->stream));
    c->lowp_levels = 1;
    return RC_OK;
  }
  return launch_sobolev(c->curve, c->alpha, c->beta, c->dtype, c->x, c->tmp, c->diag, c->stream);
}

// The solver's set-up, then one wait for the device: a constraint factorisation that failed anywhere in
// the hierarchy is reported here (before any error it caused downstream).
rc_status prepare_solver(rc_ctx* c, const double* gamma, const rc_solve_opts& o) {
  const rc_status st = prepare_solver_body(c, gamma, o);
  const std::string msg = last_error();
  const rc_status sc = setup_check(c);
  if (st != RC_OK || sc != RC_OK) mg_reset_power(c);
  if (st == RC_ERR_ARG || st == RC_ERR_UNSUPPORTED) {  // an option or size the set-up rejected
    set_error(msg);
    return st;
  }
  if (sc != RC_OK) return sc;
  if (st != RC_OK) set_error(msg);
  return st;
}

// Prepare and solve; the multilevel preconditioners fall back to multigrid
// when their solve diverges or runs out of iterations (o then holds the
// multigrid options, for the solves that follow at the same curve).
rc_status solve_gradient(rc_ctx* c, const double* gamma, const double* rhs, double* out, rc_solve_opts& o,
                         int* iters, double* res, int* fell) {
  *fell = 0;
  RC_TRY(prepare_solver(c, gamma, o));
  rc_status st = solve_prepared(c, rhs, out, o, iters, res);
  if (st == RC_ERR_NOT_CONVERGED && o.fallback_after > 0 && o.solver == RC_SOLVE_PCG_LEARNED) {
    if (trace_on()) fprintf(stderr, "[rc pcg] falling back to multigrid after %d iterations\n", *iters);
    const int spent = *iters;
    o.solver = RC_SOLVE_PCG_MG;
    *fell = 1;
    RC_TRY(prepare_solver(c, gamma, o));
    st = solve_prepared(c, rhs, out, o, iters, res);
    *iters += spent;
  }
  return st;
}

// ---------------------------------------------------------------------------
// The paper's standalone multigrid (App. B.3.1): full-multigrid
// initialisation, then V-cycles with a conjugate-gradient smoother on each
// level's projected system P A_l P y = P b (App. B.3.3), until the relative
// residual |P (b - A x)| / |P b| reaches the tolerance.  The smoother runs
// with its scalars on the device (no host reads); being nonlinear it serves
// this stationary iteration, not a Krylov preconditioner.
// ---------------------------------------------------------------------------
static constexpr int kCgScal = 32;  // scal[32 + 6 l ...]: the level's r.r (two slots), p.q, e.r, e.Ae

// x += (num / den) e with the two scalars on the device (no step when den <= 0)
__global__ void k_axpy_ratio(const double* __restrict__ num, const double* __restrict__ den,
                             const double* __restrict__ e, double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = den[0] > 0.0 ? num[0] / den[0] : 0.0;
  x[i] += a * e[i];
}

// `steps` CG steps on P A_l P y = P b from x (in range(P)); scratch st.r, st.d, st.t.
static rc_status cg_smooth(rc_ctx* c, int l, double* x, const double* b, int steps) {
  const Curve& cv = level_curve(c, l);
  Cons& K = level_cons(c, l);
  MGLevelState& st = c->mg[l];
  hipStream_t s = c->stream;
  const int n3 = 3 * cv.nV;
  double* sc = c->scal + kCgScal + 6 * l;
  RC_TRY(apply_level(c, l, x, st.t));
  vec_copy(b, st.r, n3, s);
  vec_axpby(-1.0, st.t, 1.0, st.r, n3, s);
  cons_project(c, cv, K, st.r, st.r);  // r = P (b - A x)
  vec_copy(st.r, st.d, n3, s);
  vec_dot(st.r, st.r, n3, c->red, sc, s);
  int par = 0;
  for (int k = 0; k < steps; ++k) {
    RC_TRY(apply_level(c, l, st.d, st.t));
    cons_project(c, cv, K, st.t, st.t);  // q = P A p
    vec_dot(st.d, st.t, n3, c->red, sc + 2, s);
    hipLaunchKernelGGL(k_pcg_xr, dim3(cdiv(n3, 256)), dim3(256), 0, s, (const double*)(sc + par),
                       (const double*)(sc + 2), (const double*)st.d, (const double*)st.t, x, st.r, n3);
    if (k + 1 == steps) break;
    vec_dot(st.r, st.r, n3, c->red, sc + (par ^ 1), s);
    hipLaunchKernelGGL(k_pcg_p, dim3(cdiv(n3, 256)), dim3(256), 0, s, (const double*)(sc + (par ^ 1)),
                       (const double*)(sc + par), (const double*)st.r, st.d, n3);
    par ^= 1;
  }
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// x <- one V-cycle on level l for right-hand side b from the guess x.
static rc_status vcycle_cg(rc_ctx* c, int l, const double* b, double* x, int steps) {
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  if (l == nl - 1) {
    dense_solve(c, c->coarse, b, x);
    return RC_OK;
  }
  const Curve& cv = level_curve(c, l);
  Cons& K = level_cons(c, l);
  MGLevelState& st = c->mg[l];
  const int n3 = 3 * cv.nV;
  RC_TRY(cg_smooth(c, l, x, b, steps));
  RC_TRY(apply_level(c, l, x, st.t));
  vec_copy(b, st.r, n3, s);
  vec_axpby(-1.0, st.t, 1.0, st.r, n3, s);
  cons_project(c, cv, K, st.r, st.r);  // r = P (b - A x)
  Level& C = *c->levels[l + 1];
  MGLevelState& sc = c->mg[l + 1];
  hipLaunchKernelGGL(k_restrict, dim3(cdiv(C.curve.nV, 256)), dim3(256), 0, s, C.restr_off, C.restr_idx, C.prolong,
                     C.curve.nV, st.r, sc.b);
  hipLaunchKernelGGL(k_fill, dim3(cdiv(3 * C.curve.nV, 256)), dim3(256), 0, s, sc.x, 3 * C.curve.nV, 0.0);
  RC_TRY(vcycle_cg(c, l + 1, sc.b, sc.x, steps));
  hipLaunchKernelGGL(k_prolong, dim3(cdiv(cv.nV, 256)), dim3(256), 0, s, C.prolong, cv.nV, sc.x, st.t);
  cons_project(c, cv, K, st.t, st.t);  // e = P J x_c
  // the correction's step minimises the A-norm error along e: x += (e.r / e.A e) e (the rediscretised
  // coarse operators over-correct, and the unit step diverges)
  double* scl = c->scal + kCgScal + 6 * l;
  RC_TRY(apply_level(c, l, st.t, st.d));
  cons_project(c, cv, K, st.d, st.d);
  vec_dot(st.t, st.r, n3, c->red, scl + 3, s);
  vec_dot(st.t, st.d, n3, c->red, scl + 4, s);
  hipLaunchKernelGGL(k_axpy_ratio, dim3(cdiv(n3, 256)), dim3(256), 0, s, (const double*)(scl + 3),
                     (const double*)(scl + 4), (const double*)st.t, x, n3);
  RC_TRY(cg_smooth(c, l, x, b, steps));
  RC_HIP(hipGetLastError());
  return RC_OK;
}

static rc_status fmg_solve(rc_ctx* c, const double* b, double* x, const rc_solve_opts& o, int* iters_out,
                           double* res_out) {
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  const int n3 = 3 * c->nV, steps = std::max(1, o.cheb_degree);
  const rc_dtype op = o.op_f64 ? RC_F64 : c->dtype;
  *iters_out = 0;
  *res_out = 0.0;
  if (kCgScal + 6 * nl > 128) {
    set_error("standalone multigrid: too many levels for the smoother's device scalars");
    return RC_ERR_UNSUPPORTED;
  }
  // finest right-hand side P b, restricted level by level (each level's own projection first)
  double* b0 = c->tmp2;
  cons_project(c, c->curve, c->cons, b, b0);
  vec_dot(b0, b0, n3, c->red, c->scal, s);
  double bb;
  RC_TRY(fetch(c, c->scal, &bb, 1));
  const double bn = std::sqrt(bb);
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n3, 256)), dim3(256), 0, s, x, n3, 0.0);
  if (!(bn > 0)) return RC_OK;
  for (int l = 1; l < nl; ++l) {
    const double* bf = l == 1 ? b0 : c->mg[l - 1].b;
    Level& C = *c->levels[l];
    if (l > 1) {
      const Curve& fv = level_curve(c, l - 1);
      cons_project(c, fv, level_cons(c, l - 1), c->mg[l - 1].b, c->mg[l - 1].b);
    }
    hipLaunchKernelGGL(k_restrict, dim3(cdiv(C.curve.nV, 256)), dim3(256), 0, s, C.restr_off, C.restr_idx,
                       C.prolong, C.curve.nV, bf, c->mg[l].b);
  }
  // direct solve on the coarsest level, then prolong and smooth level by level
  double* xc = nl == 1 ? x : c->mg[nl - 1].x;
  const double* bc = nl == 1 ? b0 : c->mg[nl - 1].b;
  if (nl == 1) {
    set_error("standalone multigrid: the curve has no coarser level (raise n or lower mg_min_vertices)");
    return RC_ERR_UNSUPPORTED;
  }
  dense_solve(c, c->coarse, bc, xc);
  for (int l = nl - 2; l >= 0; --l) {
    const Curve& cv = level_curve(c, l);
    double* xl = l == 0 ? x : c->mg[l].x;
    const double* bl = l == 0 ? b0 : c->mg[l].b;
    hipLaunchKernelGGL(k_prolong, dim3(cdiv(cv.nV, 256)), dim3(256), 0, s, c->levels[l + 1]->prolong, cv.nV,
                       c->mg[l + 1].x, xl);
    cons_project(c, cv, level_cons(c, l), xl, xl);
    RC_TRY(cg_smooth(c, l, xl, bl, steps));
  }
  // V-cycles in correction form: the residual r = P (b - A x) with the operator in precision op,
  // a V-cycle (the levels' own operators) from zero for A e = r, x += e; so the cycles converge in
  // that precision even when the levels' products are FP32
  int cycles = 0;
  double res = 1.0;
  double *r = c->r, *e = c->z;
  for (;;) {
    RC_TRY(apply_A(c, c->curve, x, c->tmp, op));
    vec_copy(b0, r, n3, s);
    vec_axpby(-1.0, c->tmp, 1.0, r, n3, s);
    cons_project(c, c->curve, c->cons, r, r);
    vec_dot(r, r, n3, c->red, c->scal, s);
    double rr;
    RC_TRY(fetch(c, c->scal, &rr, 1));
    res = std::sqrt(rr) / bn;
    if (trace_on()) fprintf(stderr, "[rc fmg] cycle %d res %.3e\n", cycles, res);
    if (!(res >= o.tol) || cycles >= o.max_iter) break;
    hipLaunchKernelGGL(k_fill, dim3(cdiv(n3, 256)), dim3(256), 0, s, e, n3, 0.0);
    RC_TRY(vcycle_cg(c, 0, r, e, steps));
    vec_axpby(1.0, e, 1.0, x, n3, s);
    ++cycles;
  }
  *iters_out = cycles;
  *res_out = res;
  if (!(res < o.tol)) {
    set_error("standalone multigrid did not reach the tolerance");
    return RC_ERR_NOT_CONVERGED;
  }
  return RC_OK;
}

// The solve of the projected system for the prepared solver kind.
static rc_status solve_projected(rc_ctx* c, const double* b, double* x, const rc_solve_opts& o, int* iters,
                                 double* res) {
  if (o.solver == RC_SOLVE_MG_FMG) return fmg_solve(c, b, x, o, iters, res);
  return pcg_solve(c, b, x, o, iters, res);
}

rc_status solve_prepared(rc_ctx* c, const double* rhs, double* out, const rc_solve_opts& o, int* iters,
                         double* res) {
  if (o.solver == RC_SOLVE_DENSE) {
    dense_solve(c, c->dense, rhs, out);
    *iters = 0;
    *res = 0.0;
    return sync(c);
  }
  return solve_projected(c, rhs, out, o, iters, res);
}

// Projection increment for the violation phi (external order): eq.
// ConstraintSaddlePointProblem, through eq. SaddleSolutionTransformation on
// the PCG paths (z with C z = -phi, y from the projected system with
// right-hand side Abar z, x = z - y; any particular solution z gives the same
// x, the minimum-norm one C^T (C C^T)^-1 (-phi) without pinned vertices).
static rc_status projection_increment(rc_ctx* c, const double* phi, double* x, const rc_solve_opts& o, int* iters) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV, k = c->cons.k;
  *iters = 0;
  if (o.solver == RC_SOLVE_DENSE) {
    dense_increment(c, c->dense, phi, x);
    return RC_OK;
  }
  hipLaunchKernelGGL(k_negate, dim3(cdiv(k, 256)), dim3(256), 0, s, phi, c->phi + k, k);
  cons_min_norm(c, c->phi + k, c->zmin, c->inc);
  if (o.lowp_outer == 2 && c->lowp_levels > 0) RC_TRY(launch_lowp_apply(c->lowp, c->zmin, c->inc, s, nullptr));
  else RC_TRY(apply_A(c, c->curve, c->zmin, c->inc, o.op_f64 ? RC_F64 : c->dtype));
  double res = 0.0;
  rc_status st = solve_projected(c, c->inc, c->x, o, iters, &res);
  if (st != RC_OK && st != RC_ERR_NOT_CONVERGED) return st;
  vec_copy(c->zmin, x, n3, s);
  vec_axpby(-1.0, c->x, 1.0, x, n3, s);
  return RC_OK;
}

rc_status line_search(rc_ctx* c, double* gamma, double E0, const double* dE, const double* g, const rc_ls_opts& ls,
                      const rc_solve_opts& so, LsResult* out) {
  hipStream_t s = c->stream;
  const int n3 = 3 * c->nV, k = c->cons.k;
  if (!(ls.bh_theta >= 0.0 && ls.bh_theta < 0.5)) {
    set_error("line search options: bh_theta must be 0 or lie in (0, 0.5)");
    return RC_ERR_ARG;
  }
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
  // per-row projection tolerances relative to the mean edge length at gamma
  std::vector<double> phi_h(std::max(k, 1));
  double Ltot = 0.0;
  {
    std::vector<double> ga(4 * (size_t)c->nE);
    RC_TRY(load_geometry(c, gamma));
    RC_HIP(hipMemcpyAsync(ga.data(), c->curve.gd.a, sizeof(double) * 4 * c->nE, hipMemcpyDeviceToHost, s));
    RC_TRY(sync(c));
    for (int I = 0; I < c->nE; ++I) Ltot += ga[4 * I + 3];
  }
  const double lbar = Ltot / std::max(1, c->nE);
  const Cons& K = c->cons;
  double tau = ls.tau0;
  if (ls.ccd) {
    // Sec. 4.4: start at 2/3 of the first collision time tau_max of gamma - tau g/|g|, sought
    // up to 1.5 tau0 (so that without a collision the search starts at tau0); any length below
    // tau_max moves the curve without a self-intersection
    const double gn = std::sqrt(h[0]);
    RC_TRY(c->ccd.ensure(c->nE));
    RC_TRY(launch_first_collision(c->curve, gamma, g, 1.5 * ls.tau0 / gn, c->ccd, c->ccd.t, s));
    double tc;
    RC_TRY(fetch(c, c->ccd.t, &tc, 1));
    out->tau_max = std::isfinite(tc) ? tc * gn : INFINITY;
    tau = (2.0 / 3.0) * std::min(out->tau_max, 1.5 * ls.tau0);
  }
  bool any_projected = false;  // some trial reached the constraint tolerance
  // Sec. 4.4 leaves the accuracy of the approximate Newton iteration's saddle solves open: the first
  // increment of a trial is solved to the relative tolerance, the later ones (whose right-hand sides
  // shrink with the violation) to the same absolute accuracy but at least to kPcgRefMaxTol relative, so
  // that their sum is about as accurate as the first; C x = -Phi holds for each whatever the solve's
  // accuracy
  struct RefReset {
    rc_ctx* c;
    ~RefReset() { c->pcg_ref = 0.0; }
  } ref_reset{c};
  for (int bt = 0; bt <= ls.max_backtracks; ++bt) {
    vec_trial(gamma, g, c->scal + 16, tau, c->trial, n3, s);
    bool ok = (k == 0);
    int it = 0;
    c->pcg_ref = 0.0;
    for (; k > 0 && it <= ls.max_proj_iter; ++it) {
      cons_values(c, c->trial, c->phi);
      RC_TRY(fetch(c, c->phi, phi_h.data(), k));
      bool done = true;
      double worst = 0.0;  // max |Phi_i| / tol_i
      for (int i = 0; i < k; ++i) {
        double tol = ls.proj_tol * lbar;
        if (K.bary && i < 3) tol *= Ltot;             // barycenter rows carry units of length^2
        else if (K.total && i == 3 * K.bary) tol *= Ltot / lbar;  // total length: relative to L
        else if (i >= K.ext_tg && i < K.ext_tg + 2 * K.ntg) tol = ls.proj_tol;  // tangent rows: dimensionless
        if (!std::isfinite(phi_h[i]) || std::fabs(phi_h[i]) > tol) done = false;
        worst = std::max(worst, std::fabs(phi_h[i]) / tol);
      }
      if (trace_on()) fprintf(stderr, "[rc ls] tau %.3e projection %d: max |Phi|/tol %.3e\n", tau, it, worst);
      if (done) {
        ok = true;
        break;
      }
      if (it == ls.max_proj_iter) break;
      int pit = 0;
      RC_TRY(load_geometry(c, gamma));
      rc_solve_opts po = so;
      if (ls.proj_solve_tol > 0) {
        // a loose increment solve: its operator runs in the context's precision
        // (C x = -Phi holds whatever the solve's accuracy)
        po.tol = ls.proj_solve_tol;
        if (ls.proj_solve_tol >= 1e-4) {
          po.op_f64 = 0;
          if (c->lowp_levels > 0) po.lowp_outer = 2;  // the finest 16-bit block, assembled at gamma
        }
      }
      c->last_bnorm = 0.0;  // set by the PCG solvers only
      RC_TRY(projection_increment(c, c->phi, c->dx, po, &pit));
      if (it == 0) c->pcg_ref = c->last_bnorm;
      out->proj_solve_iters += pit;
      vec_axpby(1.0, c->dx, 1.0, c->trial, n3, s);
    }
    any_projected |= ok;
    if (ok) {
      RC_TRY(load_geometry(c, c->trial));
      if (ls.bh_theta > 0.0)  // the Barnes-Hut energy (its differential goes to the free PCG buffer q)
        RC_TRY(launch_bh(c->curve, c->bvh, c->alpha, c->beta, ls.bh_theta, kStepBhLeaf, c->scal + 18, c->q, s,
                         ls.bh_refit != 0 && c->bvh.n_nodes > 0));
      else
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
  out->backtracks = ls.max_backtracks;
  if (!any_projected) {
    set_error("constraint projection did not reach its tolerance at any step length");
    return RC_ERR_PROJECTION;
  }
  set_error("line search found no admissible step");
  return RC_ERR_LINESEARCH;
}

// ---------------------------------------------------------------------------
// Learned smoother weights (k_learn.hip): the hierarchy of the multigrid
// V-cycle, one closed loop numbered along itself on every level; features and
// FP64 diagonals of every level stacked finest first (level l at row
// learn_off[l]), the network's output, and the regression targets.
// ---------------------------------------------------------------------------
void learn_free(rc_ctx* c) {
  dfree(c->learn_diag);
  dfree(c->learn_scratch);
  dfree(c->learn_X);
  dfree(c->learn_Y);
  c->learn_cap = 0;
  c->learn_nmin = -1;
}

// Hierarchy for coarsest size n_min; every level must be one closed loop
// whose vertices are numbered along it (checked once per hierarchy).
rc_status learn_prepare_levels(rc_ctx* c, int n_min) {
  if (n_min < 4) {
    set_error("learned smoother: n_min must be at least 4");
    return RC_ERR_ARG;
  }
  if (c->mg_min != n_min) {
    RC_TRY(sync(c));
    mg_free(c);
    c->mg_min = n_min;
  }
  if (c->mg_built && c->learn_nmin == n_min) return RC_OK;
  const int n0 = c->curve.nV;
  bool ok = c->curve.chain && c->curve.nE == n0 && n0 >= 3;
  for (int i = 0; ok && i < n0; ++i)
    ok = c->curve.h_edges[2 * i] == i && c->curve.h_edges[2 * i + 1] == (i + 1) % n0;
  if (!ok) {
    set_error("learned smoother: needs one closed loop with edges (i, i + 1 mod n)");
    return RC_ERR_UNSUPPORTED;
  }
  RC_TRY(mg_build(c));
  const int nl = (int)c->levels.size();
  for (int l = 0; l < nl; ++l) {
    std::vector<Chain> chs = chains_of(level_curve(c, l));
    bool good = chs.size() == 1 && chs[0].loop;
    for (int i = 0; good && i < (int)chs[0].verts.size(); ++i) good = chs[0].verts[i] == i;
    if (!good) {
      set_error("learned smoother: a level is not one loop numbered along itself");
      return RC_ERR_UNSUPPORTED;
    }
  }
  c->learn_off.assign(nl + 1, 0);
  for (int l = 0; l < nl; ++l) c->learn_off[l + 1] = c->learn_off[l] + level_curve(c, l).nV;
  const int N = c->learn_off[nl];
  if (N > c->learn_cap) {
    RC_TRY(sync(c));
    learn_free(c);
    RC_TRY(dalloc(&c->learn_diag, N));
    RC_TRY(dalloc(&c->learn_scratch, 9 * (size_t)n0 + 2));
    RC_TRY(dalloc(&c->learn_X, (size_t)kMlpIn * N));
    RC_TRY(dalloc(&c->learn_Y, N));
    c->learn_cap = N;
  }
  c->learn_N = N;
  c->learn_nmin = n_min;
  return RC_OK;
}

// Level curves at gamma (geometry loaded, finest last), and with X the
// features and FP64 diagonals of every level; with R (device float[N]) the
// targets T_v = r_v lambda_l from each level's dense FP64 operator A_l:
// r_v = sum_w |A_vw| / A_vv, lambda_l the largest eigenvalue of
// S = D_r^-1/2 A_l D_r^-1/2 (D_r = diag(r_v A_vv)) by kTargetPowerIts power
// steps from the alternating vector (close to the top eigenvector), their
// Rayleigh quotients a lower bound.
constexpr int kTargetPowerIts = 60;
rc_status learn_levels_at(rc_ctx* c, const double* gamma, int n_min, bool features, float* R) {
  RC_TRY(learn_prepare_levels(c, n_min));
  hipStream_t s = c->stream;
  const int nl = (int)c->levels.size();
  const double* g = gamma;
  for (int l = 1; l < nl; ++l) {
    Level& L = *c->levels[l];
    hipLaunchKernelGGL(k_gather_coarse, dim3(cdiv(L.curve.nV, 256)), dim3(256), 0, s, g, L.fine_of, L.curve.nV,
                       L.gamma);
    g = L.gamma;
  }
  double* dense = nullptr;
  if (R) {
    const size_t n0 = (size_t)c->curve.nV;
    if (n0 > 16384) {
      set_error("learned smoother targets: at most 16,384 vertices (dense FP64 level operators)");
      return RC_ERR_ARG;
    }
    RC_TRY(dalloc(&dense, n0 * n0 + 4 * n0));
  }
  rc_status st = RC_OK;
  for (int l = nl - 1; l >= 0 && st == RC_OK; --l) {  // finest last: its geometry stays loaded
    const Curve& cv = level_curve(c, l);
    const double* gl = l == 0 ? gamma : c->levels[l]->gamma;
    const int o = c->learn_off[l];
    st = launch_geometry(cv, gl, RC_F32, s);
    if (st == RC_OK && features) {
      hipMemsetAsync(c->learn_scratch, 0, sizeof(double) * 3 * cv.nV, s);  // a zero operand: only the diagonal
      st = launch_sobolev(cv, c->alpha, c->beta, RC_F64, c->learn_scratch, nullptr, c->learn_diag + o, s);
      if (st == RC_OK)
        st = launch_level_features(cv, gl, c->learn_diag + o, c->learn_scratch, c->learn_X + (size_t)kMlpIn * o, s);
    }
    if (st == RC_OK && R) {
      const int n = cv.nV;
      double* r = dense + (size_t)n * n;
      double* sc = r + n;
      double* x = sc + n;
      double* y = x + n;
      st = launch_assemble_dense(cv, c->alpha, c->beta, dense, s);
      if (st == RC_OK) st = launch_row_l1_ratio(dense, n, r, sc, s);
      if (st == RC_OK) st = launch_alternating(n, x, s);
      double lam = 0.0;
      for (int it = 0; st == RC_OK && it < kTargetPowerIts; ++it) {
        vec_dot(x, x, n, c->red, c->scal, s);
        st = launch_sym_scaled_mv(dense, sc, x, n, y, s);
        if (st != RC_OK) break;
        vec_dot(x, y, n, c->red, c->scal + 1, s);
        double h[2];
        st = fetch(c, c->scal, h, 2);
        if (st != RC_OK) break;
        lam = h[1] / h[0];  // Rayleigh quotient of x
        double h2;
        vec_dot(y, y, n, c->red, c->scal + 2, s);
        st = fetch(c, c->scal + 2, &h2, 1);
        if (st != RC_OK) break;
        vec_axpby(1.0 / std::sqrt(h2), y, 0.0, x, n, s);
      }
      if (st == RC_OK) {
        RC_HIP(hipMemcpyAsync(c->scal + 3, &lam, sizeof(double), hipMemcpyHostToDevice, s));
        st = launch_ratio_targets(r, c->scal + 3, n, R + o, s);
        if (st == RC_OK) st = sync(c);
      }
    }
  }
  if (dense) {
    const rc_status s2 = sync(c);
    dfree(dense);
    if (st == RC_OK) st = s2;
  }
  return st;
}

}  // namespace rc
