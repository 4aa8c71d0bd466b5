// Launchers of the FP64 vector, dense and constraint kernels (k_linalg.hip).
#pragma once

#include "rc_internal.h"

namespace rc {

// out[r] = X_r . Y_r for r < m (X_r = X + r ldx, Y_r = Y + r ldy); scratch >= dot_scratch_size(m)
void vec_dots(const double* X, int ldx, const double* Y, int ldy, int n, int m, double* scratch, double* out,
              hipStream_t s);
constexpr int kRedSets = 128;  // dot products the context's reduction scratch holds at once
int dot_scratch_size(int m);
// out[r mx + j] = X_j . Y_r for j < mx, r < my (rows ldx and ldy apart), in two launches; the same sums in
// the same order as vec_dots; scratch of dot_scratch_size(mx my).
void vec_gram(const double* X, int ldx, const double* Y, int ldy, int n, int mx, int my, double* scratch,
              double* out, hipStream_t s);
// out = gamma - tau g / sqrt(gg[0])
void vec_trial(const double* gamma, const double* g, const double* gg, double tau, double* out, int n,
               hipStream_t s);

// Tridiagonal systems, block-partitioned (see k_linalg.hip): kSpThreads
// threads per block of S = kSpThreads m rows, at most kSpMaxB blocks.
constexpr int kTriThreads = 1024, kTriWaves = kTriThreads / 64;
constexpr int kSpThreads = 256, kSpWaves = kSpThreads / 64, kSpMaxM = 16, kSpMaxB = 512;
struct TriBlocks {
  int n = 0;   // rows
  int S = 1;   // rows per block
  int B = 1;   // blocks (a single block when n <= kTriThreads)
  int m = 1;   // rows per thread
  int nr = 0;  // size of the reduced boundary system, 2 (B - 1)
};
TriBlocks tri_blocks(int n);
struct TriSys {
  TriBlocks L;
  const double *lo = nullptr, *uinv = nullptr, *c = nullptr;  // block-local factors l, 1/u and the couplings c
  const double *V = nullptr, *W = nullptr;                    // spikes [n] each
  const double* Rt = nullptr;                                 // inverse of the reduced system, transposed [nr][nr]
};
// Block-local factorisation, spikes (VW: [2 n], V then W) and the reduced
// inverse Rt; a, d, c: the rows' coefficients; lo, uinv: [n]; scratch: [2 n];
// info: device int, 0 on success, else 1 + a row with a non-positive pivot.
void tri_prepare(const double* a, const double* d, const double* c, const TriBlocks& L, double* lo, double* uinv,
                 double* VW, double* Rt, double* scratch, int* info, hipStream_t s);
// y_r = K^-1 rhs_r for m columns (ldr, ldy apart); g: [m n] and U: [m nr] scratch.
void tri_solve(const TriSys& T, const double* rhs, int ldr, double* y, int ldy, int m, double* g, double* U,
               hipStream_t s);
void dense_gemv(const double* A, const double* x, double* y, int n, hipStream_t s);

// constraint pieces
void cons_geometry(const double* gamma, const int2* edges, int nE, double* geo, hipStream_t s);
void cons_phi_edge(const double* geo, const double* x0, int nE, const double* len0, double* vals, double* phi_edges,
                   hipStream_t s);
void cons_border_rows(const double* geo, const int* inc_off, const int* inc, const int2* edges, const double* x0,
                      int nV, int bary, int total, const int* tg, const double* tgb, int ntg, const int* cut_edge,
                      int ncut, double* rows, int nrows, hipStream_t s);
// point and surface constraints by elimination: weights (w or 1) times the free mask, x_v <- W_v x_v
// (W_v = w_v (I - n_v n_v^T), nrm may be null), unit zero diagonals
void free_weights(const double* w, const double* free, int nV, double* out, hipStream_t s);
void mask_vertices(double* x, const double* w, const double* nrm, int nV, hipStream_t s);
void unit_zero_diag(double* A, int n, hipStream_t s);
// The border Schur complement's inverse on the device: S = D - K (nb x nb; K may be null), with a unit
// diagonal where S has a zero one when unit_zero is set, inverted by Gauss-Jordan elimination with
// partial pivoting into Sinv; a zero pivot sets `flag` in *flags (Sinv is then undefined).  nb <=
// kSchurDevMax.
constexpr int kSchurDevMax = 32;
void schur_inverse_device(const double* D, const double* K, int nb, bool unit_zero, double* Sinv, unsigned* flags,
                          unsigned flag, hipStream_t s);
// *flags |= flag when *v != 0 (a factorisation's info word).
void flag_if_nonzero(const int* v, unsigned* flags, unsigned flag, hipStream_t s);
// y = x / sqrt(*sq), n entries (sq on the device).
void vec_scale_rsqrt(const double* x, const double* sq, double* y, int n, hipStream_t s);
void cons_path_coeffs(const double* geo, const int2* edges, const int* path_edge, const int* path_prev, int np,
                      const double* w, const double* nrm, double* ta, double* td, double* tc, hipStream_t s);
void cons_scale_rows(const double* rows, const double* w, const double* nrm, int nV, int nrows, double* out,
                     hipStream_t s);
void cons_path_apply(const double* geo, const int2* edges, const int* path_edge, int np, const double* V, int nV,
                     int m, double* W, hipStream_t s);
void cons_apply_CT(const double* geo, const int* inc_off, const int* inc, const int* edge_path_row,
                   const double* yp, const double* rows, const double* yb, int nb, int nV, const double* in,
                   double* out, hipStream_t s);
void cons_border_solve(const double* Sinv, const double* wb, const double* dots, double* rhs, int nb, double* yb,
                       hipStream_t s);
void cons_sub_Zy(const double* Z, const double* yb, int nb, int np, double* yp, hipStream_t s);
// P x in three launches when nb <= kProjMaxBorder (in and out may alias:
// every output entry is written by the last launch from its own input
// entry); with packed rows and vertices (vertex degree <= 2), levels with
// np, nV <= 1024 take one launch.
constexpr int kProjMaxBorder = 8;
struct __align__(16) ProjRow {  // path row: T_I and the ends of edge I
  double t[3];
  int2 ends;
};
struct __align__(16) ProjVert {  // up to two incident path rows and s(v) T_I for each (-1: none)
  double c[2][3];
  int row[2];
};
struct ProjData {
  int np = 0, nb = 0, nV = 0;
  const double* geo = nullptr;
  const int2* edges = nullptr;
  const int* path_edge = nullptr;
  const double* rows = nullptr;  // border rows [nb][nV][3]
  const double* Z = nullptr;     // [nb][np]
  const double* Sinv = nullptr;  // [nb][nb]
  TriBlocks tri;                 // the path block's partition
  const double *lo = nullptr, *uinv = nullptr, *tc = nullptr;  // block-local factors and couplings
  const double *V = nullptr, *W = nullptr, *Rt = nullptr;     // spikes and reduced inverse (tri_prepare)
  const int *inc_off = nullptr, *inc = nullptr, *edge_path_row = nullptr;
  const ProjRow* prow = nullptr;    // packed rows [np] (null: from path_edge, edges, geo)
  const ProjVert* pvert = nullptr;  // packed vertices [nV] (null: from the incidence lists)
  double* part = nullptr;           // [max(B, 64) * 2 * kProjMaxBorder]
  double* g = nullptr;              // block-local solution [np]
  double* U = nullptr;              // boundary values [nr]
  double* yb = nullptr;             // [nb]
  // weighted form: with per-vertex weights w (C C^T above then being C W C^T),
  // out = beta prev + scale M in with M = W - W C^T (C W C^T)^-1 C W, the
  // inverse of W^-1 on the null space of C; w null: M = P
  const double* w = nullptr;
  // per-vertex unit normals [nV][3] (zero where a vertex has none): W_v = w_v (I - n_v n_v^T), the
  // tangent plane of a surface constraint eliminated like a weight
  const double* nrm = nullptr;
  double scale = 1.0, beta = 0.0;
  const double* prev = nullptr;  // null: no beta term (prev may alias out)
  double* xacc = nullptr;        // also xacc = out (xset) or xacc += out, per entry
  bool xset = false;
  // optional: also the operand of the next 16-bit product taken of out (of
  // xacc when prep_x), in the difference form of that product's preparation:
  // pp [nkt][3][32] = sqrt(d_v) (x_v - x_head), pcref [nkt][3] = x_head, the
  // head being the first vertex of v's 32-vertex column tile
  float* pp = nullptr;
  double* pcref = nullptr;
  const double* psqd = nullptr;
  bool prep_x = false;
};
void cons_project_fused(const ProjData& d, const double* in, double* out, hipStream_t s);
void cons_project_pack(const double* geo, const int2* edges, const int* path_edge, int np, const int* inc_off,
                       const int* inc, const int* edge_path_row, int nV, ProjRow* prow, ProjVert* pvert,
                       hipStream_t s);

// dense direct path
void dense_build_H(const double* A, const double* CtC, int nV, double* H, hipStream_t s);
void dense_C_edges(const double* geo, const int2* edges, int nE, int row0, int nV, const double* free, double* Cd,
                   hipStream_t s);
void dense_C_points(const int* pt, int npt, int row0, int nV, double* Cd, hipStream_t s);

}  // namespace rc
