// Launchers of the FP64 vector, dense and constraint kernels (k_linalg.hip).
#pragma once

#include "rc_internal.h"

namespace rc {

// out[r] = X_r . Y_r for r < m (X_r = X + r ldx, Y_r = Y + r ldy); scratch >= dot_scratch_size(m)
void vec_dots(const double* X, int ldx, const double* Y, int ldy, int n, int m, double* scratch, double* out,
              hipStream_t s);
int dot_scratch_size(int m);
// out = gamma - tau g / sqrt(gg[0])
void vec_trial(const double* gamma, const double* g, const double* gg, double tau, double* out, int n,
               hipStream_t s);

// Tridiagonal systems: factorisation (l, 1/u; info[0] = 0 on success) and
// solves by parallel scans in one workgroup.
void tridiag_factor(const double* a, const double* d, const double* c, int n, double* lo, double* uinv, int* info,
                    hipStream_t s);
void tridiag_solve(const double* lo, const double* uinv, const double* c, const double* b, double* y, int n,
                   hipStream_t s);
void dense_gemv(const double* A, const double* x, double* y, int n, hipStream_t s);

// constraint pieces
void cons_geometry(const double* gamma, const int2* edges, int nE, double* geo, hipStream_t s);
void cons_phi_edge(const double* geo, const double* x0, int nE, const double* len0, double* vals, double* phi_edges,
                   hipStream_t s);
void cons_border_rows(const double* geo, const int* inc_off, const int* inc, const int2* edges, const double* x0,
                      int nV, int bary, int total, const int* cut_edge, int ncut, double* rows, int nrows,
                      hipStream_t s);
void cons_path_coeffs(const double* geo, const int2* edges, const int* path_edge, const int* path_prev, int np,
                      double* ta, double* td, double* tc, hipStream_t s);
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
// entry).  part: device double [64 * 2 * kProjMaxBorder]; yb: [nb].  The
// factors lo_ch, uinv_ch, tc_ch (from tridiag_chunk_copy) and the work vectors
// wp_ch, yp_ch are in the solve's chunk-transposed order, tri_chunk_size(np)
// entries each.
constexpr int kProjMaxBorder = 8;
void cons_project_fused(const double* geo, const int2* edges, const int* path_edge, int np, const double* rows,
                        int nb, const double* Z, const double* Sinv, const double* lo_ch, const double* uinv_ch,
                        const double* tc_ch, const int* inc_off, const int* inc, const int* edge_path_row, int nV,
                        const double* in, double* out, double* part, double* wp_ch, double* yp_ch, double* yb,
                        hipStream_t s);
int tri_chunk_size(int n);
void tridiag_chunk_copy(const double* lo, const double* uinv, const double* c, int n, double* lo_ch,
                        double* uinv_ch, double* c_ch, hipStream_t s);

// dense direct path
void dense_build_H(const double* A, const double* CtC, int nV, double* H, hipStream_t s);
void dense_C_edges(const double* geo, const int2* edges, int nE, int row0, int nV, double* Cd, hipStream_t s);

}  // namespace rc
