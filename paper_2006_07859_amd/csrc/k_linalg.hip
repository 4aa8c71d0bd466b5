// FP64 vector, dense and constraint kernels used by the solvers.
//
// Reductions are two-pass (per-block partials, then one block) in a fixed
// order, so every result is bitwise reproducible.

#include "rc_internal.h"
#include "k_linalg.h"

#include <algorithm>

namespace rc {

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }
constexpr int kRedBlocks = 240;

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* __restrict__ y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

void vec_axpby(double a, const double* x, double b, double* y, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(cdiv(n, 256)), dim3(256), 0, s, a, x, b, y, n);
}

void vec_copy(const double* x, double* y, int n, hipStream_t s) {
  hipMemcpyAsync(y, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
}

__global__ void k_diag_inv(const double* __restrict__ r, const double* __restrict__ d, double* __restrict__ z,
                           int nV) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * nV) z[i] = r[i] / d[i / 3];
}

void vec_scale_diag_inv(const double* r, const double* d, double* z, int nV, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_inv, dim3(cdiv(3 * nV, 256)), dim3(256), 0, s, r, d, z, nV);
}

// Batched dots: out[r] = X_r . Y_r for r < m, X_r = X + r*ldx, Y_r = Y + r*ldy
// (ldy = 0 dots every X_r with the same Y).  grid = (kRedBlocks, m).
__global__ void k_dot_partial(const double* __restrict__ X, int ldx, const double* __restrict__ Y, int ldy, int n,
                              double* __restrict__ partial) {
  __shared__ double sm[256];
  const double* x = X + (size_t)blockIdx.y * ldx;
  const double* y = Y + (size_t)blockIdx.y * ldy;
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += x[i] * y[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sm[0];
}

__global__ void k_dot_final(const double* __restrict__ partial, int nb, double* __restrict__ out) {
  __shared__ double sm[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) v += partial[(size_t)blockIdx.x * nb + i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

void vec_dot(const double* x, const double* y, int n, double* scratch, double* result, hipStream_t s) {
  vec_dots(x, 0, y, 0, n, 1, scratch, result, s);
}

void vec_dots(const double* X, int ldx, const double* Y, int ldy, int n, int m, double* scratch, double* out,
              hipStream_t s) {
  int nb = std::min(kRedBlocks, std::max(1, cdiv(n, 256)));
  hipLaunchKernelGGL(k_dot_partial, dim3(nb, m), dim3(256), 0, s, X, ldx, Y, ldy, n, scratch);
  hipLaunchKernelGGL(k_dot_final, dim3(m), dim3(256), 0, s, scratch, nb, out);
}

int dot_scratch_size(int m) { return kRedBlocks * m; }

// Partial sums of the Gram entries X_j . Y_r, blockIdx.y = r mx + j (the blocks and tree of k_dot_partial).
__global__ void k_gram_partial(const double* __restrict__ X, int ldx, const double* __restrict__ Y, int ldy, int n,
                               int mx, double* __restrict__ partial) {
  __shared__ double sm[256];
  const int j = blockIdx.y % mx, r = blockIdx.y / mx;
  const double* x = X + (size_t)j * ldx;
  const double* y = Y + (size_t)r * ldy;
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += x[i] * y[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sm[0];
}

void vec_gram(const double* X, int ldx, const double* Y, int ldy, int n, int mx, int my, double* scratch,
              double* out, hipStream_t s) {
  const int nb = std::min(kRedBlocks, std::max(1, cdiv(n, 256)));
  hipLaunchKernelGGL(k_gram_partial, dim3(nb, mx * my), dim3(256), 0, s, X, ldx, Y, ldy, n, mx, scratch);
  hipLaunchKernelGGL(k_dot_final, dim3(mx * my), dim3(256), 0, s, scratch, nb, out);
}

// ---------------------------------------------------------------------------
// dense products (the coarsest level's saddle operator)
// ---------------------------------------------------------------------------
// C[m x n] = op(A) op(B) + beta C, row-major; op(A) is m x k (A stored k x m
// when transA), op(B) is k x n (B stored n x k when transB).
// C = op(A) op(B) (+ beta C), row major, op = transpose when the flag is set:
// 64 x 64 tiles of C per workgroup of 256 threads, each thread 4 x 4 entries
// (rows ty + 16 i, columns tx + 16 j), k staged through LDS 16 at a time;
// out-of-range rows, columns and k are zero-filled.
constexpr int kGemmT = 64, kGemmK = 16;

__global__ __launch_bounds__(256) void k_gemm(const double* __restrict__ A, const double* __restrict__ B,
                                              double* __restrict__ C, int m, int n, int k, double beta, int transA,
                                              int transB) {
  __shared__ double As[kGemmK][kGemmT + 1], Bs[kGemmK][kGemmT + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i0 = blockIdx.y * kGemmT, j0 = blockIdx.x * kGemmT;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int p0 = 0; p0 < k; p0 += kGemmK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // 64 x 16 of op(A) and 16 x 64 of op(B), four entries per thread
      const int e = threadIdx.x + 256 * q;
      {
        // op(A)(i, p): consecutive threads along p when A is row major, along i when transposed
        const int ii = transA ? e % kGemmT : e / kGemmK, pp = transA ? e / kGemmT : e % kGemmK;
        const int i = i0 + ii, p = p0 + pp;
        As[pp][ii] = (i < m && p < k) ? (transA ? A[(size_t)p * m + i] : A[(size_t)i * k + p]) : 0.0;
      }
      {
        // op(B)(p, j): consecutive threads along j when B is row major, along p when transposed
        const int jj = transB ? e / kGemmK : e % kGemmT, pp = transB ? e % kGemmK : e / kGemmT;
        const int j = j0 + jj, p = p0 + pp;
        Bs[pp][jj] = (j < n && p < k) ? (transB ? B[(size_t)j * k + p] : B[(size_t)p * n + j]) : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kGemmK; ++p) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[p][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[p][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = i0 + ty + 16 * i, c = j0 + tx + 16 * j;
      if (r < m && c < n) {
        const size_t idx = (size_t)r * n + c;
        C[idx] = acc[i][j] + (beta != 0.0 ? beta * C[idx] : 0.0);
      }
    }
}

void dense_gemm(const double* A, const double* B, double* C, int m, int n, int k, double beta, bool transA,
                hipStream_t s, bool transB) {
  dim3 g(cdiv(n, kGemmT), cdiv(m, kGemmT));
  hipLaunchKernelGGL(k_gemm, g, dim3(256), 0, s, A, B, C, m, n, k, beta, transA ? 1 : 0, transB ? 1 : 0);
}

// y = A x for a dense n x n row-major A and a vector x (one wave per row).
__global__ __launch_bounds__(256) void k_gemv(const double* __restrict__ A, const double* __restrict__ x,
                                              double* __restrict__ y, int n) {
  const int row = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += A[(size_t)row * n + j] * x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[row] = s;
}

void dense_gemv(const double* A, const double* x, double* y, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_gemv, dim3(cdiv(n, 4)), dim3(256), 0, s, A, x, y, n);
}

// ---------------------------------------------------------------------------
// tridiagonal systems: block-partitioned factorisation and solves
// ---------------------------------------------------------------------------
// Rows k < n: a[k] y[k-1] + d[k] y[k] + c[k] y[k+1] = b[k] with a[0] = c[n-1] = 0
// (zero couplings also separate independent segments).  The rows are cut into
// B blocks of S consecutive rows; with D the block-diagonal part and R the
// couplings across block boundaries (c at a block's last row, a at the next
// block's first row), K y = b becomes (I + D^-1 R) y = g with g = D^-1 b.
// D^-1 R is zero except for two columns per boundary, the spikes
//   V_q = D_q^-1 (c[e_q] e_last),   W_q = D_q^-1 (a[f_q] e_first)
// (e_q, f_q: last and first row of block q), so on block q
//   y = g - V_q y[f_{q+1}] - W_q y[e_{q-1}],
// and the 2 (B - 1) boundary values (y[e_q], y[f_{q+1}]) solve a reduced
// system that is block tridiagonal in 2 x 2 blocks.  Its inverse is formed
// once per factorisation (block elimination, one column per thread); a solve
// is then a local solve per block (B workgroups in parallel), one small dense
// product and the spike correction.
// Block-local factorisation (one wave per block): l[k] = a[k] / u[k-1],
// u[k] = d[k] - l[k] c[k-1], restarted (l = 0) at each block's first row, and
// stored as l and 1/u.  A local solve is two first-order linear recurrences,
// forward z[k] = b[k] - l[k] z[k-1] and backward y[k] = (z[k] - c[k] y[k+1]) / u[k],
// each an affine map per row: a workgroup composes the maps of each thread's
// rows, scans the composites (wave shuffles, then the wave totals) and
// replays its rows.
// The system is symmetric positive definite (a constraint Gram matrix), so
// the factorisation needs no pivoting.
__device__ __forceinline__ double readlane_f64(double v, int j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

TriBlocks tri_blocks(int n) {
  TriBlocks L;
  L.n = n;
  if (n <= kTriThreads) {  // one block (the one-workgroup projector relies on it)
    L.B = 1;
    L.S = std::max(n, 1);
    L.m = std::max(1, cdiv(L.S, kSpThreads));
  } else {
    L.m = std::min(kSpMaxM, cdiv(n, kSpThreads * 64));
    L.S = kSpThreads * L.m;
    L.B = cdiv(n, L.S);
  }
  L.nr = 2 * (L.B - 1);
  return L;
}

// One wave per block: the coefficients of 64 rows at a time are loaded
// coalesced and handed to the recurrence by lane reads; lane j keeps row j's
// factors.  The recurrence is carried in 1/u: l = a (1/u_prev),
// u = d - l c_prev, and 1/u by the hardware reciprocal and two Newton-Raphson
// steps y <- y + y (1 - u y), each of which squares the estimate's relative
// error (full FP64 precision for the u in [1, 2] of the edge-length Gram
// matrix: diagonal 2, couplings of size <= 1).
__global__ __launch_bounds__(64) void k_tridiag_factor(const double* __restrict__ a, const double* __restrict__ d,
                                                       const double* __restrict__ c, int n, int S,
                                                       double* __restrict__ lo, double* __restrict__ uinv,
                                                       int* __restrict__ info) {
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * S, r1 = min(n, r0 + S);
  double ui_prev = 0.0, c_prev = 0.0;  // the block's first row has l = 0
  int bad = 0;
  for (int k0 = r0; k0 < r1; k0 += 64) {
    const int k = k0 + lane;
    const double ak = k < r1 ? a[k] : 0.0, dk = k < r1 ? d[k] : 1.0, ck = k < r1 ? c[k] : 0.0;
    const int cnt = min(64, r1 - k0);
    double my_l = 0.0, my_ui = 0.0;
    for (int j = 0; j < cnt; ++j) {
      const double l = readlane_f64(ak, j) * ui_prev;
      const double u = fma(-l, c_prev, readlane_f64(dk, j));
      if (!(u > 0.0)) bad = k0 + j + 1;
      double y = __builtin_amdgcn_rcp(u);
      y = fma(y, fma(-u, y, 1.0), y);
      y = fma(y, fma(-u, y, 1.0), y);
      my_l = lane == j ? l : my_l;
      my_ui = lane == j ? y : my_ui;
      ui_prev = y;
      c_prev = readlane_f64(ck, j);
    }
    if (k < r1) {
      lo[k] = my_l;
      uinv[k] = my_ui;
    }
  }
  if (lane == 0 && bad) atomicMax(info, bad);
}

// Composite affine maps: (a, b) is v -> a v + b.  scan_compose returns, for
// every thread of an NW-wave workgroup, the composite of the maps of all
// threads before it in scan order (increasing thread index, or decreasing
// when rev), the first thread getting the identity (1, 0).  wa, wb: LDS [NW].
template <int NW>
__device__ __forceinline__ void scan_compose(double& a, double& b, bool rev, double* wa, double* wb) {
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  // inclusive scan inside the wave, in scan order (lane order reversed for rev)
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double pa = rev ? __shfl_down(a, off, 64) : __shfl_up(a, off, 64);
    const double pb = rev ? __shfl_down(b, off, 64) : __shfl_up(b, off, 64);
    const bool has = rev ? lane + off < 64 : lane >= off;
    if (has) {  // earlier composite (pa, pb) first, then this one
      b = a * pb + b;
      a = a * pa;
    }
  }
  // wave totals: the last lane in scan order holds its wave's composite
  const int last = rev ? 0 : 63;
  if (lane == last) {
    wa[w] = a;
    wb[w] = b;
  }
  // exclusive value inside the wave: the inclusive value of the previous lane in scan order
  double ea = rev ? __shfl_down(a, 1, 64) : __shfl_up(a, 1, 64);
  double eb = rev ? __shfl_down(b, 1, 64) : __shfl_up(b, 1, 64);
  const bool first = rev ? lane == 63 : lane == 0;
  if (first) {
    ea = 1.0;
    eb = 0.0;
  }
  __syncthreads();
  if (w == 0) {  // exclusive scan of the wave totals in scan order, in place: lane q holds the q-th total
    const int ww = rev ? NW - 1 - lane : lane;
    double ta = lane < NW ? wa[ww] : 1.0, tb = lane < NW ? wb[ww] : 0.0;
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const double pa = __shfl_up(ta, off, 64), pb = __shfl_up(tb, off, 64);
      if (lane >= off) {
        tb = ta * pb + tb;
        ta = ta * pa;
      }
    }
    double xa = __shfl_up(ta, 1, 64), xb = __shfl_up(tb, 1, 64);
    if (lane == 0) {
      xa = 1.0;
      xb = 0.0;
    }
    if (lane < NW) {
      wa[ww] = xa;
      wb[ww] = xb;
    }
  }
  __syncthreads();
  // prefix of this thread = (waves before) then (lanes before in this wave)
  const double pa = wa[w], pb = wb[w];
  a = ea * pa;
  b = ea * pb + eb;
}

// Local solve on block blk by a workgroup of kSpThreads threads (all must
// call it): thread t holds the right-hand sides of rows blk S + t m + j
// (j < m) in v and gets the block-local solution back.
__device__ __forceinline__ void tri_local_solve(const double* __restrict__ lo, const double* __restrict__ uinv,
                                                const double* __restrict__ c, const TriBlocks& L, int blk,
                                                double (&v)[kSpMaxM], double* wa, double* wb) {
  const int t = threadIdx.x;
  const int r1 = min(L.n, (blk + 1) * L.S);
  const int k0 = blk * L.S + t * L.m;
  const int cnt = max(0, min(L.m, r1 - k0));
  double rl[kSpMaxM], rq[kSpMaxM];
  double A = 1.0, B = 0.0;
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j)
    if (j < cnt) {
      rl[j] = lo[k0 + j];
      A = -rl[j] * A;
      B = -rl[j] * B + v[j];
    }
  scan_compose<kSpWaves>(A, B, false, wa, wb);
  double zin = B;  // z before the thread's rows (z = 0 before the block)
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j)
    if (j < cnt) {
      zin = -rl[j] * zin + v[j];
      v[j] = zin;
    }
  __syncthreads();  // the LDS slots are reused by the second scan
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j)
    if (j < cnt) {
      const double ui = uinv[k0 + j];
      rq[j] = -c[k0 + j] * ui;  // coupling
      v[j] *= ui;               // offset
    }
  A = 1.0;
  B = 0.0;
#pragma unroll
  for (int j = kSpMaxM - 1; j >= 0; --j)
    if (j < cnt) {
      A = rq[j] * A;
      B = rq[j] * B + v[j];
    }
  scan_compose<kSpWaves>(A, B, true, wa, wb);
  double yin = B;  // y after the thread's rows (y = 0 after the block)
#pragma unroll
  for (int j = kSpMaxM - 1; j >= 0; --j)
    if (j < cnt) {
      yin = rq[j] * yin + v[j];
      v[j] = yin;
    }
}

// g_r = D^-1 b_r for m right-hand sides (grid: blocks x m; columns ld apart)
__global__ __launch_bounds__(kSpThreads) void k_tri_local(const double* __restrict__ lo,
                                                          const double* __restrict__ uinv,
                                                          const double* __restrict__ c, const TriBlocks L,
                                                          const double* __restrict__ rhs, int ldr,
                                                          double* __restrict__ g, int ldg) {
  __shared__ double wa[kSpWaves], wb[kSpWaves];
  const int blk = blockIdx.x, col = blockIdx.y;
  const int k0 = blk * L.S + threadIdx.x * L.m;
  const int cnt = max(0, min(L.m, min(L.n, (blk + 1) * L.S) - k0));
  const double* b = rhs + (size_t)col * ldr;
  double v[kSpMaxM];
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j) v[j] = j < cnt ? b[k0 + j] : 0.0;
  tri_local_solve(lo, uinv, c, L, blk, v, wa, wb);
  double* out = g + (size_t)col * ldg;
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j)
    if (j < cnt) out[k0 + j] = v[j];
}

// Right-hand sides of the spikes: column 0 c[e_q] at each block's last row
// (blocks before the last), column 1 a[f_q] at each block's first row (blocks
// after the first).
__global__ void k_spike_unit(const double* __restrict__ a, const double* __restrict__ c, const TriBlocks L,
                             double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L.n) return;
  const int q = k / L.S, pos = k - q * L.S;
  out[k] = (q < L.B - 1 && pos == L.S - 1) ? c[k] : 0.0;
  out[L.n + k] = (q > 0 && pos == 0) ? a[k] : 0.0;
}

// The reduced system on the boundary values U_q = (y[e_q], y[f_{q+1}]),
// q < B - 1 (rows of the spike equations at e_q and f_{q+1}):
//   y[e_q] + V[e_q] y[f_{q+1}] + W[e_q] y[e_{q-1}] = g[e_q]
//   y[f_{q+1}] + W[f_{q+1}] y[e_q] + V[f_{q+1}] y[f_{q+2}] = g[f_{q+1}].
// Block elimination: D'_q = D_q - L_q D'_{q-1}^-1 R_{q-1} changes only the
// (0, 1) entry of D_q = [[1, V[e_q]], [W[f_{q+1}], 1]] (L_q has W[e_q] at (0, 0),
// R_{q-1} has V[f_q] at (1, 1)).  Thread 0 forms the 2 x 2 inverses; thread
// j < nr then solves for column j of the inverse, using row j of Rt as its
// scratch, and leaves Rt[j nr + i] = (M^-1)_ij.
__global__ __launch_bounds__(kSpThreads) void k_spike_rinv(const double* __restrict__ V,
                                                           const double* __restrict__ W, const TriBlocks L,
                                                           double* __restrict__ Rt) {
  __shared__ double dinv[kSpMaxB][4];
  const int nq = L.B - 1, nr = L.nr, S = L.S;
  if (threadIdx.x == 0) {
    double prev01 = 0.0;  // (D'_{q-1}^-1)_01
    for (int q = 0; q < nq; ++q) {
      const int e = (q + 1) * S - 1, f = (q + 1) * S;
      const double m00 = 1.0, m11 = 1.0, m10 = W[f];
      const double m01 = V[e] - (q > 0 ? W[e] * V[(q) * S] * prev01 : 0.0);
      const double det = m00 * m11 - m01 * m10;
      dinv[q][0] = m11 / det;
      dinv[q][1] = -m01 / det;
      dinv[q][2] = -m10 / det;
      dinv[q][3] = m00 / det;
      prev01 = dinv[q][1];
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nr; j += blockDim.x) {
    double* x = Rt + (size_t)j * nr;
    // forward: G'_q = G_q - L_q D'_{q-1}^-1 G'_{q-1} (only the first entry changes)
    double p0 = 0.0, p1 = 0.0;  // G'_{q-1}
    for (int q = 0; q < nq; ++q) {
      double g0 = (2 * q == j) ? 1.0 : 0.0, g1 = (2 * q + 1 == j) ? 1.0 : 0.0;
      if (q > 0) g0 -= W[(q + 1) * S - 1] * (dinv[q - 1][0] * p0 + dinv[q - 1][1] * p1);
      x[2 * q] = g0;
      x[2 * q + 1] = g1;
      p0 = g0;
      p1 = g1;
    }
    // backward: U_q = D'_q^-1 (G'_q - R_q U_{q+1})
    double u1n = 0.0;  // U_{q+1}[1]
    for (int q = nq - 1; q >= 0; --q) {
      const double g0 = x[2 * q];
      const double g1 = x[2 * q + 1] - (q < nq - 1 ? V[(q + 1) * S] * u1n : 0.0);
      const double u0 = dinv[q][0] * g0 + dinv[q][1] * g1, u1 = dinv[q][2] * g0 + dinv[q][3] * g1;
      x[2 * q] = u0;
      x[2 * q + 1] = u1;
      u1n = u1;
    }
  }
}

// U_r = M^-1 (g_r[e_q], g_r[f_{q+1}])_q for m columns (grid: m)
__global__ __launch_bounds__(kSpThreads) void k_tri_reduce(const double* __restrict__ g, int ldg, const TriBlocks L,
                                                           const double* __restrict__ Rt, double* __restrict__ U) {
  __shared__ double rhs[2 * (kSpMaxB - 1)];
  const int col = blockIdx.y * gridDim.x + blockIdx.x, nr = L.nr;
  const double* gc = g + (size_t)col * ldg;
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    const int q = i / 2;
    rhs[i] = gc[(i % 2 == 0) ? (q + 1) * L.S - 1 : (q + 1) * L.S];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
    double u = 0.0;
    for (int j = 0; j < nr; ++j) u += Rt[(size_t)j * nr + i] * rhs[j];
    U[(size_t)col * nr + i] = u;
  }
}

// y = g - V U[2q + 1] - W U[2 (q - 1)] on block q (grid: row blocks x m)
__global__ void k_tri_correct(const double* __restrict__ g, int ldg, const double* __restrict__ V,
                              const double* __restrict__ W, const double* __restrict__ U, const TriBlocks L,
                              double* __restrict__ y, int ldy) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, col = blockIdx.y;
  if (k >= L.n) return;
  const int q = k / L.S;
  const double* Uc = U + (size_t)col * L.nr;
  double v = g[(size_t)col * ldg + k];
  if (q < L.B - 1) v -= V[k] * Uc[2 * q + 1];
  if (q > 0) v -= W[k] * Uc[2 * (q - 1)];
  y[(size_t)col * ldy + k] = v;
}

void tri_prepare(const double* a, const double* d, const double* c, const TriBlocks& L, double* lo, double* uinv,
                 double* VW, double* Rt, double* scratch, int* info, hipStream_t s) {
  hipMemsetAsync(info, 0, sizeof(int), s);
  if (L.n <= 0) return;
  hipLaunchKernelGGL(k_tridiag_factor, dim3(L.B), dim3(64), 0, s, a, d, c, L.n, L.S, lo, uinv, info);
  if (L.B == 1) {  // no boundaries: zero spikes
    hipMemsetAsync(VW, 0, sizeof(double) * 2 * (size_t)L.n, s);
    return;
  }
  hipLaunchKernelGGL(k_spike_unit, dim3(cdiv(L.n, 256)), dim3(256), 0, s, a, c, L, scratch);
  hipLaunchKernelGGL(k_tri_local, dim3(L.B, 2), dim3(kSpThreads), 0, s, lo, uinv, c, L, (const double*)scratch,
                     L.n, VW, L.n);
  hipLaunchKernelGGL(k_spike_rinv, dim3(1), dim3(kSpThreads), 0, s, (const double*)VW, (const double*)(VW + L.n), L,
                     Rt);
}

void tri_solve(const TriSys& T, const double* rhs, int ldr, double* y, int ldy, int m, double* g, double* U,
               hipStream_t s) {
  const TriBlocks& L = T.L;
  if (L.n <= 0 || m <= 0) return;
  if (L.B == 1) {
    hipLaunchKernelGGL(k_tri_local, dim3(1, m), dim3(kSpThreads), 0, s, T.lo, T.uinv, T.c, L, rhs, ldr, y, ldy);
    return;
  }
  hipLaunchKernelGGL(k_tri_local, dim3(L.B, m), dim3(kSpThreads), 0, s, T.lo, T.uinv, T.c, L, rhs, ldr, g, L.n);
  hipLaunchKernelGGL(k_tri_reduce, dim3(m), dim3(kSpThreads), 0, s, (const double*)g, L.n, L, T.Rt, U);
  hipLaunchKernelGGL(k_tri_correct, dim3(cdiv(L.n, 256), m), dim3(256), 0, s, (const double*)g, L.n, T.V, T.W,
                     (const double*)U, L, y, ldy);
}

// ---------------------------------------------------------------------------
// constraints (FP64): Jacobian products for the edge rows and the dense
// border rows (barycenter, total length, one cut edge per loop)
// ---------------------------------------------------------------------------
// Edge-length row I (Phi_I = l0_I - l_I): +T_I at i1, -T_I at i2.
// Path rows are the edge rows except the cut edges, in chain order: path_edge[k].

// Geometry in FP64 for the constraint kernels: l, T, x per edge.
__global__ void k_cons_geom(const double* __restrict__ gamma, const int2* __restrict__ edges, int nE,
                            double* __restrict__ geo /* [nE][8]: l, T(3), x(3), - */) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  int2 e = edges[I];
  double p[3], q[3];
  for (int k = 0; k < 3; ++k) {
    p[k] = gamma[3 * e.x + k];
    q[k] = gamma[3 * e.y + k];
  }
  double d0 = q[0] - p[0], d1 = q[1] - p[1], d2 = q[2] - p[2];
  double l = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double* o = geo + 8 * (size_t)I;
  o[0] = l;
  o[1] = d0 / l;
  o[2] = d1 / l;
  o[3] = d2 / l;
  o[4] = 0.5 * (p[0] + q[0]);
  o[5] = 0.5 * (p[1] + q[1]);
  o[6] = 0.5 * (p[2] + q[2]);
  o[7] = 0.0;
}

void cons_geometry(const double* gamma, const int2* edges, int nE, double* geo, hipStream_t s) {
  hipLaunchKernelGGL(k_cons_geom, dim3(cdiv(nE, 256)), dim3(256), 0, s, gamma, edges, nE, geo);
}

// Per-edge values summed by the border-row evaluations, stored as four
// columns vals[c * nE + I]: l_I (x_I - x0)_c for c < 3 and l_I for c = 3.
__global__ void k_cons_phi_edge(const double* __restrict__ geo, const double* __restrict__ x0, int nE,
                                const double* __restrict__ len0, double* __restrict__ vals,
                                double* __restrict__ phi_edges) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const double* g = geo + 8 * (size_t)I;
  vals[I] = g[0] * (g[4] - x0[0]);
  vals[nE + I] = g[0] * (g[5] - x0[1]);
  vals[2 * (size_t)nE + I] = g[0] * (g[6] - x0[2]);
  vals[3 * (size_t)nE + I] = g[0];
  if (phi_edges) phi_edges[I] = len0[I] - g[0];
}

void cons_phi_edge(const double* geo, const double* x0, int nE, const double* len0, double* vals,
                   double* phi_edges, hipStream_t s) {
  hipLaunchKernelGGL(k_cons_phi_edge, dim3(cdiv(nE, 256)), dim3(256), 0, s, geo, x0, nE, len0, vals, phi_edges);
}

// Border rows as dense vertex vectors rows[r][nV][3], in the order barycenter (3),
// total length (1), tangents (2 each), cut edges (1 each).
//   barycenter row c: at v, sum_{I at v} (l_I/2) e_c + sigma_I(v) (x_I - x0)_c T_I, sigma(i1) = -1, sigma(i2) = +1
//   total-length row: at v, sum_{I at v} s_I(v) T_I with s(i1) = +1, s(i2) = -1
//   cut-edge row for edge I: +T_I at i1, -T_I at i2
__global__ void k_border_rows(const double* __restrict__ geo, const int* __restrict__ inc_off,
                              const int* __restrict__ inc, const double* __restrict__ x0, int nV, int bary,
                              int total, double* __restrict__ rows) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double L[3] = {0, 0, 0};
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int I = inc[k] >> 1;
    const double sg = (inc[k] & 1) ? 1.0 : -1.0;  // sigma
    const double* g = geo + 8 * (size_t)I;
    for (int r = 0; r < 3; ++r) {
      M[r][r] += 0.5 * g[0];
      for (int cc = 0; cc < 3; ++cc) M[r][cc] += sg * (g[4 + r] - x0[r]) * g[1 + cc];
      L[r] += -sg * g[1 + r];
    }
  }
  int row = 0;
  if (bary) {
    for (int r = 0; r < 3; ++r) {
      for (int cc = 0; cc < 3; ++cc) rows[((size_t)row * nV + v) * 3 + cc] = M[r][cc];
      ++row;
    }
  }
  if (total) {
    for (int cc = 0; cc < 3; ++cc) rows[((size_t)row * nV + v) * 3 + cc] = L[cc];
    ++row;
  }
}

__global__ void k_cut_rows(const double* __restrict__ geo, const int2* __restrict__ edges,
                           const int* __restrict__ cut_edge, int ncut, int row0, int nV, double* __restrict__ rows) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncut) return;
  const int I = cut_edge[q];
  const double* g = geo + 8 * (size_t)I;
  double* r = rows + (size_t)(row0 + q) * nV * 3;
  int2 e = edges[I];
  for (int cc = 0; cc < 3; ++cc) {
    r[3 * e.x + cc] = g[1 + cc];
    r[3 * e.y + cc] = -g[1 + cc];
  }
}

// tangent rows (Sec. 7.1, read as (u . T_I, v . T_I)): d(b . T_I) = (b - (b . T_I) T_I) / l_I at i2,
// its negative at i1; rows row0 + 2 j (b = u) and row0 + 2 j + 1 (b = v) of tangent j
__global__ void k_tangent_rows(const double* __restrict__ geo, const int2* __restrict__ edges,
                               const int* __restrict__ tg, const double* __restrict__ tgb, int ntg, int row0, int nV,
                               double* __restrict__ rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ntg) return;
  const int I = tg[i / 2];
  const double* g = geo + 8 * (size_t)I;
  const double* b = tgb + 6 * (i / 2) + 3 * (i % 2);
  const double bt = b[0] * g[1] + b[1] * g[2] + b[2] * g[3];
  const int2 e = edges[I];
  double* r = rows + (size_t)(row0 + i) * nV * 3;
  for (int cc = 0; cc < 3; ++cc) {
    const double v = (b[cc] - bt * g[1 + cc]) / g[0];
    r[3 * e.y + cc] = v;
    r[3 * e.x + cc] = -v;
  }
}

void cons_border_rows(const double* geo, const int* inc_off, const int* inc, const int2* edges, const double* x0,
                      int nV, int bary, int total, const int* tg, const double* tgb, int ntg, const int* cut_edge,
                      int ncut, double* rows, int nrows, hipStream_t s) {
  hipMemsetAsync(rows, 0, sizeof(double) * (size_t)nrows * nV * 3, s);
  hipLaunchKernelGGL(k_border_rows, dim3(cdiv(nV, 256)), dim3(256), 0, s, geo, inc_off, inc, x0, nV, bary, total,
                     rows);
  const int row_tg = 3 * bary + total;
  if (ntg > 0)
    hipLaunchKernelGGL(k_tangent_rows, dim3(cdiv(2 * ntg, 64)), dim3(64), 0, s, geo, edges, tg, tgb, ntg, row_tg, nV,
                       rows);
  if (ncut > 0)
    hipLaunchKernelGGL(k_cut_rows, dim3(cdiv(ncut, 256)), dim3(256), 0, s, geo, edges, cut_edge, ncut,
                       row_tg + 2 * ntg, nV, rows);
}

// Tridiagonal coefficients of C_p W C_p^T over the path rows (chain order),
// W = diag(w) per vertex (w null: the identity): diag w_i1 + w_i2 (|T_I| = 1),
// off-diagonal s_I(v) s_J(v) w_v T_I.T_J for consecutive rows sharing v.
// T_I^T W_v T_J with W_v = w_v (I - n_v n_v^T) (unit tangents)
__device__ __forceinline__ double tw_dot(const double* __restrict__ w, const double* __restrict__ nrm, int v,
                                         const double* ti, const double* tj) {
  double d = ti[0] * tj[0] + ti[1] * tj[1] + ti[2] * tj[2];
  if (nrm) {
    const double* n = nrm + 3 * (size_t)v;
    d -= (n[0] * ti[0] + n[1] * ti[1] + n[2] * ti[2]) * (n[0] * tj[0] + n[1] * tj[1] + n[2] * tj[2]);
  }
  return w ? w[v] * d : d;
}

__global__ void k_path_coeffs(const double* __restrict__ geo, const int2* __restrict__ edges,
                              const int* __restrict__ path_edge, const int* __restrict__ path_prev, int np,
                              const double* __restrict__ w, const double* __restrict__ nrm, double* __restrict__ ta,
                              double* __restrict__ td, double* __restrict__ tc) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const int I = path_edge[k];
  const int2 ei = edges[I];
  if (nrm) {
    const double* ti = geo + 8 * (size_t)I + 1;
    td[k] = tw_dot(w, nrm, ei.x, ti, ti) + tw_dot(w, nrm, ei.y, ti, ti);
  } else {
    td[k] = w ? w[ei.x] + w[ei.y] : 2.0;
  }
  // both ends of zero weight (pinned vertices): the row of C W C^T is zero and its constraint
  // holds for every admissible vector; a unit diagonal gives it a zero multiplier (pseudo-inverse)
  if (td[k] == 0.0) td[k] = 1.0;
  if (path_prev[k]) {
    const int J = path_edge[k - 1];
    const int2 ej = edges[J];
    // shared vertex and the signs (+1 at i1, -1 at i2)
    double si, sj;
    int sv;
    if (ei.x == ej.x) { si = 1; sj = 1; sv = ei.x; }
    else if (ei.x == ej.y) { si = 1; sj = -1; sv = ei.x; }
    else if (ei.y == ej.x) { si = -1; sj = 1; sv = ei.y; }
    else { si = -1; sj = -1; sv = ei.y; }
    const double* gi = geo + 8 * (size_t)I;
    const double* gj = geo + 8 * (size_t)J;
    const double v = nrm ? si * sj * tw_dot(w, nrm, sv, gi + 1, gj + 1)
                         : si * sj * (gi[1] * gj[1] + gi[2] * gj[2] + gi[3] * gj[3]) * (w ? w[sv] : 1.0);
    ta[k] = v;
    tc[k - 1] = v;
  } else {
    ta[k] = 0.0;
  }
  if (k == np - 1) tc[k] = 0.0;
}

void cons_path_coeffs(const double* geo, const int2* edges, const int* path_edge, const int* path_prev, int np,
                      const double* w, const double* nrm, double* ta, double* td, double* tc, hipStream_t s) {
  // tc[k-1] is written by row k; rows without a predecessor leave tc[k-1] to be zero
  hipMemsetAsync(tc, 0, sizeof(double) * np, s);
  hipLaunchKernelGGL(k_path_coeffs, dim3(cdiv(np, 256)), dim3(256), 0, s, geo, edges, path_edge, path_prev, np, w,
                     nrm, ta, td, tc);
}

// out[r][v] = W_v rows[r][v] for nrows rows, W_v = w[v] (I - n_v n_v^T) (nrm may be null)
__global__ void k_scale_rows(const double* __restrict__ rows, const double* __restrict__ w,
                             const double* __restrict__ nrm, int nV, int nrows, double* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nrows * nV) return;
  const int v = (int)(i % nV);
  const double* r = rows + 3 * i;
  double x0 = r[0], x1 = r[1], x2 = r[2];
  if (nrm) {
    const double* n = nrm + 3 * (size_t)v;
    const double p = n[0] * x0 + n[1] * x1 + n[2] * x2;
    x0 -= p * n[0];
    x1 -= p * n[1];
    x2 -= p * n[2];
  }
  const double wv = w[v];
  out[3 * i] = x0 * wv;
  out[3 * i + 1] = x1 * wv;
  out[3 * i + 2] = x2 * wv;
}

void cons_scale_rows(const double* rows, const double* w, const double* nrm, int nV, int nrows, double* out,
                     hipStream_t s) {
  const size_t n = (size_t)nrows * nV;
  if (n == 0) return;
  hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows, w, nrm, nV, nrows,
                     out);
}

// w[k] = C_{path_edge[k]} v = T_I . (v_i1 - v_i2), for m vectors (v_r = V + r*3nV, w_r = W + r*np).
__global__ void k_path_apply(const double* __restrict__ geo, const int2* __restrict__ edges,
                             const int* __restrict__ path_edge, int np, const double* __restrict__ V, int nV,
                             double* __restrict__ W) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  const double* v = V + (size_t)blockIdx.y * 3 * nV;
  const int I = path_edge[k];
  const int2 e = edges[I];
  const double* g = geo + 8 * (size_t)I;
  W[(size_t)blockIdx.y * np + k] =
      g[1] * (v[3 * e.x] - v[3 * e.y]) + g[2] * (v[3 * e.x + 1] - v[3 * e.y + 1]) + g[3] * (v[3 * e.x + 2] - v[3 * e.y + 2]);
}

void cons_path_apply(const double* geo, const int2* edges, const int* path_edge, int np, const double* V, int nV,
                     int m, double* W, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_path_apply, dim3(cdiv(np, 256), m), dim3(256), 0, s, geo, edges, path_edge, np, V, nV, W);
}

// out_v = alpha * in_v - [ sum_{path rows k at v} s(v) T_I y_k + sum_r yb[r] rows[r][v] ]
// (in may be null: out = -C^T y).
__global__ void k_apply_CT(const double* __restrict__ geo, const int* __restrict__ inc_off,
                           const int* __restrict__ inc, const int* __restrict__ edge_path_row,
                           const double* __restrict__ yp, const double* __restrict__ rows,
                           const double* __restrict__ yb, int nb, int nV, const double* __restrict__ in,
                           double* __restrict__ out) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double acc[3] = {0, 0, 0};
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int I = inc[k] >> 1;
    const int pr = edge_path_row[I];
    if (pr < 0) continue;
    const double sg = (inc[k] & 1) ? -1.0 : 1.0;
    const double* g = geo + 8 * (size_t)I;
    for (int cc = 0; cc < 3; ++cc) acc[cc] += sg * g[1 + cc] * yp[pr];
  }
  for (int r = 0; r < nb; ++r)
    for (int cc = 0; cc < 3; ++cc) acc[cc] += yb[r] * rows[((size_t)r * nV + v) * 3 + cc];
  for (int cc = 0; cc < 3; ++cc) out[3 * v + cc] = (in ? in[3 * v + cc] : 0.0) - acc[cc];
}

void cons_apply_CT(const double* geo, const int* inc_off, const int* inc, const int* edge_path_row,
                   const double* yp, const double* rows, const double* yb, int nb, int nV, const double* in,
                   double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_CT, dim3(cdiv(nV, 256)), dim3(256), 0, s, geo, inc_off, inc, edge_path_row, yp, rows,
                     yb, nb, nV, in, out);
}

// y_p -= Z y_b (Z is np x nb column blocks: Z + r*np), and the small dense
// border solve y_b = Sinv rhs_b, done by one thread (nb is small).
__global__ void k_sub_Zy(const double* __restrict__ Z, const double* __restrict__ yb, int nb, int np,
                         double* __restrict__ yp) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  double s = 0.0;
  for (int r = 0; r < nb; ++r) s += Z[(size_t)r * np + k] * yb[r];
  yp[k] -= s;
}

// yb = Sinv (wb - dots): one workgroup, nb <= 128
__global__ void k_border_fused(const double* __restrict__ Sinv, const double* __restrict__ wb,
                               const double* __restrict__ dots, int nb, double* __restrict__ yb) {
  __shared__ double rhs[128];
  for (int r = threadIdx.x; r < nb; r += blockDim.x) rhs[r] = wb[r] - (dots ? dots[r] : 0.0);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < nb; ++j) s += Sinv[i * nb + j] * rhs[j];
    yb[i] = s;
  }
}

void cons_border_solve(const double* Sinv, const double* wb, const double* dots, double* rhs, int nb, double* yb,
                       hipStream_t s) {
  (void)rhs;
  hipLaunchKernelGGL(k_border_fused, dim3(1), dim3(128), 0, s, Sinv, wb, dots, nb, yb);
}

void cons_sub_Zy(const double* Z, const double* yb, int nb, int np, double* yp, hipStream_t s) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_sub_Zy, dim3(cdiv(np, 256)), dim3(256), 0, s, Z, yb, nb, np, yp);
}

// ---------------------------------------------------------------------------
// small device-side pieces of the constraint set-up (no host round trip)
// ---------------------------------------------------------------------------
// One workgroup; the matrix and its inverse in LDS.  The steps are those of
// the host routine they replace: per column the first row of largest
// magnitude as pivot, row swap, pivot row scaled by 1 / pivot, every other
// row eliminated (multipliers read before the column is overwritten).
__global__ __launch_bounds__(256) void k_schur_inverse(const double* __restrict__ D, const double* __restrict__ K,
                                                       int n, int unit_zero, double* __restrict__ Sinv,
                                                       unsigned* __restrict__ flags, unsigned flag) {
  __shared__ double A[kSchurDevMax * kSchurDevMax], I[kSchurDevMax * kSchurDevMax], f[kSchurDevMax];
  __shared__ int piv_s, bad_s;
  const int t = threadIdx.x, nn = n * n;
  for (int i = t; i < nn; i += 256) {
    A[i] = D[i] - (K ? K[i] : 0.0);
    I[i] = (i / n == i % n) ? 1.0 : 0.0;
  }
  if (t == 0) bad_s = 0;
  __syncthreads();
  if (unit_zero && t < n && A[t * n + t] == 0.0) A[t * n + t] = 1.0;
  __syncthreads();
  for (int col = 0; col < n; ++col) {
    if (t == 0) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
      piv_s = piv;
      if (!(fabs(A[piv * n + col]) > 0.0)) bad_s = 1;
    }
    __syncthreads();
    if (bad_s) break;  // uniform over the workgroup
    const int piv = piv_s;
    if (piv != col)
      for (int j = t; j < n; j += 256) {
        const double a = A[col * n + j], i = I[col * n + j];
        A[col * n + j] = A[piv * n + j];
        I[col * n + j] = I[piv * n + j];
        A[piv * n + j] = a;
        I[piv * n + j] = i;
      }
    __syncthreads();
    const double d = 1.0 / A[col * n + col];
    __syncthreads();  // every thread has read the pivot before its row is scaled
    for (int j = t; j < n; j += 256) {
      A[col * n + j] *= d;
      I[col * n + j] *= d;
    }
    for (int r = t; r < n; r += 256) f[r] = r == col ? 0.0 : A[r * n + col];
    __syncthreads();
    for (int i = t; i < nn; i += 256) {
      const double fr = f[i / n];
      if (fr == 0.0) continue;
      const int j = i % n;
      A[i] -= fr * A[col * n + j];
      I[i] -= fr * I[col * n + j];
    }
    __syncthreads();
  }
  if (bad_s) {
    if (t == 0) atomicOr(flags, flag);
    return;
  }
  for (int i = t; i < nn; i += 256) Sinv[i] = I[i];
}

void schur_inverse_device(const double* D, const double* K, int nb, bool unit_zero, double* Sinv, unsigned* flags,
                          unsigned flag, hipStream_t s) {
  hipLaunchKernelGGL(k_schur_inverse, dim3(1), dim3(256), 0, s, D, K, nb, unit_zero ? 1 : 0, Sinv, flags, flag);
}

__global__ void k_flag_if_nonzero(const int* __restrict__ v, unsigned* __restrict__ flags, unsigned flag) {
  if (threadIdx.x == 0 && *v != 0) atomicOr(flags, flag);
}

void flag_if_nonzero(const int* v, unsigned* flags, unsigned flag, hipStream_t s) {
  hipLaunchKernelGGL(k_flag_if_nonzero, dim3(1), dim3(64), 0, s, v, flags, flag);
}

__global__ void k_scale_rsqrt(const double* __restrict__ x, const double* __restrict__ sq, double* __restrict__ y,
                              int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (1.0 / sqrt(sq[0])) * x[i];
}

void vec_scale_rsqrt(const double* x, const double* sq, double* y, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rsqrt, dim3(cdiv(n, 256)), dim3(256), 0, s, x, sq, y, n);
}

// ---------------------------------------------------------------------------
// the projector P x = x - C^T (C C^T)^-1 C x in three launches (nb <= 8)
// ---------------------------------------------------------------------------
// With K = C C^T split into the path block Kpp (tridiagonal), the border
// block Kbb and their coupling Kpb, and Z = Kpp^-1 Kpb (columns), the Schur
// complement solve of K y = (wp, wb) is
//   yb = S^-1 (wb - Z^T wp),  yp = Kpp^-1 wp - Z yb,   S = Kbb - Kpb^T Z,
// using Kpb^T Kpp^-1 = Z^T (Kpp is symmetric).  Kpp^-1 is the
// block-partitioned solve above:
//   1. k_proj_rows (one workgroup per block of path rows): wp = C_path x, the
//      block-local solution g = D^-1 wp, and per-workgroup partial sums of
//      the border rows' dot products wb = rows . x and of Z^T wp;
//   2. k_proj_solve (one workgroup): the partial sums, yb, and the reduced
//      boundary values U = M^-1 (g at the block boundaries);
//   3. k_apply_CT_z: out = x - C^T y with yp = g - V U - W U - Z yb per row;
// steps 2 and 3 share one launch (k_solve_apply_CT_z, each workgroup
// repeating step 2) when the reduced system has at most 128 rows.
// With vertex degree <= 2 (curves), the row data (T_I and the edge's ends)
// and each vertex's incident path rows with their signed tangents s(v) T_I
// are packed per level (ProjRow, ProjVert), so that a row or vertex needs one
// load before the gathers.
constexpr int kProjSlots = 2 * kProjMaxBorder;

// x <- W_v x with W_v = w_v (I - n_v n_v^T) (d.w null: w_v = 1; d.nrm null: no normal part)
__device__ __forceinline__ void proj_w_apply(const ProjData& d, int v, double& x0, double& x1, double& x2) {
  if (d.nrm) {
    const double* n = d.nrm + 3 * (size_t)v;
    const double p = n[0] * x0 + n[1] * x1 + n[2] * x2;
    x0 -= p * n[0];
    x1 -= p * n[1];
    x2 -= p * n[2];
  }
  if (d.w) {
    const double s = d.w[v];
    x0 *= s;
    x1 *= s;
    x2 *= s;
  }
}

// w = C_I x for path row i
__device__ __forceinline__ double proj_row_value(const ProjData& d, int i, const double* __restrict__ x) {
  double t0, t1, t2;
  int a, b;
  if (d.prow) {
    const ProjRow p = d.prow[i];
    t0 = p.t[0];
    t1 = p.t[1];
    t2 = p.t[2];
    a = p.ends.x;
    b = p.ends.y;
  } else {
    const int I = d.path_edge[i];
    const int2 e = d.edges[I];
    const double* g = d.geo + 8 * (size_t)I;
    t0 = g[1];
    t1 = g[2];
    t2 = g[3];
    a = e.x;
    b = e.y;
  }
  if (d.nrm) {  // C (W x) with the normal parts
    double a0 = x[3 * a], a1 = x[3 * a + 1], a2 = x[3 * a + 2];
    double b0 = x[3 * b], b1 = x[3 * b + 1], b2 = x[3 * b + 2];
    proj_w_apply(d, a, a0, a1, a2);
    proj_w_apply(d, b, b0, b1, b2);
    return t0 * (a0 - b0) + t1 * (a1 - b1) + t2 * (a2 - b2);
  }
  if (d.w) {  // C (W x)
    const double wa = d.w[a], wb = d.w[b];
    return t0 * (wa * x[3 * a] - wb * x[3 * b]) + t1 * (wa * x[3 * a + 1] - wb * x[3 * b + 1]) +
           t2 * (wa * x[3 * a + 2] - wb * x[3 * b + 2]);
  }
  return t0 * (x[3 * a] - x[3 * b]) + t1 * (x[3 * a + 1] - x[3 * b + 1]) + t2 * (x[3 * a + 2] - x[3 * b + 2]);
}

__global__ __launch_bounds__(kSpThreads) void k_proj_rows(const ProjData d, const double* __restrict__ x) {
  __shared__ double wa[kSpWaves], wb[kSpWaves];
  __shared__ double sred[kSpWaves][kProjSlots];
  const int t = threadIdx.x, blk = blockIdx.x;
  const int np = d.np, nV = d.nV, nb = d.nb;
  const TriBlocks& L = d.tri;
  double acc[kProjSlots];
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) acc[q] = 0.0;
  // the thread's path rows
  const int k0 = blk * L.S + t * L.m;
  const int cnt = max(0, min(L.m, min(np, (blk + 1) * L.S) - k0));
  double v[kSpMaxM];
#pragma unroll
  for (int j = 0; j < kSpMaxM; ++j) {
    v[j] = 0.0;
    if (j < cnt) {
      const int i = k0 + j;
      const double w = proj_row_value(d, i, x);
      v[j] = w;
#pragma unroll
      for (int r = 0; r < kProjMaxBorder; ++r)
        if (r < nb) acc[kProjMaxBorder + r] += d.Z[(size_t)r * np + i] * w;
    }
  }
  // border dot products over the vertices, spread over the workgroups
  if (d.nrm) {  // rows . (W x) with the normal parts
    for (int i = blk * kSpThreads + t; i < nV; i += gridDim.x * kSpThreads) {
      double x0 = x[3 * i], x1 = x[3 * i + 1], x2 = x[3 * i + 2];
      proj_w_apply(d, i, x0, x1, x2);
#pragma unroll
      for (int r = 0; r < kProjMaxBorder; ++r)
        if (r < nb) {
          const double* rv = d.rows + ((size_t)r * nV + i) * 3;
          acc[r] += rv[0] * x0 + rv[1] * x1 + rv[2] * x2;
        }
    }
  } else {
    for (int i = blk * kSpThreads + t; i < nV; i += gridDim.x * kSpThreads) {
      const double wi = d.w ? d.w[i] : 1.0;
#pragma unroll
      for (int r = 0; r < kProjMaxBorder; ++r)
        if (r < nb) {
          const double* rv = d.rows + ((size_t)r * nV + i) * 3;
          acc[r] += wi * (rv[0] * x[3 * i] + rv[1] * x[3 * i + 1] + rv[2] * x[3 * i + 2]);
        }
    }
  }
  if (np > 0) {
    tri_local_solve(d.lo, d.uinv, d.tc, L, blk, v, wa, wb);
#pragma unroll
    for (int j = 0; j < kSpMaxM; ++j)
      if (j < cnt) d.g[k0 + j] = v[j];
  }
  const int lane = t % 64, w = t / 64;
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) {
    if ((q % kProjMaxBorder) >= nb) continue;  // unused slot (uniform)
    double s = acc[q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) sred[w][q] = s;
  }
  __syncthreads();
  if (t < kProjSlots) {
    const int q = t;
    d.part[(size_t)blk * kProjSlots + q] =
        (q % kProjMaxBorder) < nb ? ((sred[0][q] + sred[1][q]) + sred[2][q]) + sred[3][q] : 0.0;
  }
}

__global__ __launch_bounds__(kSpThreads) void k_proj_solve(const ProjData d, int nblk) {
  __shared__ double tot[kProjSlots];
  __shared__ double rhs[2 * (kSpMaxB - 1)];
  const int t = threadIdx.x, nb = d.nb;
  {  // slot q = t / 16 summed over the workgroups of k_proj_rows by 16 lanes
    const int q = t / 16, sgm = t % 16;
    double v = 0.0;
    if ((q % kProjMaxBorder) < nb)
      for (int k = sgm; k < nblk; k += 16) v += d.part[(size_t)k * kProjSlots + q];
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (sgm == 0) tot[q] = v;
  }
  const TriBlocks& L = d.tri;
  const int nr = L.nr;
  for (int i = t; i < nr; i += kSpThreads) {
    const int q = i / 2;
    rhs[i] = d.g[(i % 2 == 0) ? (q + 1) * L.S - 1 : (q + 1) * L.S];
  }
  __syncthreads();
  if (t < nb) {  // yb = S^-1 (wb - Z^T wp)
    double v = 0.0;
    for (int j = 0; j < nb; ++j) v += d.Sinv[t * nb + j] * (tot[j] - tot[kProjMaxBorder + j]);
    d.yb[t] = v;
  }
  // U = M^-1 rhs: row i by two threads (halves of j), four independent partial sums each
  __shared__ double half_sum[kSpThreads];
  constexpr int kHalf = kSpThreads / 2;
  const int jh = (nr + 1) / 2;
  for (int i0 = 0; i0 < nr; i0 += kHalf) {
    const int i = i0 + t % kHalf, h = t / kHalf;
    const int j0 = h * jh, j1 = min(nr, j0 + jh);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < nr) {
      const double* col = d.Rt + i;
      int j = j0;
      for (; j + 4 <= j1; j += 4) {
        s0 += col[(size_t)j * nr] * rhs[j];
        s1 += col[(size_t)(j + 1) * nr] * rhs[j + 1];
        s2 += col[(size_t)(j + 2) * nr] * rhs[j + 2];
        s3 += col[(size_t)(j + 3) * nr] * rhs[j + 3];
      }
      for (; j < j1; ++j) s0 += col[(size_t)j * nr] * rhs[j];
    }
    half_sum[t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (h == 0 && i < nr) d.U[i] = half_sum[t] + half_sum[t + kHalf];
    __syncthreads();
  }
}

// The product operand of d.pp for the workgroup's vertices (NT threads, the
// first vertex a multiple of 32, one vertex per thread): the tile heads are
// exchanged through LDS.  Every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ void proj_prep_operand(const ProjData& d, int v, bool vert, const double (&val)[3]) {
  __shared__ double heads[NT / 32][3];
  const int lt = threadIdx.x;
  if (vert && lt % 32 == 0)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) heads[lt / 32][cc] = val[cc];
  __syncthreads();
  if (!vert) return;
  const int kt = v / 32, j = v % 32;
  const double sq = d.psqd[v];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const double h = heads[lt / 32][cc];
    d.pp[(size_t)kt * 96 + cc * 32 + j] = (float)(sq * (val[cc] - h));
    if (j == 0) d.pcref[kt * 3 + cc] = h;
  }
}

// out_v = in_v - [ sum_{path rows k at v} s(v) T_I (yp_k - (Z yb)_k) + sum_r yb[r] rows[r][v] ]
// for vertex v (the body of k_apply_CT_z); val receives out_v (xacc_v when prep_x).
// yb, U: the border solution and the reduced boundary values (global memory,
// or LDS in the fused launch).
// The loads of the last step that do not depend on the border and reduced
// solves, for a packed vertex: issued at the start of the fused launch so
// that their latency overlaps those solves (prev and in may alias out: every
// entry is read by its own thread before that thread writes it).
struct CtPre {
  ProjVert pv;
  double g[2], V[2], W[2], Z[2][kProjMaxBorder], rows[kProjMaxBorder][3], in[3];
};

__device__ __forceinline__ void ct_prefetch(const ProjData& d, int v, const double* __restrict__ in, CtPre& p) {
  const int np = d.np, nb = d.nb;
  p.pv = d.pvert[v];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int pr = p.pv.row[q];
    if (pr < 0) continue;
    p.g[q] = d.g[pr];
    p.V[q] = d.V[pr];
    p.W[q] = d.W[pr];
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) p.Z[q][r] = d.Z[(size_t)r * np + pr];
  }
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r)
    if (r < nb)
      for (int cc = 0; cc < 3; ++cc) p.rows[r][cc] = d.rows[((size_t)r * d.nV + v) * 3 + cc];
  for (int cc = 0; cc < 3; ++cc) p.in[cc] = in[3 * v + cc];
}

__device__ __forceinline__ void ct_store(const ProjData& d, int v, double (&res)[3], double* __restrict__ out,
                                         double (&val)[3]);

// apply_CT_z_vertex on prefetched loads (the same arithmetic in the same order)
__device__ __forceinline__ void ct_finish(const ProjData& d, int v, const CtPre& p, double* __restrict__ out,
                                          double (&val)[3], const double* yb, const double* U) {
  const int nb = d.nb;
  const TriBlocks& L = d.tri;
  double ybr[kProjMaxBorder];
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r) ybr[r] = r < nb ? yb[r] : 0.0;
  double acc[3] = {0, 0, 0};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int pr = p.pv.row[q];
    if (pr < 0) continue;
    double y = p.g[q];
    const int qb = pr / L.S;
    if (qb < L.B - 1) y -= p.V[q] * U[2 * qb + 1];
    if (qb > 0) y -= p.W[q] * U[2 * (qb - 1)];
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) y -= p.Z[q][r] * ybr[r];
    acc[0] += p.pv.c[q][0] * y;
    acc[1] += p.pv.c[q][1] * y;
    acc[2] += p.pv.c[q][2] * y;
  }
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r)
    if (r < nb)
      for (int cc = 0; cc < 3; ++cc) acc[cc] += ybr[r] * p.rows[r][cc];
  double res[3] = {p.in[0] - acc[0], p.in[1] - acc[1], p.in[2] - acc[2]};
  ct_store(d, v, res, out, val);
}

__device__ __forceinline__ void apply_CT_z_vertex(const ProjData& d, int v, const double* __restrict__ in,
                                                  double* __restrict__ out, double (&val)[3], const double* yb,
                                                  const double* U) {
  const int np = d.np, nb = d.nb;
  const TriBlocks& L = d.tri;
  double ybr[kProjMaxBorder];
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r) ybr[r] = r < nb ? yb[r] : 0.0;
  double acc[3] = {0, 0, 0};
  auto add_row = [&](int pr, double c0, double c1, double c2) {
    double y = d.g[pr];
    const int q = pr / L.S;
    if (q < L.B - 1) y -= d.V[pr] * U[2 * q + 1];
    if (q > 0) y -= d.W[pr] * U[2 * (q - 1)];
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) y -= d.Z[(size_t)r * np + pr] * ybr[r];
    acc[0] += c0 * y;
    acc[1] += c1 * y;
    acc[2] += c2 * y;
  };
  if (d.pvert) {
    const ProjVert pv = d.pvert[v];
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (pv.row[q] >= 0) add_row(pv.row[q], pv.c[q][0], pv.c[q][1], pv.c[q][2]);
  } else {
    for (int k = d.inc_off[v]; k < d.inc_off[v + 1]; ++k) {
      const int I = d.inc[k] >> 1;
      const int pr = d.edge_path_row[I];
      if (pr < 0) continue;
      const double sg = (d.inc[k] & 1) ? -1.0 : 1.0;
      const double* g = d.geo + 8 * (size_t)I;
      add_row(pr, sg * g[1], sg * g[2], sg * g[3]);
    }
  }
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r)
    if (r < nb)
      for (int cc = 0; cc < 3; ++cc) acc[cc] += ybr[r] * d.rows[((size_t)r * d.nV + v) * 3 + cc];
  double res[3] = {in[3 * v] - acc[0], in[3 * v + 1] - acc[1], in[3 * v + 2] - acc[2]};
  ct_store(d, v, res, out, val);
}

// out_v = beta prev_v + scale W_v res (and xacc) from res = in_v - (C^T y)_v
__device__ __forceinline__ void ct_store(const ProjData& d, int v, double (&res)[3], double* __restrict__ out,
                                         double (&val)[3]) {
  double sw = d.scale;
  if (d.nrm)  // W_v (in - C^T y) with the normal part
    proj_w_apply(d, v, res[0], res[1], res[2]);
  else if (d.w)
    sw *= d.w[v];
  for (int cc = 0; cc < 3; ++cc) {
    const double o0 = sw * res[cc];
    const double o = d.prev ? d.beta * d.prev[3 * v + cc] + o0 : o0;
    out[3 * v + cc] = o;
    val[cc] = o;
    if (d.xacc) {
      const double xa = d.xset ? o : d.xacc[3 * v + cc] + o;
      d.xacc[3 * v + cc] = xa;
      if (d.prep_x) val[cc] = xa;
    }
  }
}

__global__ __launch_bounds__(256) void k_apply_CT_z(const ProjData d, const double* __restrict__ in,
                                                    double* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool vert = v < d.nV;
  double val[3] = {0.0, 0.0, 0.0};
  if (vert) apply_CT_z_vertex(d, v, in, out, val, d.yb, d.U);
  if (d.pp) proj_prep_operand<256>(d, v, vert, val);
}

// k_proj_solve and k_apply_CT_z in one launch when the reduced system is
// small (nr <= kFuseMaxNr): every workgroup sums the partials, solves the
// border (yb) and applies M^-1 to the block-boundary values (U) itself, in
// the order k_proj_solve uses, into LDS, then applies C^T y to its vertices.
constexpr int kFuseMaxNr = 128;
constexpr int kPrefetchMaxV = 65536;  // 256 workgroups of 256 vertices
template <bool PRE>
__global__ __launch_bounds__(256) void k_solve_apply_CT_z(const ProjData d, int nblk, const double* __restrict__ in,
                                                          double* __restrict__ out) {
  __shared__ double tot[kProjSlots], ybs[kProjMaxBorder];
  __shared__ double rhs[kFuseMaxNr], Us[kFuseMaxNr], half_sum[256];
  const int t = threadIdx.x, nb = d.nb;
  const TriBlocks& L = d.tri;
  const int nr = L.nr;
  const int v = blockIdx.x * blockDim.x + t;
  const bool vert = v < d.nV;
  CtPre pre;
  if (PRE && vert && d.pvert) ct_prefetch(d, v, in, pre);
  {  // slot q = t / 16 summed over the workgroups of k_proj_rows by 16 lanes
    const int q = t / 16, sgm = t % 16;
    double v = 0.0;
    if ((q % kProjMaxBorder) < nb)
      for (int k = sgm; k < nblk; k += 16) v += d.part[(size_t)k * kProjSlots + q];
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (sgm == 0) tot[q] = v;
  }
  for (int i = t; i < nr; i += 256) {
    const int q = i / 2;
    rhs[i] = d.g[(i % 2 == 0) ? (q + 1) * L.S - 1 : (q + 1) * L.S];
  }
  __syncthreads();
  if (t < nb) {  // yb = S^-1 (wb - Z^T wp)
    double v = 0.0;
    for (int j = 0; j < nb; ++j) v += d.Sinv[t * nb + j] * (tot[j] - tot[kProjMaxBorder + j]);
    ybs[t] = v;
  }
  {  // U = M^-1 rhs: row i by two threads (halves of j), four independent partial sums each
    constexpr int kHalf = 128;
    const int i = t % kHalf, h = t / kHalf;
    const int jh = (nr + 1) / 2;
    const int j0 = h * jh, j1 = min(nr, j0 + jh);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < nr) {
      const double* col = d.Rt + i;
      int j = j0;
      for (; j + 4 <= j1; j += 4) {
        s0 += col[(size_t)j * nr] * rhs[j];
        s1 += col[(size_t)(j + 1) * nr] * rhs[j + 1];
        s2 += col[(size_t)(j + 2) * nr] * rhs[j + 2];
        s3 += col[(size_t)(j + 3) * nr] * rhs[j + 3];
      }
      for (; j < j1; ++j) s0 += col[(size_t)j * nr] * rhs[j];
    }
    half_sum[t] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (h == 0 && i < nr) Us[i] = half_sum[t] + half_sum[t + kHalf];
  }
  __syncthreads();
  double val[3] = {0.0, 0.0, 0.0};
  if (vert) {
    if (PRE && d.pvert) ct_finish(d, v, pre, out, val, ybs, Us);
    else apply_CT_z_vertex(d, v, in, out, val, ybs, Us);
  }
  if (d.pp) proj_prep_operand<256>(d, v, vert, val);
}

// The last step of k_proj_small for vertex t; val receives out_t (xacc_t when
// prep_x); pin and ain hold prev_t and xacc_t, loaded before the barriers.
// Z of the vertex's path rows for the first kSmallPreB border rows, loaded
// before the barriers of k_proj_small (the rest is loaded at the end)
constexpr int kSmallPreB = 4;

__device__ __forceinline__ void proj_small_vertex(const ProjData& d, int t, double* __restrict__ out,
                                                  const ProjVert& pv, double w_t, double x0, double x1, double x2,
                                                  const double* yps, const double* ybs, const double (&pin)[3],
                                                  const double (&ain)[3], const double (&zp)[2][kSmallPreB],
                                                  double (&val)[3]) {
  const int np = d.np, nV = d.nV, nb = d.nb;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int p = pv.row[q];
    if (p < 0) continue;
    double y = yps[p];
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) y -= (r < kSmallPreB ? zp[q][r < kSmallPreB ? r : 0] : d.Z[(size_t)r * np + p]) * ybs[r];
    a0 += pv.c[q][0] * y;
    a1 += pv.c[q][1] * y;
    a2 += pv.c[q][2] * y;
  }
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r)
    if (r < nb) {
      const double* rv = d.rows + ((size_t)r * nV + t) * 3;
      a0 += ybs[r] * rv[0];
      a1 += ybs[r] * rv[1];
      a2 += ybs[r] * rv[2];
    }
  double o[3];
  if (d.nrm) {  // scale W_t (x - C^T y)
    double r0 = x0 - a0, r1 = x1 - a1, r2 = x2 - a2;
    proj_w_apply(d, t, r0, r1, r2);
    o[0] = d.scale * r0;
    o[1] = d.scale * r1;
    o[2] = d.scale * r2;
  } else {
    const double sw = d.scale * w_t;
    o[0] = sw * (x0 - a0);
    o[1] = sw * (x1 - a1);
    o[2] = sw * (x2 - a2);
  }
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    if (d.prev) o[cc] += d.beta * pin[cc];
    out[3 * t + cc] = o[cc];
    val[cc] = o[cc];
    if (d.xacc) {
      const double xa = d.xset ? o[cc] : ain[cc] + o[cc];
      d.xacc[3 * t + cc] = xa;
      if (d.prep_x) val[cc] = xa;
    }
  }
}

// The same projector in one workgroup and one launch for the coarse
// multigrid levels (np, nV <= kTriThreads, so the path is one block; packed
// rows and vertices), where three launches cost more than the work: thread t
// owns path row t and vertex t.  Everything that does not depend on x is
// loaded first; the partial sums are reduced in the workgroup, the
// tridiagonal solve is one scan per direction with one row per thread, and
// yp stays in LDS.
__global__ __launch_bounds__(kTriThreads) void k_proj_small(const ProjData d, const double* __restrict__ x,
                                                            double* __restrict__ out) {
  __shared__ double yps[kTriThreads];
  __shared__ double red[kTriWaves][kProjSlots];
  __shared__ double tot[kProjSlots], ybs[kProjMaxBorder];
  __shared__ double wa[kTriWaves], wbs[kTriWaves];
  static_assert(kProjSlots == kTriWaves, "one slot per group of 16 lanes");
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int np = d.np, nV = d.nV, nb = d.nb;
  const bool row = t < np, vert = t < nV;
  ProjRow pr_t;
  double l_t = 0.0, ui_t = 0.0, c_t = 0.0;
  if (row) {
    pr_t = d.prow[t];
    l_t = d.lo[t];
    ui_t = d.uinv[t];
    c_t = d.tc[t];
  }
  ProjVert pv;
  pv.row[0] = pv.row[1] = -1;
  if (vert) pv = d.pvert[t];
  double zp[2][kSmallPreB];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int r = 0; r < kSmallPreB; ++r)
      zp[q][r] = (pv.row[q] >= 0 && r < nb) ? d.Z[(size_t)r * np + pv.row[q]] : 0.0;
  // the last step's inputs that do not depend on x, loaded ahead of the barriers
  double pin[3] = {0.0, 0.0, 0.0}, ain[3] = {0.0, 0.0, 0.0};
  if (vert) {
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      if (d.prev) pin[cc] = d.prev[3 * t + cc];
      if (d.xacc && !d.xset) ain[cc] = d.xacc[3 * t + cc];
    }
  }
  double acc[kProjSlots];
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) acc[q] = 0.0;
  double wv = 0.0;
  if (row) {
    const int a = pr_t.ends.x, b = pr_t.ends.y;
    if (d.nrm) {
      double a0 = x[3 * a], a1 = x[3 * a + 1], a2 = x[3 * a + 2];
      double b0 = x[3 * b], b1 = x[3 * b + 1], b2 = x[3 * b + 2];
      proj_w_apply(d, a, a0, a1, a2);
      proj_w_apply(d, b, b0, b1, b2);
      wv = pr_t.t[0] * (a0 - b0) + pr_t.t[1] * (a1 - b1) + pr_t.t[2] * (a2 - b2);
    } else {
      const double wa = d.w ? d.w[a] : 1.0, wb = d.w ? d.w[b] : 1.0;
      wv = pr_t.t[0] * (wa * x[3 * a] - wb * x[3 * b]) + pr_t.t[1] * (wa * x[3 * a + 1] - wb * x[3 * b + 1]) +
           pr_t.t[2] * (wa * x[3 * a + 2] - wb * x[3 * b + 2]);
    }
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) acc[kProjMaxBorder + r] = d.Z[(size_t)r * np + t] * wv;
  }
  const double x0 = vert ? x[3 * t] : 0.0, x1 = vert ? x[3 * t + 1] : 0.0, x2 = vert ? x[3 * t + 2] : 0.0;
  const double w_t = (vert && d.w) ? d.w[t] : 1.0;
  if (vert && d.nrm) {  // rows . (W x)
    double y0 = x0, y1 = x1, y2 = x2;
    proj_w_apply(d, t, y0, y1, y2);
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) {
        const double* rv = d.rows + ((size_t)r * nV + t) * 3;
        acc[r] = rv[0] * y0 + rv[1] * y1 + rv[2] * y2;
      }
  } else if (vert) {
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) {
        const double* rv = d.rows + ((size_t)r * nV + t) * 3;
        acc[r] = w_t * (rv[0] * x0 + rv[1] * x1 + rv[2] * x2);
      }
  }
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) {
    if ((q % kProjMaxBorder) >= nb) continue;  // unused slot (uniform)
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[w][q] = v;
  }
  __syncthreads();
  if (t < kTriWaves * kProjSlots) {  // slot q = t / 16 summed over the 16 waves by 16 lanes
    const int q = t / kTriWaves, ww = t % kTriWaves;
    double v = (q % kProjMaxBorder) < nb ? red[ww][q] : 0.0;
    for (int off = kTriWaves / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (ww == 0) tot[q] = v;
  }
  __syncthreads();
  if (t < nb) {  // yb = S^-1 (wb - Z^T wp)
    double v = 0.0;
    for (int j = 0; j < nb; ++j) v += d.Sinv[t * nb + j] * (tot[j] - tot[kProjMaxBorder + j]);
    ybs[t] = v;
  }
  if (np > 0) {
    // forward z = b - l z_prev, then backward y = (z - c y_next) / u, one row per thread
    double A = row ? -l_t : 1.0, B = row ? wv : 0.0;
    scan_compose<kTriWaves>(A, B, false, wa, wbs);
    const double z = row ? -l_t * B + wv : 0.0;
    __syncthreads();  // the LDS slots are reused by the second scan
    A = row ? -c_t * ui_t : 1.0;
    B = row ? z * ui_t : 0.0;
    scan_compose<kTriWaves>(A, B, true, wa, wbs);
    if (row) yps[t] = -c_t * ui_t * B + z * ui_t;
  }
  __syncthreads();
  double val[3] = {0.0, 0.0, 0.0};
  if (vert) proj_small_vertex(d, t, out, pv, w_t, x0, x1, x2, yps, ybs, pin, ain, zp, val);
  if (d.pp) proj_prep_operand<kTriThreads>(d, t, vert, val);
}


void cons_project_fused(const ProjData& d, const double* in, double* out, hipStream_t s) {
  if (d.prow && d.pvert && d.np <= kTriThreads && d.nV <= kTriThreads && d.tri.B == 1) {
    hipLaunchKernelGGL(k_proj_small, dim3(1), dim3(kTriThreads), 0, s, d, in, out);
    return;
  }
  // one workgroup per block of path rows; at least enough for the vertices' border sums
  const int nblk = std::max(d.np > 0 ? d.tri.B : 1, std::min(64, cdiv(d.nV, kSpThreads)));
  hipLaunchKernelGGL(k_proj_rows, dim3(nblk), dim3(kSpThreads), 0, s, d, in);
  if (d.tri.nr <= kFuseMaxNr) {
    // the prefetching variant holds more registers: for grids of one wave of workgroups over the chip
    if (d.nV <= kPrefetchMaxV)
      hipLaunchKernelGGL(k_solve_apply_CT_z<true>, dim3(cdiv(d.nV, 256)), dim3(256), 0, s, d, nblk, in, out);
    else
      hipLaunchKernelGGL(k_solve_apply_CT_z<false>, dim3(cdiv(d.nV, 256)), dim3(256), 0, s, d, nblk, in, out);
    return;
  }
  hipLaunchKernelGGL(k_proj_solve, dim3(1), dim3(kSpThreads), 0, s, d, nblk);
  hipLaunchKernelGGL(k_apply_CT_z, dim3(cdiv(d.nV, 256)), dim3(256), 0, s, d, in, out);
}

// Packed rows and vertices (vertex degree <= 2).
__global__ void k_proj_pack(const double* __restrict__ geo, const int2* __restrict__ edges,
                            const int* __restrict__ path_edge, int np, const int* __restrict__ inc_off,
                            const int* __restrict__ inc, const int* __restrict__ edge_path_row, int nV,
                            ProjRow* __restrict__ prow, ProjVert* __restrict__ pvert) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) {
    const int I = path_edge[i];
    const double* g = geo + 8 * (size_t)I;
    ProjRow p;
    p.t[0] = g[1];
    p.t[1] = g[2];
    p.t[2] = g[3];
    p.ends = edges[I];
    prow[i] = p;
  }
  if (i < nV) {
    ProjVert pv;
    int q = 0;
    for (int k = inc_off[i]; k < inc_off[i + 1] && q < 2; ++k) {
      const int I = inc[k] >> 1;
      const int pr = edge_path_row[I];
      if (pr < 0) continue;
      const double sg = (inc[k] & 1) ? -1.0 : 1.0;
      const double* g = geo + 8 * (size_t)I;
      pv.row[q] = pr;
      pv.c[q][0] = sg * g[1];
      pv.c[q][1] = sg * g[2];
      pv.c[q][2] = sg * g[3];
      ++q;
    }
    for (; q < 2; ++q) {
      pv.row[q] = -1;
      pv.c[q][0] = pv.c[q][1] = pv.c[q][2] = 0.0;
    }
    pvert[i] = pv;
  }
}

void cons_project_pack(const double* geo, const int2* edges, const int* path_edge, int np, const int* inc_off,
                       const int* inc, const int* edge_path_row, int nV, ProjRow* prow, ProjVert* pvert,
                       hipStream_t s) {
  const int n = std::max(np, nV);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_proj_pack, dim3(cdiv(n, 256)), dim3(256), 0, s, geo, edges, path_edge, np, inc_off, inc,
                     edge_path_row, nV, prow, pvert);
}

// ---------------------------------------------------------------------------
// misc small kernels for the solvers
// ---------------------------------------------------------------------------
// gamma_out = gamma - tau * g / gnorm   (gnorm read on device)
__global__ void k_trial(const double* __restrict__ gamma, const double* __restrict__ g, const double* __restrict__ gg,
                        double tau, double* __restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = gamma[i] - tau * g[i] / sqrt(gg[0]);
}

void vec_trial(const double* gamma, const double* g, const double* gg, double tau, double* out, int n,
               hipStream_t s) {
  hipLaunchKernelGGL(k_trial, dim3(cdiv(n, 256)), dim3(256), 0, s, gamma, g, gg, tau, out, n);
}

// Dense Abar + C^T C for the direct path: H[3v+a][3w+b] = A[v][w] delta_ab + sum_r C[r][3v+a] C[r][3w+b].
__global__ void k_build_H(const double* __restrict__ A, const double* __restrict__ CtC, int nV,
                          double* __restrict__ H) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y * blockDim.y + threadIdx.y;
  int n = 3 * nV;
  if (i >= n || j >= n) return;
  double v = CtC[(size_t)i * n + j];
  if (i % 3 == j % 3) v += A[(size_t)(i / 3) * nV + j / 3];
  H[(size_t)i * n + j] = v;
}

void dense_build_H(const double* A, const double* CtC, int nV, double* H, hipStream_t s) {
  int n = 3 * nV;
  dim3 b(16, 16), g(cdiv(n, 16), cdiv(n, 16));
  hipLaunchKernelGGL(k_build_H, g, b, 0, s, A, CtC, nV, H);
}

// Dense constraint matrix in the external row order (bary, total, points, edges)
// from the border rows, the point rows and the edge rows: Cd[k][3 nV].  An
// edge whose ends are both pinned (free[v] = 0) keeps a zero row: its
// linearised length is fixed by the point rows, so the row would be dependent.
__global__ void k_dense_C_edges(const double* __restrict__ geo, const int2* __restrict__ edges, int nE, int row0,
                                int nV, const double* __restrict__ free, double* __restrict__ Cd) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const double* g = geo + 8 * (size_t)I;
  int2 e = edges[I];
  if (free && free[e.x] == 0.0 && free[e.y] == 0.0) return;
  double* r = Cd + (size_t)(row0 + I) * 3 * nV;
  for (int cc = 0; cc < 3; ++cc) {
    r[3 * e.x + cc] = g[1 + cc];
    r[3 * e.y + cc] = -g[1 + cc];
  }
}

void dense_C_edges(const double* geo, const int2* edges, int nE, int row0, int nV, const double* free, double* Cd,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_dense_C_edges, dim3(cdiv(nE, 256)), dim3(256), 0, s, geo, edges, nE, row0, nV, free, Cd);
}

// point rows (Sec. 7.1, Phi = gamma_i - x_i): row row0 + 3 j + c of Cd is e_c at vertex pt[j]
__global__ void k_dense_C_points(const int* __restrict__ pt, int npt, int row0, int nV, double* __restrict__ Cd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * npt) return;
  Cd[(size_t)(row0 + i) * 3 * nV + 3 * pt[i / 3] + i % 3] = 1.0;
}

void dense_C_points(const int* pt, int npt, int row0, int nV, double* Cd, hipStream_t s) {
  if (npt > 0) hipLaunchKernelGGL(k_dense_C_points, dim3(cdiv(3 * npt, 64)), dim3(64), 0, s, pt, npt, row0, nV, Cd);
}

// A[i][i] = 1 where the diagonal of the SPD matrix A [n][n] is exactly zero (a zero row and column)
__global__ void k_unit_zero_diag(double* __restrict__ A, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && A[(size_t)i * n + i] == 0.0) A[(size_t)i * n + i] = 1.0;
}

void unit_zero_diag(double* A, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_unit_zero_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, A, n);
}

// out[v] = (w ? w[v] : 1) free[v]: the weights of C W C^T with the pinned vertices' columns removed
__global__ void k_free_weights(const double* __restrict__ w, const double* __restrict__ free, int nV,
                               double* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nV) out[v] = (w ? w[v] : 1.0) * free[v];
}

void free_weights(const double* w, const double* free, int nV, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_free_weights, dim3(cdiv(nV, 256)), dim3(256), 0, s, w, free, nV, out);
}

// x_v <- W_v x_v, W_v = w[v] (I - n_v n_v^T) (nrm may be null)
__global__ void k_mask_vertices(double* __restrict__ x, const double* __restrict__ w, const double* __restrict__ nrm,
                                int nV) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double x0 = x[3 * v], x1 = x[3 * v + 1], x2 = x[3 * v + 2];
  if (nrm) {
    const double* n = nrm + 3 * (size_t)v;
    const double p = n[0] * x0 + n[1] * x1 + n[2] * x2;
    x0 -= p * n[0];
    x1 -= p * n[1];
    x2 -= p * n[2];
  }
  const double s = w[v];
  x[3 * v] = x0 * s;
  x[3 * v + 1] = x1 * s;
  x[3 * v + 2] = x2 * s;
}

void mask_vertices(double* x, const double* w, const double* nrm, int nV, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_vertices, dim3(cdiv(nV, 256)), dim3(256), 0, s, x, w, nrm, nV);
}

}  // namespace rc
