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

// ---------------------------------------------------------------------------
// blocked dense Cholesky (lower, row-major, in place), block size 32
// ---------------------------------------------------------------------------
constexpr int kNB = 32;

__global__ void k_potrf_diag(double* __restrict__ A, int n, int k0, int* __restrict__ info) {
  __shared__ double L[kNB][kNB + 1];
  const int nb = min(kNB, n - k0);
  const int tid = threadIdx.x;  // 256 threads
  for (int idx = tid; idx < nb * nb; idx += 256) {
    int i = idx / nb, j = idx % nb;
    L[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      double d = L[k][k];
      if (!(d > 0.0)) {
        if (info[0] == 0) info[0] = k0 + k + 1;
        d = 1.0;
      }
      L[k][k] = sqrt(d);
    }
    __syncthreads();
    const double piv = L[k][k];
    for (int i = k + 1 + tid; i < nb; i += 256) L[i][k] /= piv;
    __syncthreads();
    for (int idx = tid; idx < (nb - k - 1) * (nb - k - 1); idx += 256) {
      int i = k + 1 + idx / (nb - k - 1), j = k + 1 + idx % (nb - k - 1);
      if (j <= i) L[i][j] -= L[i][k] * L[j][k];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nb * nb; idx += 256) {
    int i = idx / nb, j = idx % nb;
    A[(size_t)(k0 + i) * n + k0 + j] = (j <= i) ? L[i][j] : 0.0;
  }
}

// Rows below the diagonal block: A[i, k0:k0+nb] <- A[i, k0:k0+nb] L_kk^-T.
// One thread per row; 64 rows per block.
__global__ void k_trsm_panel(double* __restrict__ A, int n, int k0) {
  __shared__ double L[kNB][kNB + 1];
  const int nb = min(kNB, n - k0);
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    int i = idx / nb, j = idx % nb;
    L[i][j] = A[(size_t)(k0 + i) * n + k0 + j];
  }
  __syncthreads();
  const int i = k0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[kNB];
  for (int j = 0; j < nb; ++j) x[j] = A[(size_t)i * n + k0 + j];
  for (int j = 0; j < nb; ++j) {
    double v = x[j];
    for (int p = 0; p < j; ++p) v -= x[p] * L[j][p];
    x[j] = v / L[j][j];
  }
  for (int j = 0; j < nb; ++j) A[(size_t)i * n + k0 + j] = x[j];
}

// Trailing update A[i,j] -= sum_p A[i,k0+p] A[j,k0+p] for i >= j >= k1 = k0+nb.
// 32x32 output tiles, 256 threads, each 4 outputs.
__global__ void k_syrk_update(double* __restrict__ A, int n, int k0) {
  const int nb = min(kNB, n - k0);
  const int k1 = k0 + nb;
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  const int i0 = k1 + ti * 32, j0 = k1 + tj * 32;
  __shared__ double Pi[32][kNB + 1], Pj[32][kNB + 1];
  for (int idx = threadIdx.x; idx < 32 * nb; idx += 256) {
    int r = idx / nb, p = idx % nb;
    Pi[r][p] = (i0 + r < n) ? A[(size_t)(i0 + r) * n + k0 + p] : 0.0;
    Pj[r][p] = (j0 + r < n) ? A[(size_t)(j0 + r) * n + k0 + p] : 0.0;
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    int idx = threadIdx.x + 256 * q;
    int r = idx / 32, cc = idx % 32;
    int i = i0 + r, j = j0 + cc;
    if (i >= n || j >= n || j > i) continue;
    double s = 0.0;
    for (int p = 0; p < nb; ++p) s += Pi[r][p] * Pj[cc][p];
    A[(size_t)i * n + j] -= s;
  }
}

void dense_cholesky(double* A, int n, int* info, hipStream_t s) {
  hipMemsetAsync(info, 0, sizeof(int), s);
  for (int k0 = 0; k0 < n; k0 += kNB) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, A, n, k0, info);
    const int rest = n - k0 - kNB;
    if (rest <= 0) break;
    hipLaunchKernelGGL(k_trsm_panel, dim3(cdiv(rest, 64)), dim3(64), 0, s, A, n, k0);
    const int nt = cdiv(rest, 32);
    hipLaunchKernelGGL(k_syrk_update, dim3(nt, nt), dim3(256), 0, s, A, n, k0);
  }
}

// L L^T X = B, B is n x m row-major; each workgroup owns up to 16
// right-hand-side columns.
constexpr int kSolveCols = 16;
constexpr int kSolveRows = 32;  // row block of the blocked substitution

// Blocked substitution: for each block of 32 rows, the block's triangular
// system is solved in LDS (one thread per right-hand-side column, no barriers
// inside), then the rows after it (forward) or before it (backward) take a
// rank-32 update.  512 threads per workgroup, kSolveCols columns.
__global__ __launch_bounds__(512) void k_chol_solve(const double* __restrict__ L, double* __restrict__ B, int n,
                                                     int m) {
  __shared__ double Ld[kSolveRows][kSolveRows + 1];
  __shared__ double Bb[kSolveRows][kSolveCols + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * kSolveCols;
  const int mc = min(kSolveCols, m - c0);
  // forward: L y = b
  for (int j0 = 0; j0 < n; j0 += kSolveRows) {
    const int nb = min(kSolveRows, n - j0);
    for (int idx = tid; idx < nb * nb; idx += 512) Ld[idx / nb][idx % nb] = L[(size_t)(j0 + idx / nb) * n + j0 + idx % nb];
    for (int idx = tid; idx < nb * mc; idx += 512) Bb[idx / mc][idx % mc] = B[(size_t)(j0 + idx / mc) * m + c0 + idx % mc];
    __syncthreads();
    if (tid < mc) {
      for (int i = 0; i < nb; ++i) {
        double v = Bb[i][tid];
        for (int jj = 0; jj < i; ++jj) v -= Ld[i][jj] * Bb[jj][tid];
        Bb[i][tid] = v / Ld[i][i];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * mc; idx += 512) B[(size_t)(j0 + idx / mc) * m + c0 + idx % mc] = Bb[idx / mc][idx % mc];
    for (int idx = tid; idx < (n - j0 - nb) * mc; idx += 512) {
      const int i = j0 + nb + idx / mc, c = idx % mc;
      const double* Li = L + (size_t)i * n + j0;
      double v = 0.0;
      for (int jj = 0; jj < nb; ++jj) v += Li[jj] * Bb[jj][c];
      B[(size_t)i * m + c0 + c] -= v;
    }
    __syncthreads();
  }
  // backward: L^T x = y, blocks from the last
  for (int j0 = ((n - 1) / kSolveRows) * kSolveRows; j0 >= 0; j0 -= kSolveRows) {
    const int nb = min(kSolveRows, n - j0);
    for (int idx = tid; idx < nb * nb; idx += 512) Ld[idx / nb][idx % nb] = L[(size_t)(j0 + idx / nb) * n + j0 + idx % nb];
    for (int idx = tid; idx < nb * mc; idx += 512) Bb[idx / mc][idx % mc] = B[(size_t)(j0 + idx / mc) * m + c0 + idx % mc];
    __syncthreads();
    if (tid < mc) {
      for (int i = nb - 1; i >= 0; --i) {
        double v = Bb[i][tid];
        for (int jj = i + 1; jj < nb; ++jj) v -= Ld[jj][i] * Bb[jj][tid];
        Bb[i][tid] = v / Ld[i][i];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * mc; idx += 512) B[(size_t)(j0 + idx / mc) * m + c0 + idx % mc] = Bb[idx / mc][idx % mc];
    // rows i < j0: b_i -= sum_jj L[j0 + jj][i] x_{j0 + jj}
    for (int idx = tid; idx < j0 * mc; idx += 512) {
      const int i = idx / mc, c = idx % mc;
      double v = 0.0;
      for (int jj = 0; jj < nb; ++jj) v += L[(size_t)(j0 + jj) * n + i] * Bb[jj][c];
      B[(size_t)i * m + c0 + c] -= v;
    }
    __syncthreads();
  }
}

void dense_chol_solve(const double* L, double* B, int n, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_solve, dim3(cdiv(m, kSolveCols)), dim3(512), 0, s, L, B, n, m);
}

// C[m x n] = op(A) op(B) + beta C, row-major; op(A) is m x k (A stored k x m
// when transA), op(B) is k x n (B stored n x k when transB).
__global__ void k_gemm(const double* __restrict__ A, const double* __restrict__ B, double* __restrict__ C, int m,
                       int n, int k, double beta, int transA, int transB) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= m || j >= n) return;
  double s = 0.0;
  for (int p = 0; p < k; ++p) {
    const double av = transA ? A[(size_t)p * m + i] : A[(size_t)i * k + p];
    const double bv = transB ? B[(size_t)j * k + p] : B[(size_t)p * n + j];
    s += av * bv;
  }
  C[(size_t)i * n + j] = s + (beta != 0.0 ? beta * C[(size_t)i * n + j] : 0.0);
}

void dense_gemm(const double* A, const double* B, double* C, int m, int n, int k, double beta, bool transA,
                hipStream_t s, bool transB) {
  dim3 b(16, 16), g(cdiv(n, 16), cdiv(m, 16));
  hipLaunchKernelGGL(k_gemm, g, b, 0, s, A, B, C, m, n, k, beta, transA ? 1 : 0, transB ? 1 : 0);
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
// tridiagonal systems: Thomas factorisation once, solves by parallel scans
// ---------------------------------------------------------------------------
// Rows k < n: a[k] y[k-1] + d[k] y[k] + c[k] y[k+1] = b[k] with a[0] = c[n-1] = 0
// (zero couplings also separate independent segments).  The factorisation
// l[k] = a[k] / u[k-1], u[k] = d[k] - l[k] c[k-1] is a nonlinear recurrence and
// runs in one wave once per system; it stores l and 1/u.  A solve is two
// first-order linear recurrences, forward  z[k] = b[k] - l[k] z[k-1]  and
// backward  y[k] = (z[k] - c[k] y[k+1]) / u[k].  Each is an affine map per row;
// one workgroup composes the maps of contiguous chunks per thread (held in
// registers up to 16 rows per thread), scans the chunk composites across the
// workgroup (wave shuffles, then one LDS exchange of the 16 wave totals), and
// then replays its chunk.
// The system is symmetric positive definite (a constraint Gram matrix), so
// the factorisation needs no pivoting.
__device__ __forceinline__ double readlane_f64(double v, int j) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, j);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), j);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One wave: the coefficients of 64 rows at a time are loaded coalesced and
// handed to the recurrence by lane reads; lane j keeps row j's factors.
__global__ __launch_bounds__(64) void k_tridiag_factor(const double* __restrict__ a, const double* __restrict__ d,
                                                       const double* __restrict__ c, int n, double* __restrict__ lo,
                                                       double* __restrict__ uinv, int* __restrict__ info) {
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x;
  double u_prev = 1.0, c_prev = 0.0;
  int bad = 0;
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int k = k0 + lane;
    const double ak = k < n ? a[k] : 0.0, dk = k < n ? d[k] : 1.0, ck = k < n ? c[k] : 0.0;
    const int cnt = min(64, n - k0);
    double my_l = 0.0, my_ui = 0.0;
    for (int j = 0; j < cnt; ++j) {
      const double aj = readlane_f64(ak, j), dj = readlane_f64(dk, j);
      const double l = (k0 + j == 0) ? 0.0 : aj / u_prev;
      const double u = dj - l * c_prev;
      if (!(u > 0.0)) bad = k0 + j + 1;
      if (lane == j) {
        my_l = l;
        my_ui = 1.0 / u;
      }
      u_prev = u;
      c_prev = readlane_f64(ck, j);
    }
    if (k < n) {
      lo[k] = my_l;
      uinv[k] = my_ui;
    }
  }
  if (lane == 0) info[0] = bad;
}

constexpr int kTriThreads = 1024;
constexpr int kTriWaves = kTriThreads / 64;
constexpr int kTriReg = 16;  // rows per thread held in registers (n <= 16,384); longer chunks reload

// Composite affine maps: (a, b) is v -> a v + b.  scan_compose returns, for
// every thread, the composite of all maps of the threads before it (in scan
// order: increasing t, or decreasing t when `rev`), i.e. the map from the
// value entering the recurrence to the value entering this thread's chunk.
// Within a wave: shuffles; across waves: one LDS exchange (2 barriers).
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
    const int ww = rev ? kTriWaves - 1 - lane : lane;
    double ta = lane < kTriWaves ? wa[ww] : 1.0, tb = lane < kTriWaves ? wb[ww] : 0.0;
#pragma unroll
    for (int off = 1; off < kTriWaves; off <<= 1) {
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
    if (lane < kTriWaves) {
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

// y = K^-1 b for the factorised tridiagonal K, by one workgroup of
// kTriThreads threads (every thread must call it); wa, wb: LDS [kTriWaves].
// Thread t owns rows t m .. t m + m - 1 (m = ceil(n / kTriThreads)).  With
// Chunked, every array is stored chunk-transposed: row t m + j at position
// j kTriThreads + t (tri_chunk_pos), so that the j-th row of all threads is one
// coalesced load; otherwise arrays are in row order.
__host__ __device__ __forceinline__ int tri_chunk_pos(int k, int m) { return (k % m) * kTriThreads + k / m; }

template <bool Chunked>
__device__ __forceinline__ void tridiag_solve_wg(const double* __restrict__ lo, const double* __restrict__ uinv,
                                                 const double* __restrict__ c, const double* __restrict__ b,
                                                 double* __restrict__ y, int n, double* wa, double* wb) {
  const int t = threadIdx.x;
  const int m = (n + kTriThreads - 1) / kTriThreads;
  const int k0 = min(n, t * m), k1 = min(n, k0 + m), cnt = k1 - k0;
  // position of the thread's j-th row
  auto at = [&](int j) { return Chunked ? j * kTriThreads + t : k0 + j; };
  const bool reg = m <= kTriReg;
  double rl[kTriReg], rz[kTriReg];
  // forward: z[k] = -l[k] z[k-1] + b[k]; chunk composite z_out = A z_in + B
  double A = 1.0, B = 0.0;
  if (reg) {
#pragma unroll
    for (int j = 0; j < kTriReg; ++j) {
      rl[j] = j < cnt ? lo[at(j)] : 0.0;
      rz[j] = j < cnt ? b[at(j)] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kTriReg; ++j)
      if (j < cnt) {
        A = -rl[j] * A;
        B = -rl[j] * B + rz[j];
      }
  } else {
    for (int j = 0; j < cnt; ++j) {
      const double l = lo[at(j)];
      A = -l * A;
      B = -l * B + b[at(j)];
    }
  }
  scan_compose(A, B, false, wa, wb);
  double zin = B;  // z before the chunk (z[-1] = 0)
  if (reg) {
#pragma unroll
    for (int j = 0; j < kTriReg; ++j)
      if (j < cnt) {
        zin = -rl[j] * zin + rz[j];
        rz[j] = zin;
      }
  } else {
    for (int j = 0; j < cnt; ++j) {
      zin = -lo[at(j)] * zin + b[at(j)];
      y[at(j)] = zin;
    }
  }
  __syncthreads();  // the LDS slots are reused by the second scan
  // backward: y[k] = -c[k] uinv[k] y[k+1] + z[k] uinv[k], scanned from the end
  A = 1.0;
  B = 0.0;
  if (reg) {
    // rl <- -c/u (the coupling), rz <- z/u (the offset)
#pragma unroll
    for (int j = 0; j < kTriReg; ++j) {
      const double ui = j < cnt ? uinv[at(j)] : 0.0;
      rl[j] = j < cnt ? -c[at(j)] * ui : 0.0;
      rz[j] *= ui;
    }
#pragma unroll
    for (int j = kTriReg - 1; j >= 0; --j)
      if (j < cnt) {
        A = rl[j] * A;
        B = rl[j] * B + rz[j];
      }
    scan_compose(A, B, true, wa, wb);
    double yin = B;  // y after the chunk (y[n] = 0)
#pragma unroll
    for (int j = kTriReg - 1; j >= 0; --j)
      if (j < cnt) {
        yin = rl[j] * yin + rz[j];
        rz[j] = yin;
      }
#pragma unroll
    for (int j = 0; j < kTriReg; ++j)
      if (j < cnt) y[at(j)] = rz[j];
  } else {
    for (int j = cnt - 1; j >= 0; --j) {
      const double ui = uinv[at(j)];
      A = -c[at(j)] * ui * A;
      B = -c[at(j)] * ui * B + y[at(j)] * ui;
    }
    scan_compose(A, B, true, wa, wb);
    double yin = B;
    for (int j = cnt - 1; j >= 0; --j) {
      const double ui = uinv[at(j)];
      yin = -c[at(j)] * ui * yin + y[at(j)] * ui;
      y[at(j)] = yin;
    }
  }
}

__global__ __launch_bounds__(kTriThreads) void k_tridiag_solve(const double* __restrict__ lo,
                                                                const double* __restrict__ uinv,
                                                                const double* __restrict__ c,
                                                                const double* __restrict__ b, double* __restrict__ y,
                                                                int n) {
  __shared__ double wa[kTriWaves], wb[kTriWaves];
  tridiag_solve_wg<false>(lo, uinv, c, b, y, n, wa, wb);
}

void tridiag_factor(const double* a, const double* d, const double* c, int n, double* lo, double* uinv, int* info,
                    hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tridiag_factor, dim3(1), dim3(64), 0, s, a, d, c, n, lo, uinv, info);
}

void tridiag_solve(const double* lo, const double* uinv, const double* c, const double* b, double* y, int n,
                   hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tridiag_solve, dim3(1), dim3(kTriThreads), 0, s, lo, uinv, c, b, y, n);
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

// Border rows as dense vertex vectors rows[r][nV][3].
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

void cons_border_rows(const double* geo, const int* inc_off, const int* inc, const int2* edges, const double* x0,
                      int nV, int bary, int total, const int* cut_edge, int ncut, double* rows, int nrows,
                      hipStream_t s) {
  hipMemsetAsync(rows, 0, sizeof(double) * (size_t)nrows * nV * 3, s);
  hipLaunchKernelGGL(k_border_rows, dim3(cdiv(nV, 256)), dim3(256), 0, s, geo, inc_off, inc, x0, nV, bary, total,
                     rows);
  if (ncut > 0)
    hipLaunchKernelGGL(k_cut_rows, dim3(cdiv(ncut, 256)), dim3(256), 0, s, geo, edges, cut_edge, ncut,
                       3 * bary + total, nV, rows);
}

// Tridiagonal coefficients of C_p C_p^T over the path rows (chain order):
// diag 2, off-diagonal s_I(v) s_J(v) T_I.T_J for consecutive rows sharing v.
__global__ void k_path_coeffs(const double* __restrict__ geo, const int2* __restrict__ edges,
                              const int* __restrict__ path_edge, const int* __restrict__ path_prev, int np,
                              double* __restrict__ ta, double* __restrict__ td, double* __restrict__ tc) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  td[k] = 2.0;
  const int I = path_edge[k];
  if (path_prev[k]) {
    const int J = path_edge[k - 1];
    int2 ei = edges[I], ej = edges[J];
    // shared vertex and the signs (+1 at i1, -1 at i2)
    double si, sj;
    if (ei.x == ej.x) { si = 1; sj = 1; }
    else if (ei.x == ej.y) { si = 1; sj = -1; }
    else if (ei.y == ej.x) { si = -1; sj = 1; }
    else { si = -1; sj = -1; }
    const double* gi = geo + 8 * (size_t)I;
    const double* gj = geo + 8 * (size_t)J;
    const double v = si * sj * (gi[1] * gj[1] + gi[2] * gj[2] + gi[3] * gj[3]);
    ta[k] = v;
    tc[k - 1] = v;
  } else {
    ta[k] = 0.0;
  }
  if (k == np - 1) tc[k] = 0.0;
}

void cons_path_coeffs(const double* geo, const int2* edges, const int* path_edge, const int* path_prev, int np,
                      double* ta, double* td, double* tc, hipStream_t s) {
  // tc[k-1] is written by row k; rows without a predecessor leave tc[k-1] to be zero
  hipMemsetAsync(tc, 0, sizeof(double) * np, s);
  hipLaunchKernelGGL(k_path_coeffs, dim3(cdiv(np, 256)), dim3(256), 0, s, geo, edges, path_edge, path_prev, np,
                     ta, td, tc);
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
// the projector P x = x - C^T (C C^T)^-1 C x in three launches (nb <= 8)
// ---------------------------------------------------------------------------
// With K = C C^T split into the path block Kpp (tridiagonal), the border
// block Kbb and their coupling Kpb, and Z = Kpp^-1 Kpb (columns), the Schur
// complement solve of K y = (wp, wb) is
//   yb = S^-1 (wb - Z^T wp),  yp = Kpp^-1 wp - Z yb,   S = Kbb - Kpb^T Z,
// using Kpb^T Kpp^-1 = Z^T (Kpp is symmetric).
//   1. k_proj_rows: wp = C_path x, and per-workgroup partial sums of the
//      border rows' dot products wb = rows . x and of Z^T wp;
//   2. k_proj_solve (one workgroup): the partial sums, yb, and Kpp^-1 wp;
//   3. k_apply_CT_z: out = x - C^T y with yp corrected by -Z yb per row.
// wp, yp and the factors of Kpp are chunk-transposed (tri_chunk_pos with
// m = ceil(np / kTriThreads)) so that the one-workgroup solve loads them
// coalesced; Z and everything else are in row order.
constexpr int kProjBlocks = 64, kProjSlots = 2 * kProjMaxBorder;
static_assert(kProjBlocks == 64 && kProjSlots == kTriWaves, "k_proj_solve reduces one slot per wave");

__global__ __launch_bounds__(256) void k_proj_rows(const double* __restrict__ geo, const int2* __restrict__ edges,
                                                   const int* __restrict__ path_edge, int np,
                                                   const double* __restrict__ rows, int nb,
                                                   const double* __restrict__ Z, int nV, const double* __restrict__ x,
                                                   double* __restrict__ wp, double* __restrict__ part) {
  double acc[kProjSlots];
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) acc[q] = 0.0;
  const int nmax = max(np, nV);
  const int m = (np + kTriThreads - 1) / kTriThreads;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nmax; i += gridDim.x * 256) {
    if (i < np) {
      const int I = path_edge[i];
      const int2 e = edges[I];
      const double* g = geo + 8 * (size_t)I;
      const double w = g[1] * (x[3 * e.x] - x[3 * e.y]) + g[2] * (x[3 * e.x + 1] - x[3 * e.y + 1]) +
                       g[3] * (x[3 * e.x + 2] - x[3 * e.y + 2]);
      wp[tri_chunk_pos(i, m)] = w;
#pragma unroll
      for (int r = 0; r < kProjMaxBorder; ++r)
        if (r < nb) acc[kProjMaxBorder + r] += Z[(size_t)r * np + i] * w;
    }
    if (i < nV) {
#pragma unroll
      for (int r = 0; r < kProjMaxBorder; ++r)
        if (r < nb) {
          const double* rv = rows + ((size_t)r * nV + i) * 3;
          acc[r] += rv[0] * x[3 * i] + rv[1] * x[3 * i + 1] + rv[2] * x[3 * i + 2];
        }
    }
  }
  __shared__ double sred[4][kProjSlots];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
  for (int q = 0; q < kProjSlots; ++q) {
    if ((q % kProjMaxBorder) >= nb) continue;  // unused slot (uniform)
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sred[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < kProjSlots) {
    const int q = threadIdx.x;
    part[(size_t)blockIdx.x * kProjSlots + q] =
        (q % kProjMaxBorder) < nb ? ((sred[0][q] + sred[1][q]) + sred[2][q]) + sred[3][q] : 0.0;
  }
}

__global__ __launch_bounds__(kTriThreads) void k_proj_solve(const double* __restrict__ part, int nblk, int nb,
                                                           const double* __restrict__ Sinv,
                                                           const double* __restrict__ lo,
                                                           const double* __restrict__ uinv,
                                                           const double* __restrict__ tc,
                                                           const double* __restrict__ wp, double* __restrict__ yp,
                                                           double* __restrict__ yb, int np) {
  __shared__ double wa[kTriWaves], wbs[kTriWaves];
  __shared__ double tot[kProjSlots];
  const int t = threadIdx.x, lane = t % 64;
  {  // wave q sums slot q over the workgroups of k_proj_rows
    const int q = t / 64;
    double v = (lane < nblk && (q % kProjMaxBorder) < nb) ? part[(size_t)lane * kProjSlots + q] : 0.0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) tot[q] = v;
  }
  __syncthreads();
  if (t < nb) {  // yb = S^-1 (wb - Z^T wp)
    double v = 0.0;
    for (int j = 0; j < nb; ++j) v += Sinv[t * nb + j] * (tot[j] - tot[kProjMaxBorder + j]);
    yb[t] = v;
  }
  if (np > 0) tridiag_solve_wg<true>(lo, uinv, tc, wp, yp, np, wa, wbs);
}

// out_v = in_v - [ sum_{path rows k at v} s(v) T_I (yp_k - (Z yb)_k) + sum_r yb[r] rows[r][v] ]
__global__ __launch_bounds__(256) void k_apply_CT_z(const double* __restrict__ geo, const int* __restrict__ inc_off,
                                                    const int* __restrict__ inc,
                                                    const int* __restrict__ edge_path_row,
                                                    const double* __restrict__ yp, const double* __restrict__ Z,
                                                    int np, const double* __restrict__ rows,
                                                    const double* __restrict__ yb, int nb, int nV,
                                                    const double* __restrict__ in, double* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  const int m = (np + kTriThreads - 1) / kTriThreads;
  double ybr[kProjMaxBorder];
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r) ybr[r] = r < nb ? yb[r] : 0.0;
  double acc[3] = {0, 0, 0};
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int I = inc[k] >> 1;
    const int pr = edge_path_row[I];
    if (pr < 0) continue;
    double y = yp[tri_chunk_pos(pr, m)];
#pragma unroll
    for (int r = 0; r < kProjMaxBorder; ++r)
      if (r < nb) y -= Z[(size_t)r * np + pr] * ybr[r];
    const double sg = (inc[k] & 1) ? -1.0 : 1.0;
    const double* g = geo + 8 * (size_t)I;
    for (int cc = 0; cc < 3; ++cc) acc[cc] += sg * g[1 + cc] * y;
  }
#pragma unroll
  for (int r = 0; r < kProjMaxBorder; ++r)
    if (r < nb)
      for (int cc = 0; cc < 3; ++cc) acc[cc] += ybr[r] * rows[((size_t)r * nV + v) * 3 + cc];
  for (int cc = 0; cc < 3; ++cc) out[3 * v + cc] = in[3 * v + cc] - acc[cc];
}

void cons_project_fused(const double* geo, const int2* edges, const int* path_edge, int np, const double* rows,
                        int nb, const double* Z, const double* Sinv, const double* lo_ch, const double* uinv_ch,
                        const double* tc_ch, const int* inc_off, const int* inc, const int* edge_path_row, int nV,
                        const double* in, double* out, double* part, double* wp_ch, double* yp_ch, double* yb,
                        hipStream_t s) {
  const int nblk = std::min(kProjBlocks, std::max(1, cdiv(std::max(np, nV), 256)));
  hipLaunchKernelGGL(k_proj_rows, dim3(nblk), dim3(256), 0, s, geo, edges, path_edge, np, rows, nb, Z, nV, in,
                     wp_ch, part);
  hipLaunchKernelGGL(k_proj_solve, dim3(1), dim3(kTriThreads), 0, s, (const double*)part, nblk, nb, Sinv, lo_ch,
                     uinv_ch, tc_ch, (const double*)wp_ch, yp_ch, yb, np);
  hipLaunchKernelGGL(k_apply_CT_z, dim3(cdiv(nV, 256)), dim3(256), 0, s, geo, inc_off, inc, edge_path_row,
                     (const double*)yp_ch, Z, np, rows, (const double*)yb, nb, nV, in, out);
}

// Copies of the factors l, 1/u and the coupling c of an n-row tridiagonal
// system in the chunk-transposed order of the one-workgroup solve.
__global__ void k_tri_chunk(const double* __restrict__ lo, const double* __restrict__ uinv,
                            const double* __restrict__ c, int n, double* __restrict__ lo_ch,
                            double* __restrict__ uinv_ch, double* __restrict__ c_ch) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int p = tri_chunk_pos(k, (n + kTriThreads - 1) / kTriThreads);
  lo_ch[p] = lo[k];
  uinv_ch[p] = uinv[k];
  c_ch[p] = c[k];
}

int tri_chunk_size(int n) { return n <= 0 ? 1 : cdiv(n, kTriThreads) * kTriThreads; }

void tridiag_chunk_copy(const double* lo, const double* uinv, const double* c, int n, double* lo_ch,
                        double* uinv_ch, double* c_ch, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tri_chunk, dim3(cdiv(n, 256)), dim3(256), 0, s, lo, uinv, c, n, lo_ch, uinv_ch, c_ch);
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

// Dense constraint matrix in the external row order (bary, total, edges) from
// the border rows and the edge rows: Cd[k][3 nV].
__global__ void k_dense_C_edges(const double* __restrict__ geo, const int2* __restrict__ edges, int nE, int row0,
                                int nV, double* __restrict__ Cd) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const double* g = geo + 8 * (size_t)I;
  int2 e = edges[I];
  double* r = Cd + (size_t)(row0 + I) * 3 * nV;
  for (int cc = 0; cc < 3; ++cc) {
    r[3 * e.x + cc] = g[1 + cc];
    r[3 * e.y + cc] = -g[1 + cc];
  }
}

void dense_C_edges(const double* geo, const int2* edges, int nE, int row0, int nV, double* Cd, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_C_edges, dim3(cdiv(nE, 256)), dim3(256), 0, s, geo, edges, nE, row0, nV, Cd);
}

}  // namespace rc
