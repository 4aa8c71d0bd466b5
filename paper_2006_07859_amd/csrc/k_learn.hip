// Learned smoother weights of the multigrid V-cycle: the MLP and the
// per-vertex features, the training targets and the regression loss.
//
// MLP (3 layers, width 64): y = softplus(W3 . relu(W2^T relu(W1^T x + b1) + b2) + b3)
// for every row x of 8 features.  Parameters are kept in FP32 (master copy,
// Adam state) and in FP16 (the weights the forward pass uses); biases stay
// FP32.  Forward: one wave per 16 rows, layers 1 and 2 on
// v_mfma_f32_16x16x32_f16 (FP16 operands, FP32 accumulation; layer 1's 8
// inputs padded to the MFMA depth of 32), layer 3 a wave-reduced dot product.
// The forward keeps, for the backward pass, the FP16-rounded first hidden
// layer (the values layer 2 consumed), the second hidden layer and the
// pre-activation output.  Backward in FP32: a thread per row for the
// per-row deltas, then deterministic chunked sums of outer products for the
// weight gradients.  Flat parameter order: W1 [8][64], b1, W2 [64][64], b2,
// W3 [64], b3.
//
// The network predicts p_v = 1 + y_v, a diagonal scaling of the level's
// operator A_l: the target T_v = r_v lambda_l with r_v = sum_w |A_vw| / A_vv
// (the row's l1 norm over its diagonal, >= 2 since A annihilates constants)
// and lambda_l the largest eigenvalue of D_r^-1 A_l, D_r = diag(r_v A_vv)
// (<= 1 by Gershgorin).  With D = diag(T_v A_vv) the spectrum of D^-1 A_l
// tops out at exactly 1, so the smoother's Chebyshev interval is fixed at
// [frac, 1] with no spectral estimate.
//
// Features of vertex v on a level of n vertices (a closed loop numbered
// along itself): log2(n) / 16; log of the mean incident edge length over the
// level's mean edge length; turning angle between the incoming and outgoing
// edge; unit vertex tangent (3); log of diag(A_l)_v over its level mean; log
// of the incoming over the outgoing edge length.

#include <algorithm>
#include <cmath>
#include <vector>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = kMlpIn, kW = kMlpWidth;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kW, oW2 = oB1 + kW, oB2 = oW2 + kW * kW, oW3 = oB2 + kW, oB3 = oW3 + kW;

__device__ __forceinline__ float softplusf(float o) { return o > 20.f ? o : log1pf(expf(o)); }
__device__ __forceinline__ float logisticf(float o) { return 1.f / (1.f + expf(-o)); }

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// Y[r] = y(X[r]); when cache != null also H1 (FP16-rounded, [N][64]),
// H2 ([N][64]) and O ([N]) for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* __restrict__ X, int N, const _Float16* __restrict__ w16,
                                                 const float* __restrict__ theta, float* __restrict__ Y,
                                                 float* __restrict__ H1, float* __restrict__ H2,
                                                 float* __restrict__ O) {
  __shared__ _Float16 sW1[32][kW];        // rows >= 8 are zero
  __shared__ _Float16 sW2[kW][kW];
  __shared__ float sB1[kW], sB2[kW], sW3[kW];
  __shared__ _Float16 sH[4][16][kW + 8];  // per wave: the first hidden layer of its 16 rows
  const int tid = threadIdx.x;
  for (int e = tid; e < 32 * kW; e += 256) {
    const int k = e / kW, n = e % kW;
    sW1[k][n] = k < kIn ? w16[oW1 + k * kW + n] : (_Float16)0.f;
  }
  for (int e = tid; e < kW * kW; e += 256) sW2[e / kW][e % kW] = w16[oW2 + e];
  if (tid < kW) {
    sB1[tid] = theta[oB1 + tid];
    sB2[tid] = theta[oB2 + tid];
    sW3[tid] = (float)w16[oW3 + tid];
  }
  __syncthreads();
  const int wave = tid / 64, l = tid % 64;
  const int r0 = (blockIdx.x * 4 + wave) * 16;
  const int g = l / 16, cl = l % 16;
  // layer 1: A = X rows (k 0..7 in lane group 0), B = W1
  f16x8 a;
  {
    const int row = r0 + cl;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (g == 0 && row < N) ? (_Float16)X[(size_t)row * kIn + j] : (_Float16)0.f;
  }
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f16x8 b;
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = sW1[8 * g + j][16 * t + cl];
    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
  }
  // h1 = relu(a1 + b1): lane holds rows 4 g + j of column 16 t + cl
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = 16 * t + cl, rloc = 4 * g + j;
      const _Float16 h = (_Float16)fmaxf(acc[t][j] + sB1[col], 0.f);
      sH[wave][rloc][col] = h;
      if (H1 && r0 + rloc < N) H1[(size_t)(r0 + rloc) * kW + col] = (float)h;
    }
  __syncthreads();
  // layer 2: A = h1 (two depth-32 steps), B = W2
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    f16x8 a2;
#pragma unroll
    for (int j = 0; j < 8; ++j) a2[j] = sH[wave][cl][32 * ks + 8 * g + j];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f16x8 b;
#pragma unroll
      for (int j = 0; j < 8; ++j) b[j] = sW2[32 * ks + 8 * g + j][16 * t + cl];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, b, acc[t], 0, 0, 0);
    }
  }
  // h2 = relu(a2 + b2); layer 3 per row
  float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = 16 * t + cl, rloc = 4 * g + j;
      const float h = fmaxf(acc[t][j] + sB2[col], 0.f);
      if (H2 && r0 + rloc < N) H2[(size_t)(r0 + rloc) * kW + col] = h;
      part[j] += h * sW3[col];
    }
#pragma unroll
  for (int j = 0; j < 4; ++j)
    for (int o = 8; o > 0; o >>= 1) part[j] += __shfl_xor(part[j], o, 16);
  if (cl == 0) {
    const float b3 = theta[oB3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = r0 + 4 * g + j;
      if (row < N) {
        const float o = part[j] + b3;
        Y[row] = softplusf(o);
        if (O) O[row] = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// Per row: do = dy logistic(o); D2 = do W3 (h2 > 0); D1 = (D2 W2^T) (h1 > 0).
__global__ __launch_bounds__(256) void k_mlp_bwd_rows(int N, const float* __restrict__ dY,
                                                      const _Float16* __restrict__ w16, const float* __restrict__ H1,
                                                      const float* __restrict__ H2, const float* __restrict__ O,
                                                      float* __restrict__ Do, float* __restrict__ D1,
                                                      float* __restrict__ D2) {
  __shared__ float sW2[kW][kW + 1];
  __shared__ float sW3[kW];
  for (int e = threadIdx.x; e < kW * kW; e += 256) sW2[e / kW][e % kW] = (float)w16[oW2 + e];
  if (threadIdx.x < kW) sW3[threadIdx.x] = (float)w16[oW3 + threadIdx.x];
  __syncthreads();
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= N) return;
  const float d_o = dY[r] * logisticf(O[r]);
  Do[r] = d_o;
  float d2[kW];
#pragma unroll
  for (int n = 0; n < kW; ++n) {
    d2[n] = H2[(size_t)r * kW + n] > 0.f ? d_o * sW3[n] : 0.f;
    D2[(size_t)r * kW + n] = d2[n];
  }
  for (int i = 0; i < kW; ++i) {
    float s = 0.f;
#pragma unroll
    for (int n = 0; n < kW; ++n) s += d2[n] * sW2[i][n];
    D1[(size_t)r * kW + i] = H1[(size_t)r * kW + i] > 0.f ? s : 0.f;
  }
}

// part[chunk][i][j] = sum over the chunk's rows of A[r][i] B[r][j]
// (A = null: a column of ones, for the bias gradients).
__global__ __launch_bounds__(256) void k_outer_partial(const float* __restrict__ A, int lda, int P,
                                                       const float* __restrict__ B, int ldb, int Q, int N, int rows,
                                                       float* __restrict__ part) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= P * Q) return;
  const int i = e / Q, j = e % Q;
  const int r0 = blockIdx.y * rows, r1 = min(N, r0 + rows);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += (A ? A[(size_t)r * lda + i] : 1.f) * B[(size_t)r * ldb + j];
  part[(size_t)blockIdx.y * P * Q + e] = s;
}

__global__ void k_outer_reduce(const float* __restrict__ part, int PQ, int nchunk, float* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= PQ) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * PQ + e];
  out[e] = s;
}

// Adam (Kingma and Ba, Algorithm 1) on the FP32 master copy; refreshes the
// FP16 weights.
__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, _Float16* __restrict__ w16, int n, float lr, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float g = grad[k];
  const float mk = 0.9f * m[k] + 0.1f * g;
  const float vk = 0.999f * v[k] + 0.001f * g * g;
  m[k] = mk;
  v[k] = vk;
  const float t = theta[k] - lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
  theta[k] = t;
  w16[k] = (_Float16)t;
}

__global__ void k_to_f16(const float* __restrict__ theta, _Float16* __restrict__ w16, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) w16[k] = (_Float16)theta[k];
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
// Per vertex of one level: mean incident edge length, turning angle, unit
// tangent and log(diag); per-level means are taken by k_level_means.
// Vertex v's incoming edge ends at v, its outgoing edge starts at v.
__global__ void k_feat_local(const double* __restrict__ gam, const int2* __restrict__ edges,
                             const int* __restrict__ inc_off, const int* __restrict__ inc, int n,
                             const double* __restrict__ diag, double* __restrict__ lbar, double* __restrict__ loc) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double tin[3] = {0, 0, 0}, tout[3] = {0, 0, 0}, lin = 0, lout = 0;
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int2 e = edges[inc[k] >> 1];
    const double d[3] = {gam[3 * e.y] - gam[3 * e.x], gam[3 * e.y + 1] - gam[3 * e.x + 1],
                         gam[3 * e.y + 2] - gam[3 * e.x + 2]};
    const double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (inc[k] & 1) {  // v = second endpoint: incoming
      lin = l;
      for (int c = 0; c < 3; ++c) tin[c] = d[c] / l;
    } else {
      lout = l;
      for (int c = 0; c < 3; ++c) tout[c] = d[c] / l;
    }
  }
  lbar[v] = 0.5 * (lin + lout);
  const double dotp = tin[0] * tout[0] + tin[1] * tout[1] + tin[2] * tout[2];
  double t[3] = {tin[0] + tout[0], tin[1] + tout[1], tin[2] + tout[2]};
  const double tn = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  double* o = loc + 8 * (size_t)v;
  o[0] = acos(fmin(1.0, fmax(-1.0, dotp)));
  for (int c = 0; c < 3; ++c) o[1 + c] = t[c] / tn;
  o[4] = log(diag[v]);
  o[5] = lout;  // the outgoing edge's length: their mean is the level's mean edge length
  o[6] = lin;
}

// sums[0] = mean edge length (each edge is one vertex's outgoing edge),
// sums[1] = mean of diag (one workgroup).
__global__ __launch_bounds__(256) void k_level_means(const double* __restrict__ loc, const double* __restrict__ diag,
                                                     int n, double* __restrict__ sums) {
  __shared__ double s0[256], s1[256];
  double a = 0, b = 0;
  for (int v = threadIdx.x; v < n; v += 256) {
    a += loc[8 * (size_t)v + 5];
    b += diag[v];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sums[0] = s0[0] / n;
    sums[1] = s1[0] / n;
  }
}

// X rows of one level (float [n][8]) from the pieces above.
__global__ void k_feat_rows(const double* __restrict__ loc, const double* __restrict__ lbar,
                            const double* __restrict__ sums, int n, float* __restrict__ X) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double* o = loc + 8 * (size_t)v;
  float* x = X + (size_t)v * kIn;
  x[0] = (float)(log2((double)n) / 16.0);
  x[1] = (float)log(lbar[v] / sums[0]);
  x[2] = (float)o[0];
  x[3] = (float)o[1];
  x[4] = (float)o[2];
  x[5] = (float)o[3];
  x[6] = (float)(o[4] - log(sums[1]));
  x[7] = (float)log(o[6] / o[5]);
}

// ---------------------------------------------------------------------------
// training targets and loss
// ---------------------------------------------------------------------------
// r_v = sum_w |A_vw| / A_vv for the rows of a dense FP64 matrix and the
// scaling sc_v = (r_v A_vv)^-1/2 (one wave per row, fixed-order lane sums
// then a wave reduction).
__global__ __launch_bounds__(256) void k_row_l1_ratio(const double* __restrict__ A, int n, double* __restrict__ r,
                                                      double* __restrict__ sc) {
  const int v = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (v >= n) return;
  const double* row = A + (size_t)v * n;
  double a = 0.0;
  for (int w = lane; w < n; w += 64) a += fabs(row[w]);
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) {
    r[v] = a / row[v];
    sc[v] = 1.0 / sqrt(a);
  }
}

// y = S x with S = diag(sc) A diag(sc) for a dense symmetric A (one wave per row).
__global__ __launch_bounds__(256) void k_sym_scaled_mv(const double* __restrict__ A, const double* __restrict__ sc,
                                                       const double* __restrict__ x, int n, double* __restrict__ y) {
  const int v = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (v >= n) return;
  const double* row = A + (size_t)v * n;
  double a = 0.0;
  for (int w = lane; w < n; w += 64) a += row[w] * sc[w] * x[w];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) y[v] = sc[v] * a;
}

// x_v = (-1)^v: the alternating vector, close to the top eigenvector of the
// scaled operator of a loop (its highest frequency)
__global__ void k_alternating(int n, double* __restrict__ x) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) x[v] = (v & 1) ? -1.0 : 1.0;
}

// T_v = r_v lambda (float)
__global__ void k_ratio_targets(const double* __restrict__ r, const double* __restrict__ lam, int n,
                                float* __restrict__ T) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) T[v] = (float)(r[v] * lam[0]);
}

// Regression of p = 1 + y on the ratio r in log space, under-prediction
// (p < r, where the Gershgorin bound of the smoother fails) weighted by
// kFitUnder: per row loss w (log p - log r)^2, dY = d(mean loss)/dy; the
// loss summed per workgroup into part.
constexpr float kFitUnder = 4.f;
__global__ __launch_bounds__(256) void k_fit_loss(const float* __restrict__ Y, const float* __restrict__ R, int N,
                                                  float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double sm[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (i < N) {
    const float p = 1.f + Y[i];
    const float e = logf(p) - logf(R[i]);
    const float w = p < R[i] ? kFitUnder : 1.f;
    l = (double)(w * e * e);
    dY[i] = 2.f * w * e / (p * (float)N);
  }
  sm[threadIdx.x] = l;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < n; ++k) a += part[k];
    out[0] = a * scale;
  }
}

// The smoother's diagonal D_v = margin (1 + y_v) diag_v (its weights are 1 / D_v).
__global__ void k_learned_diag(const float* __restrict__ Y, int n, double margin, double* __restrict__ diag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) diag[v] *= margin * (1.0 + (double)Y[v]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
rc_status Mlp::ensure_rows(int N) {
  if (N <= cap) return RC_OK;
  float** bufs[] = {&H1, &H2, &O, &Do, &D1, &D2, &Y, &dY};
  for (float** b : bufs)
    if (*b) hipFree(*b);
  const int c = std::max(N, 1024);
  size_t sizes[] = {(size_t)c * kW, (size_t)c * kW, (size_t)c, (size_t)c, (size_t)c * kW, (size_t)c * kW, (size_t)c,
                    (size_t)c};
  for (int k = 0; k < 8; ++k)
    if (hipMalloc((void**)bufs[k], sizeof(float) * sizes[k]) != hipSuccess) {
      set_error("MLP scratch allocation failed");
      return RC_ERR_NOMEM;
    }
  cap = c;
  return RC_OK;
}

rc_status Mlp::init(const float* theta_h, hipStream_t s) {
  stream = s;
  const size_t np = kMlpParams;
  if (hipMalloc((void**)&theta, sizeof(float) * np) != hipSuccess ||
      hipMalloc((void**)&m, sizeof(float) * np) != hipSuccess ||
      hipMalloc((void**)&v, sizeof(float) * np) != hipSuccess ||
      hipMalloc((void**)&grad, sizeof(float) * np) != hipSuccess ||
      hipMalloc((void**)&w16, sizeof(_Float16) * np) != hipSuccess ||
      hipMalloc((void**)&opart, sizeof(float) * 64 * kW * kW) != hipSuccess) {
    set_error("MLP allocation failed");
    return RC_ERR_NOMEM;
  }
  return set(theta_h);
}

rc_status Mlp::set(const float* theta_h) {
  const size_t np = kMlpParams;
  std::vector<float> zero(np, 0.f);
  RC_HIP(hipMemcpy(theta, theta_h ? theta_h : zero.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(m, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(v, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_to_f16, dim3(cdiv((int)np, 256)), dim3(256), 0, stream, theta, w16, (int)np);
  RC_HIP(hipGetLastError());
  RC_HIP(hipStreamSynchronize(stream));
  t = 0;
  return RC_OK;
}

void Mlp::release() {
  void* ps[] = {theta, m, v, grad, w16, opart, H1, H2, O, Do, D1, D2, Y, dY};
  for (void* p : ps)
    if (p) hipFree(p);
  theta = m = v = grad = opart = H1 = H2 = O = Do = D1 = D2 = Y = dY = nullptr;
  w16 = nullptr;
  cap = 0;
}

rc_status mlp_forward(Mlp& M, const float* X, int N, float* Y, bool keep, hipStream_t s) {
  if (keep) RC_TRY(M.ensure_rows(N));
  if (N <= 0) return RC_OK;
  if (!X || !Y) {
    set_error("MLP forward: null input or output");
    return RC_ERR_ARG;
  }
  hipLaunchKernelGGL(k_mlp_fwd, dim3(cdiv(N, 64)), dim3(256), 0, s, X, N, (const _Float16*)M.w16,
                     (const float*)M.theta, Y, keep ? M.H1 : nullptr, keep ? M.H2 : nullptr, keep ? M.O : nullptr);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// grad = d(sum dY . y)/dtheta for the rows of the last forward with keep.
rc_status mlp_backward(Mlp& M, const float* X, int N, const float* dY, float* grad, hipStream_t s) {
  if (N <= 0 || N > M.cap) {
    set_error("MLP backward: no kept forward pass of that many rows");
    return RC_ERR_ARG;
  }
  hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(cdiv(N, 256)), dim3(256), 0, s, N, dY, (const _Float16*)M.w16,
                     (const float*)M.H1, (const float*)M.H2, (const float*)M.O, M.Do, M.D1, M.D2);
  // weight and bias gradients: sums of outer products over the rows, 64 chunks
  const int nchunk = std::min(64, std::max(1, cdiv(N, 64)));
  const int rows = cdiv(N, nchunk);
  struct Job {
    const float* A;
    int lda, P;
    const float* B;
    int ldb, Q, off;
  };
  const Job jobs[] = {{X, kIn, kIn, M.D1, kW, kW, oW1},   {nullptr, 0, 1, M.D1, kW, kW, oB1},
                      {M.H1, kW, kW, M.D2, kW, kW, oW2},  {nullptr, 0, 1, M.D2, kW, kW, oB2},
                      {M.H2, kW, kW, M.Do, 1, 1, oW3},    {nullptr, 0, 1, M.Do, 1, 1, oB3}};
  for (const Job& j : jobs) {
    const int PQ = j.P * j.Q;
    hipLaunchKernelGGL(k_outer_partial, dim3(cdiv(PQ, 256), nchunk), dim3(256), 0, s, j.A, j.lda, j.P, j.B, j.ldb,
                       j.Q, N, rows, M.opart);
    hipLaunchKernelGGL(k_outer_reduce, dim3(cdiv(PQ, 256)), dim3(256), 0, s, (const float*)M.opart, PQ, nchunk,
                       grad + j.off);
  }
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status mlp_adam(Mlp& M, const float* grad, float lr, hipStream_t s) {
  M.t += 1;
  const float c1 = 1.f - powf(0.9f, (float)M.t), c2 = 1.f - powf(0.999f, (float)M.t);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(kMlpParams, 256)), dim3(256), 0, s, M.theta, grad, M.m, M.v, M.w16,
                     kMlpParams, lr, c1, c2);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// Features of one level into X (float [n][8]); scratch: 9 n + 2 doubles.
rc_status launch_level_features(const Curve& cv, const double* gam, const double* diag, double* scratch, float* X,
                                hipStream_t s) {
  const int n = cv.nV;
  double* lbar = scratch;
  double* loc = scratch + (size_t)n;
  double* sums = scratch + 9 * (size_t)n;
  hipLaunchKernelGGL(k_feat_local, dim3(cdiv(n, 256)), dim3(256), 0, s, gam, cv.edges, cv.inc_off, cv.inc, n, diag,
                     lbar, loc);
  hipLaunchKernelGGL(k_level_means, dim3(1), dim3(256), 0, s, (const double*)loc, diag, n, sums);
  hipLaunchKernelGGL(k_feat_rows, dim3(cdiv(n, 256)), dim3(256), 0, s, (const double*)loc, (const double*)lbar,
                     (const double*)sums, n, X);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_row_l1_ratio(const double* A, int n, double* r, double* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_row_l1_ratio, dim3(cdiv(n, 4)), dim3(256), 0, s, A, n, r, sc);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_sym_scaled_mv(const double* A, const double* sc, const double* x, int n, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_sym_scaled_mv, dim3(cdiv(n, 4)), dim3(256), 0, s, A, sc, x, n, y);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_alternating(int n, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_alternating, dim3(cdiv(n, 256)), dim3(256), 0, s, n, x);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_ratio_targets(const double* r, const double* lam, int n, float* T, hipStream_t s) {
  hipLaunchKernelGGL(k_ratio_targets, dim3(cdiv(n, 256)), dim3(256), 0, s, r, lam, n, T);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_learned_diag(const float* Y, int n, double margin, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_learned_diag, dim3(cdiv(n, 256)), dim3(256), 0, s, Y, n, margin, diag);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// One regression step: forward (kept), loss and dY, backward, Adam (lr > 0).
rc_status mlp_fit_step(Mlp& M, const float* X, const float* R, int N, float lr, double* loss_dev, float* grad_out,
                       hipStream_t s) {
  if (N <= 0) {
    set_error("MLP fit: N must be positive");
    return RC_ERR_ARG;
  }
  RC_TRY(M.ensure_rows(N));  // the row buffers (M.Y among them) exist before they are passed on
  RC_TRY(mlp_forward(M, X, N, M.Y, true, s));
  const int nb = cdiv(N, 256);
  if (nb > M.cap) {
    set_error("MLP fit: too many rows for the loss buffer");
    return RC_ERR_ARG;
  }
  double* part = (double*)M.D1;  // [nb] doubles: the first-layer deltas are written after the loss
  hipLaunchKernelGGL(k_fit_loss, dim3(nb), dim3(256), 0, s, (const float*)M.Y, R, N, M.dY, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (const double*)part, nb, 1.0 / N, loss_dev);
  RC_TRY(mlp_backward(M, X, N, M.dY, M.grad, s));
  if (grad_out) RC_HIP(hipMemcpyAsync(grad_out, M.grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, s));
  if (lr > 0.f) RC_TRY(mlp_adam(M, M.grad, lr, s));
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
