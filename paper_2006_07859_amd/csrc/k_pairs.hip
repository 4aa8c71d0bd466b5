// Pair kernels of the tangent-point hot path on gfx950.
//
// Every kernel here is a gather over ordered edge pairs (I, J): a thread owns
// one target edge I, the block's 256 targets sweep a range of source edges J
// that is staged through LDS in tiles of 256, and each thread accumulates its
// target's sums in registers.  Sources are split into `nchunk` ranges along
// blockIdx.y so that a launch has thousands of workgroups; per-chunk partial
// sums land in a [chunk][slot][edge] buffer that a finalize kernel reduces in
// FP64, in a fixed order (no atomics, bitwise reproducible).
//
// In FP32 the per-thread sums are kept in float over 64 sources at a time and
// then folded into FP64 accumulators, so the long sums over all sources are
// compensated blockwise.
//
// Edge pairs that share a vertex (I = J included) are omitted, as the
// discrete energy (Sec. 4.1, eq. DiscreteEnergy) and the Gram matrices
// (Sec. 4.2) prescribe.  Such a pair gets weight 0 and its coincident vertex
// pairs get a stand-in distance of 1, so no Inf or NaN is formed.

#include <type_traits>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

ExpCase exp_case(double alpha, double beta) {
  if (alpha == 2.0 && beta == 4.0) return kA2B4;
  if (alpha == 2.0 && beta == 4.5) return kA2B45;
  if (alpha == 3.0 && beta == 6.0) return kA3B6;
  return kGeneral;
}

// ---------------------------------------------------------------------------
// edge geometry: FP64 state -> rounded SoA in the kernel precision
// ---------------------------------------------------------------------------
// a_I = (g_i1, l_I), b_I = (g_i2, 0), T_I = (e_I / l_I, 0) in FP64 and, when
// Af is set, the same values rounded to FP32 (the FP32 pair kernels' copy).
// When P is set (the vertex-pair form) thread v also writes the vertex
// geometry (g_v, Lambda_v), u_0, u_1 (sqrt(l_I) T_I of v's first two incident
// edges in incidence order) in FP32 (P, U0, U1) and FP64 (Pd, U0d, U1d), its
// incident edges recomputed from gamma in the same arithmetic.  A non-finite coordinate and a zero-length edge (l_I = 0:
// T_I is undefined, Sec. 4 Notation) are latched.
__device__ __forceinline__ double edge_vector(const double* __restrict__ gamma, int2 e, double (&p)[3],
                                              double (&q)[3], double (&d)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    p[k] = gamma[3 * e.x + k];
    q[k] = gamma[3 * e.y + k];
    d[k] = q[k] - p[k];
  }
  return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

__global__ void k_geometry(const double* __restrict__ gamma, const int2* __restrict__ edges, int nE,
                           V4<double>* __restrict__ A, V4<double>* __restrict__ B, V4<double>* __restrict__ T,
                           V4<float>* __restrict__ Af, V4<float>* __restrict__ Bf, V4<float>* __restrict__ Tf,
                           const int* __restrict__ inc_off, const int* __restrict__ inc, int nV,
                           V4<float>* __restrict__ P, V4<float>* __restrict__ U0, V4<float>* __restrict__ U1,
                           V4<double>* __restrict__ Pd, V4<double>* __restrict__ U0d,
                           V4<double>* __restrict__ U1d, unsigned* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nE) {
    double p[3], q[3], d[3];
    const double l = edge_vector(gamma, edges[i], p, q, d);
    const bool fin = isfinite(p[0]) & isfinite(p[1]) & isfinite(p[2]) & isfinite(q[0]) & isfinite(q[1]) &
                     isfinite(q[2]);
    if (!fin) latch(status, kFlagInputNonfinite);
    else if (!(l > 0.0)) latch(status, kFlagZeroEdge);
    const double il = 1.0 / l;
    const double t0 = d[0] * il, t1 = d[1] * il, t2 = d[2] * il;
    A[i] = V4<double>{p[0], p[1], p[2], l};
    B[i] = V4<double>{q[0], q[1], q[2], 0.0};
    T[i] = V4<double>{t0, t1, t2, 0.0};
    if (Af) {
      Af[i] = V4<float>{(float)p[0], (float)p[1], (float)p[2], (float)l};
      Bf[i] = V4<float>{(float)q[0], (float)q[1], (float)q[2], 0.f};
      Tf[i] = V4<float>{(float)t0, (float)t1, (float)t2, 0.f};
    }
  }
  if (P && i < nV) {
    double lam = 0.0, u[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    const int k0 = inc_off[i], k1 = min(inc_off[i + 1], k0 + 2);
    for (int k = k0; k < k1; ++k) {
      double p[3], q[3], d[3];
      const double l = edge_vector(gamma, edges[inc[k] >> 1], p, q, d);
      const double il = 1.0 / l, sl = sqrt(l);
      lam += l;
#pragma unroll
      for (int c = 0; c < 3; ++c) u[k - k0][c] = sl * (d[c] * il);
    }
    const double x0 = gamma[3 * i], x1 = gamma[3 * i + 1], x2 = gamma[3 * i + 2];
    P[i] = V4<float>{(float)x0, (float)x1, (float)x2, (float)lam};
    U0[i] = V4<float>{(float)u[0][0], (float)u[0][1], (float)u[0][2], 0.f};
    U1[i] = V4<float>{(float)u[1][0], (float)u[1][1], (float)u[1][2], 0.f};
    Pd[i] = V4<double>{x0, x1, x2, lam};
    U0d[i] = V4<double>{u[0][0], u[0][1], u[0][2], 0.0};
    U1d[i] = V4<double>{u[1][0], u[1][1], u[1][2], 0.0};
  }
}

// Chain-near test: edges of the same chain at most kBand apart (cyclically on loops).
__device__ __forceinline__ bool chain_near(int4 ci, int4 cj) {
  int dd = abs(cj.y - ci.y);
  dd = ci.w ? min(dd, ci.z - dd) : dd;
  return (cj.x == ci.x) & (dd <= kBand);
}

// BAND: the graph is a union of chains and the kernel runs in FP32; pairs
// that are chain-near (which include every pair sharing a vertex) are left
// to the FP64 near-band kernel.  Otherwise only pairs sharing a vertex are
// skipped.
//
// The body works on one tile: targets I0 .. I0 + tcount - 1 (tcount <= kTile)
// against sources s0 .. s1 - 1, writing partial-sum chunk `chunk`.  It is
// called by the grid kernel (tile = blockIdx.x, chunk = blockIdx.y) and by
// the persistent work-queue kernel of a batch (tiles and source ranges kept
// inside one instance).
template <typename R, int EC, bool GRAD, bool BAND>
__device__ __forceinline__ void tpe_tile(const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB,
                                         const V4<R>* __restrict__ GT, const int2* __restrict__ edges,
                                         const int4* __restrict__ cinfo, int nE, int I0, int tcount, int s0, int s1,
                                         int chunk, R half_alpha, R half_beta, R beta, double* __restrict__ part) {
  __shared__ V4<R> sA[kTile], sB[kTile], sT[kTile];
  __shared__ int2 sE[kTile];
  __shared__ int4 sC[BAND ? kTile : 1];
  __shared__ int4 sRed[2][kTile / 64];  // chain ranges: [0] targets, [1] the staged sources
  __shared__ int2 sChain;               // (length, is loop) of the first target's chain
  const int tid = threadIdx.x;
  const int I = I0 + tid;
  const bool act = tid < tcount;
  const int Ic = act ? I : I0;
  const V4<R> a = GA[Ic], b = GB[Ic], t = GT[Ic];
  const int2 ei = act ? edges[Ic] : make_int2(-1, -2);
  int4 ci = make_int4(-1, 0, 0, 0);
  if constexpr (BAND) {
    ci = act ? cinfo[Ic] : make_int4(-1, 0, 0, 0);
    wave_range(ci, act, sRed[0]);
    if (tid == 0) sChain = make_int2(ci.z, ci.w);  // thread 0 always holds a target
  }
  constexpr int NS = GRAD ? kTpeSlots : 1;
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;

  for (int t0 = s0; t0 < s1; t0 += kTile) {
    __syncthreads();
    if (t0 + tid < s1) {
      const V4<R> qa = GA[t0 + tid];
      V4<R> qb = GB[t0 + tid];
      qb.w = R(0.25) * qa.w;
      sA[tid] = qa;
      sB[tid] = qb;
      sT[tid] = GT[t0 + tid];
      sE[tid] = edges[t0 + tid];
    }
    if constexpr (BAND) {
      const bool staged = t0 + tid < s1;
      const int4 cj = staged ? cinfo[t0 + tid] : make_int4(-1, 0, 0, 0);
      if (staged) sC[tid] = cj;
      wave_range(cj, staged, sRed[1]);
    }
    __syncthreads();
    const int cnt = min(kTile, s1 - t0);
    // Pairs are tested (and skipped) one by one only where the tile ranges
    // cannot rule out a chain-near or vertex-sharing pair.
    bool test = true;
    if constexpr (BAND) test = !tiles_far(range_of(sRed[0]), range_of(sRed[1]), sChain.x, sChain.y);
    for (int u0 = 0; u0 < cnt; u0 += kSub) {
      const int u1 = min(cnt, u0 + kSub);
      R E = 0, S = 0, G1x = 0, G1y = 0, G1z = 0, G2x = 0, G2y = 0, G2z = 0;
      R Gt1 = 0, Gt2 = 0, Hx = 0, Hy = 0, Hz = 0;
      auto sweep = [&](auto tested) {
        for (int u = u0; u < u1; ++u) {
          const V4<R> qa = sA[u], qb = sB[u], qt = sT[u];
          if constexpr (decltype(tested)::value) {
            bool skip;
            if constexpr (BAND) {
              skip = chain_near(ci, sC[u]);
            } else {
              const int2 ej = sE[u];
              skip = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
            }
            const R w = skip ? R(0) : qb.w;  // l_J / 4, staged in the free slot
            tpe_edge_pair<R, EC, GRAD, true>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y, qt.z,
                                             qa.w, w, skip ? R(1) : R(0), half_alpha, half_beta, beta, E, S, G1x,
                                             G1y, G1z, Gt1, G2x, G2y, G2z, Gt2, Hx, Hy, Hz);
          } else {
            tpe_edge_pair<R, EC, GRAD, false>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y,
                                              qt.z, qa.w, qb.w, R(0), half_alpha, half_beta, beta, E, S, G1x, G1y,
                                              G1z, Gt1, G2x, G2y, G2z, Gt2, Hx, Hy, Hz);
          }
        }
      };
      if (test) sweep(std::true_type{});
      else sweep(std::false_type{});
      acc[0] += (double)E;
      if constexpr (GRAD) {
        acc[1] += (double)S;
        acc[2] += (double)G1x; acc[3] += (double)G1y; acc[4] += (double)G1z;
        acc[5] += (double)G2x; acc[6] += (double)G2y; acc[7] += (double)G2z;
        acc[8] += (double)Gt1; acc[9] += (double)Gt2;
        acc[10] += (double)Hx; acc[11] += (double)Hy; acc[12] += (double)Hz;
        acc[13] += (double)(t.x * Hx + t.y * Hy + t.z * Hz);  // T.H: H holds multiples of T
      }
    }
  }
  if (act) {
    double* out = part + (size_t)chunk * NS * nE + I;
#pragma unroll
    for (int k = 0; k < NS; ++k) out[(size_t)k * nE] = acc[k];
  }
}

template <typename R, int EC, bool GRAD, bool BAND>
__global__ __launch_bounds__(kTile) void k_tpe_pairs(
    const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB, const V4<R>* __restrict__ GT,
    const int2* __restrict__ edges, const int4* __restrict__ cinfo, int nE, int src_per_chunk, R half_alpha,
    R half_beta, R beta, double* __restrict__ part) {
  const int I0 = blockIdx.x * kTile;
  const int s0 = blockIdx.y * src_per_chunk;
  tpe_tile<R, EC, GRAD, BAND>(GA, GB, GT, edges, cinfo, nE, I0, min(kTile, nE - I0), s0,
                              min(nE, s0 + src_per_chunk), blockIdx.y, half_alpha, half_beta, beta, part);
}

// Persistent work queue: items (t0, s0, s1, chunk << 16 | tcount), longest
// first; every workgroup takes the next item from an atomic counter (zeroed
// by k_zero_counter before the launch) until the list is exhausted.
__device__ __forceinline__ int next_item(int* counter) {
  __shared__ int it;
  __syncthreads();
  if (threadIdx.x == 0) it = atomicAdd(counter, 1);
  __syncthreads();
  return it;
}

__global__ void k_zero_counter(int* counter) { counter[0] = 0; }

template <typename R, int EC, bool GRAD, bool BAND>
__global__ __launch_bounds__(kTile) void k_tpe_items(
    const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB, const V4<R>* __restrict__ GT,
    const int2* __restrict__ edges, const int4* __restrict__ cinfo, int nE, const int4* __restrict__ items,
    int n_items, int* __restrict__ counter, const int* __restrict__ inst_of_edge, const int* __restrict__ mask,
    R half_alpha, R half_beta, R beta, double* __restrict__ part) {
  for (int it = next_item(counter); it < n_items; it = next_item(counter)) {
    const int4 w = items[it];
    if (mask && !mask[inst_of_edge[w.x]]) continue;  // instance switched off: its partials are not needed
    tpe_tile<R, EC, GRAD, BAND>(GA, GB, GT, edges, cinfo, nE, w.x, w.w & 0xffff, w.y, w.z, w.w >> 16, half_alpha,
                                half_beta, beta, part);
  }
}

// FP64 near band: for target I, every source J of the same chain at most
// kBand apart (the pairs the BAND pair kernel skips), with the exact
// shared-vertex exclusion.  Four lanes share a target's band (lane j takes the
// positions q0 + j, q0 + j + 4, ...) and their sums are added across the lanes
// in a fixed order.  Writes the partial-sum chunk `chunk`.
template <int EC, bool GRAD>
__global__ __launch_bounds__(256) void k_tpe_band(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                                                  const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                                                  const int4* __restrict__ cinfo, const int* __restrict__ chain_edge,
                                                  int nE, double half_alpha, double half_beta, double beta, int chunk,
                                                  const int* __restrict__ inst_of_edge, const int* __restrict__ mask,
                                                  double* __restrict__ part) {
  const int tg = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = tg / 4, sub = tg % 4;
  bool valid = I < nE;
  if (valid && mask) valid = mask[inst_of_edge[I]] != 0;
  double E = 0, S = 0, G1x = 0, G1y = 0, G1z = 0, G2x = 0, G2y = 0, G2z = 0;
  double Gt1 = 0, Gt2 = 0, Hx = 0, Hy = 0, Hz = 0;
  V4<double> t{0, 0, 0, 0};
  if (valid) {
    const V4<double> a = GA[I], b = GB[I];
    t = GT[I];
    const int2 ei = edges[I];
    const int4 ci = cinfo[I];
    const int m = ci.z;
    int q0, q1;
    if (ci.w && m <= 2 * kBand + 1) {
      q0 = 0;
      q1 = m - 1;
    } else if (ci.w) {
      q0 = ci.y - kBand;
      q1 = ci.y + kBand;
    } else {
      q0 = max(0, ci.y - kBand);
      q1 = min(m - 1, ci.y + kBand);
    }
    for (int q = q0 + sub; q <= q1; q += 4) {
      const int qq = ((q % m) + m) % m;
      const int J = chain_edge[ci.x + qq];
      const int2 ej = edges[J];
      const bool skip = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
      const V4<double> qa = GA[J], qb = GB[J], qt = GT[J];
      tpe_edge_pair<double, EC, GRAD, true>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y, qt.z,
                                            qa.w, skip ? 0.0 : 0.25 * qa.w, skip ? 1.0 : 0.0, half_alpha, half_beta,
                                            beta, E, S, G1x, G1y, G1z, Gt1, G2x, G2y, G2z, Gt2, Hx, Hy, Hz);
    }
  }
  auto red4 = [](double v) {  // (v0 + v1) + (v2 + v3) on every lane of the group
    v += __shfl_xor(v, 1, 64);
    return v + __shfl_xor(v, 2, 64);
  };
  constexpr int NS = GRAD ? kTpeSlots : 1;
  double v[kTpeSlots] = {E, S, G1x, G1y, G1z, G2x, G2y, G2z, Gt1, Gt2, Hx, Hy, Hz, 0.0};
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = red4(v[k]);
  if (GRAD) v[13] = t.x * v[10] + t.y * v[11] + t.z * v[12];  // T.H: H holds multiples of T
  if (!valid || sub != 0) return;
  double* out = part + (size_t)chunk * NS * nE + I;
#pragma unroll
  for (int k = 0; k < NS; ++k) out[(size_t)k * nE] = v[k];
}

// Sums over the partial-sum chunks of ns <= NS slots for the 64 edges of a
// workgroup of 256 threads (edge I = 64 blockIdx.x + lane): wave g sums the
// chunks g, g + 4, ... below nc, the four partial sums are added in wave
// order and then the chunk band_chunk (when >= 0).  Every thread must call
// it; the sums are returned in wave 0.
template <int NS>
__device__ __forceinline__ void sum_chunks4(const double* __restrict__ part, int nc, int band_chunk, int ns, int nE,
                                            int I, bool valid, double (&s)[NS]) {
  __shared__ double red[3][NS][64];
  const int g = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = 0.0;
  if (valid)
    for (int c = g; c < nc; c += 4)
#pragma unroll
      for (int k = 0; k < NS; ++k)
        if (k < ns) s[k] += part[((size_t)c * ns + k) * nE + I];
  if (g > 0)
#pragma unroll
    for (int k = 0; k < NS; ++k) red[g - 1][k][lane] = s[k];
  __syncthreads();
  if (g == 0)
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      s[k] = ((s[k] + red[0][k][lane]) + red[1][k][lane]) + red[2][k][lane];
      if (valid && k < ns && band_chunk >= 0) s[k] += part[((size_t)band_chunk * ns + k) * nE + I];
    }
}

// Sum the chunks and turn the accumulators into per-edge energy and endpoint
// partials: edge_out[I] = (E_I, dE/dg_i1 (3), dE/dg_i2 (3), -) (tpe_edge_record).
// Chunks 0 .. n - 1 with n = nch_e[I] (batch) or nchunk, then the near-band
// chunk `band_chunk` when it is >= 0.  64 edges per workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_tpe_finalize(const double* __restrict__ part, int nchunk,
                                                      const int* __restrict__ nch_e, int band_chunk, int nE, int grad,
                                                      const double* __restrict__ gd_a,
                                                      const double* __restrict__ gd_t, double* __restrict__ edge_out,
                                                      unsigned* __restrict__ status) {
  const int I = blockIdx.x * 64 + threadIdx.x % 64;
  const bool valid = I < nE;
  const int NS = grad ? kTpeSlots : 1;
  const int nc = valid ? (nch_e ? nch_e[I] : nchunk) : 0;
  double s[kTpeSlots];
  sum_chunks4<kTpeSlots>(part, nc, band_chunk, NS, nE, I, valid, s);
  if (threadIdx.x >= 64 || !valid) return;
  tpe_edge_record(s, grad != 0, gd_a[4 * I + 3], gd_t[4 * I], gd_t[4 * I + 1], gd_t[4 * I + 2],
                  edge_out + 8 * (size_t)I, status);
}

// dE_v = sum over incident (edge, endpoint) of the edge's endpoint partial.
__global__ void k_gather_vertex(const double* __restrict__ edge_out, const int* __restrict__ inc_off,
                                const int* __restrict__ inc, int nV, double* __restrict__ dE,
                                unsigned* __restrict__ status) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double gx = 0, gy = 0, gz = 0;
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    int code = inc[k];
    const double* o = edge_out + 8 * (size_t)(code >> 1) + 1 + 3 * (code & 1);
    gx += o[0];
    gy += o[1];
    gz += o[2];
  }
  dE[3 * v] = gx;
  dE[3 * v + 1] = gy;
  dE[3 * v + 2] = gz;
  if (!(isfinite(gx) & isfinite(gy) & isfinite(gz))) latch(status, kFlagResultNonfinite);
}

// Deterministic sum of edge_out[8 I + slot] over I: per-block partials, then one block.
__global__ void k_sum_slot(const double* __restrict__ edge_out, int slot, int n, double* __restrict__ partial) {
  __shared__ double sm[256];
  double v = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += edge_out[8 * (size_t)i + slot];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double* __restrict__ out,
                               unsigned* __restrict__ status) {
  __shared__ double sm[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += partial[i];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0];
    if (!isfinite(sm[0])) latch(status, kFlagResultNonfinite);
  }
}

static void sum_edge_slot(const Curve& c, int slot, double* out, hipStream_t s) {
  int nb = c.red_blocks;
  hipLaunchKernelGGL(k_sum_slot, dim3(nb), dim3(256), 0, s, c.edge_out, slot, c.nE, c.red);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, c.red, nb, out, c.status);
}

// ---------------------------------------------------------------------------
// Sobolev operator A = B + B0, matrix-free (gather form of the increment tables)
// ---------------------------------------------------------------------------
// Per RHS component u (three at once), per edge J:
//   s_J = (u_j2 - u_j1) / l_J  (D_J u = s_J T_J),   ubar_J = (u_j1 + u_j2) / 2.
// For target I, with rho = |g_ia - g_jb|^-(2 sigma + 1) and c_X = |T_X x d|^2:
//   Wq = sum_J l_J sum_ab rho               Q = sum_J l_J sum_ab rho <T_I,T_J> s_J
//   P0 = sum_J l_J sum_ab rho (c_I + c_J) / r^4      P = same weights times ubar_J
// then  q_I = l_I/2 (Wq s_I - Q)  and  p_I = l_I/4 (P0 ubar_I - P)  and
//   (B u)_i2 += q_I / l_I, (B u)_i1 -= q_I / l_I, (B0 u)_i1,i2 += p_I / 2,
// which is the printed increment table summed over J.  The diagonal of A is
//   diag_v = sum_{I at v} Wq_I / (2 l_I) + l_I P0_I / 16.
template <typename R>
__global__ void k_edge_rhs(const double* __restrict__ X, const int2* __restrict__ edges, int nE,
                           V4<R>* __restrict__ Sout, V4<R>* __restrict__ Uout) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  int2 e = edges[I];
  double ax = X[3 * e.x], ay = X[3 * e.x + 1], az = X[3 * e.x + 2];
  double bx = X[3 * e.y], by = X[3 * e.y + 1], bz = X[3 * e.y + 2];
  Sout[I] = V4<R>{R(bx - ax), R(by - ay), R(bz - az), R(0)};  // divided by l in the finalize / kernel
  Uout[I] = V4<R>{R(0.5 * (ax + bx)), R(0.5 * (ay + by)), R(0.5 * (az + bz)), R(0)};
}

template <typename R, int EC>
__device__ __forceinline__ void sob_tile(const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB,
                                         const V4<R>* __restrict__ GT, const int2* __restrict__ edges,
                                         const V4<R>* __restrict__ RS, const V4<R>* __restrict__ RU, int nE, int I0,
                                         int tcount, int s0, int s1, int chunk, R half_expo,
                                         double* __restrict__ part) {
  __shared__ V4<R> sA[kTile], sB[kTile], sT[kTile], sS[kTile], sU[kTile];
  __shared__ int2 sE[kTile];
  __shared__ int4 sRed[2][kTile / 64];  // vertex ranges: [0] targets, [1] the staged sources
  const int tid = threadIdx.x;
  const int I = I0 + tid;
  const bool act = tid < tcount;
  const int Ic = act ? I : I0;
  const V4<R> a = GA[Ic], b = GB[Ic], t = GT[Ic];
  const int2 ei = act ? edges[Ic] : make_int2(-1, -2);
  wave_range(make_int4(min(ei.x, ei.y), max(ei.x, ei.y), 0, 0), act, sRed[0]);
  double acc[kSobSlots];
#pragma unroll
  for (int k = 0; k < kSobSlots; ++k) acc[k] = 0.0;
  for (int t0 = s0; t0 < s1; t0 += kTile) {
    __syncthreads();
    const bool staged = t0 + tid < s1;
    int2 ej = make_int2(-1, -2);
    if (staged) {
      const int j = t0 + tid;
      V4<R> ga = GA[j], gs = RS[j];
      const R il = R(1) / ga.w;
      sA[tid] = ga;
      sB[tid] = GB[j];
      sT[tid] = GT[j];
      sS[tid] = V4<R>{gs.x * il, gs.y * il, gs.z * il, R(0)};
      sU[tid] = RU[j];
      ej = edges[j];
      sE[tid] = ej;
    }
    wave_range(make_int4(min(ej.x, ej.y), max(ej.x, ej.y), 0, 0), staged, sRed[1]);
    __syncthreads();
    const int cnt = min(kTile, s1 - t0);
    // Pairs are tested for a shared vertex one by one only where the vertex
    // ranges of the two tiles overlap.
    const int4 tr = range_of(sRed[0]), sr = range_of(sRed[1]);
    const bool test = !(tr.w < sr.x || sr.w < tr.x);
    for (int u0 = 0; u0 < cnt; u0 += kSub) {
      const int u1 = min(cnt, u0 + kSub);
      R Wq = 0, Qx = 0, Qy = 0, Qz = 0, P0 = 0, Px = 0, Py = 0, Pz = 0;
      auto sweep = [&](auto tested) {
        for (int u = u0; u < u1; ++u) {
          const V4<R> qa = sA[u], qb = sB[u], qt = sT[u];
          R rho, rho0, w = qa.w;
          if constexpr (decltype(tested)::value) {
            const int2 ej = sE[u];
            const bool skip = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
            w = skip ? R(0) : w;
            sob_edge_pair<R, EC, true>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y, qt.z, qa.w,
                                       skip ? R(1) : R(0), half_expo, rho, rho0);
          } else {
            sob_edge_pair<R, EC, false>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y, qt.z, qa.w,
                                        R(0), half_expo, rho, rho0);
          }
          const V4<R> sj = sS[u], uj = sU[u];
          const R wr = w * rho, w0 = w * rho0;
          const R tt = wr * (t.x * qt.x + t.y * qt.y + t.z * qt.z);
          Wq += wr;
          Qx = fma(tt, sj.x, Qx);
          Qy = fma(tt, sj.y, Qy);
          Qz = fma(tt, sj.z, Qz);
          P0 += w0;
          Px = fma(w0, uj.x, Px);
          Py = fma(w0, uj.y, Py);
          Pz = fma(w0, uj.z, Pz);
        }
      };
      if (test) sweep(std::true_type{});
      else sweep(std::false_type{});
      acc[0] += (double)Wq; acc[1] += (double)Qx; acc[2] += (double)Qy; acc[3] += (double)Qz;
      acc[4] += (double)P0; acc[5] += (double)Px; acc[6] += (double)Py; acc[7] += (double)Pz;
    }
  }
  if (act) {
    double* out = part + (size_t)chunk * kSobSlots * nE + I;
#pragma unroll
    for (int k = 0; k < kSobSlots; ++k) out[(size_t)k * nE] = acc[k];
  }
}

template <typename R, int EC>
__global__ __launch_bounds__(kTile) void k_sob_pairs(
    const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB, const V4<R>* __restrict__ GT,
    const int2* __restrict__ edges, const V4<R>* __restrict__ RS, const V4<R>* __restrict__ RU,
    int nE, int src_per_chunk, R half_expo, double* __restrict__ part) {
  const int I0 = blockIdx.x * kTile;
  const int s0 = blockIdx.y * src_per_chunk;
  sob_tile<R, EC>(GA, GB, GT, edges, RS, RU, nE, I0, min(kTile, nE - I0), s0, min(nE, s0 + src_per_chunk),
                  blockIdx.y, half_expo, part);
}

template <typename R, int EC>
__global__ __launch_bounds__(kTile) void k_sob_items(
    const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB, const V4<R>* __restrict__ GT,
    const int2* __restrict__ edges, const V4<R>* __restrict__ RS, const V4<R>* __restrict__ RU, int nE,
    const int4* __restrict__ items, int n_items, int* __restrict__ counter, const int* __restrict__ inst_of_edge,
    const int* __restrict__ mask, R half_expo, double* __restrict__ part) {
  for (int it = next_item(counter); it < n_items; it = next_item(counter)) {
    const int4 w = items[it];
    if (mask && !mask[inst_of_edge[w.x]]) continue;
    sob_tile<R, EC>(GA, GB, GT, edges, RS, RU, nE, w.x, w.w & 0xffff, w.y, w.z, w.w >> 16, half_expo, part);
  }
}

// Per edge: endpoint contributions of B u + B0 u (3 comps each) and the
// diagonal pieces.  edge_out[I] = (y_i1 (3), y_i2 (3), dg_B, dg_B0).
__global__ __launch_bounds__(256) void k_sob_finalize(const double* __restrict__ part, int nchunk,
                                                      const int* __restrict__ nch_e, int nE,
                                                      const double* __restrict__ X, const int2* __restrict__ edges,
                                                      double* __restrict__ edge_out) {
  const int I = blockIdx.x * 64 + threadIdx.x % 64;  // 64 edges per workgroup of 256 threads
  const bool valid = I < nE;
  const int nc = valid ? (nch_e ? nch_e[I] : nchunk) : 0;
  double s[kSobSlots];
  sum_chunks4<kSobSlots>(part, nc, -1, kSobSlots, nE, I, valid, s);
  if (threadIdx.x >= 64 || !valid) return;
  int2 e = edges[I];
  double a[3], b[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = X[3 * e.x + k];
    b[k] = X[3 * e.y + k];
  }
  double* o = edge_out + 8 * (size_t)I;
  // o[6], o[7] hold l_I on entry (written by the launcher's length kernel)
  const double l = o[7];
  const double il = 1.0 / l;
  for (int k = 0; k < 3; ++k) {
    const double sI = (b[k] - a[k]) * il;
    const double uI = 0.5 * (a[k] + b[k]);
    const double qoverl = 0.5 * (s[0] * sI - s[1 + k]);  // q_I / l_I
    const double phalf = 0.125 * l * (s[4] * uI - s[5 + k]);  // p_I / 2
    o[k] = -qoverl + phalf;
    o[3 + k] = qoverl + phalf;
  }
  o[6] = s[0] * il * 0.5 + l * s[4] * (1.0 / 16.0);
}

template <typename R>
__global__ void k_edge_length(const V4<R>* __restrict__ GA, int nE, double* __restrict__ edge_out) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I < nE) edge_out[8 * (size_t)I + 7] = (double)GA[I].w;
}

__global__ void k_gather_sob(const double* __restrict__ edge_out, const int* __restrict__ inc_off,
                             const int* __restrict__ inc, int nV, double* __restrict__ Y,
                             double* __restrict__ diag) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double y0 = 0, y1 = 0, y2 = 0, dg = 0;
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    int code = inc[k];
    const double* o = edge_out + 8 * (size_t)(code >> 1);
    const double* oy = o + 3 * (code & 1);
    y0 += oy[0];
    y1 += oy[1];
    y2 += oy[2];
    dg += o[6];
  }
  if (Y) {
    Y[3 * v] = y0;
    Y[3 * v + 1] = y1;
    Y[3 * v + 2] = y2;
  }
  if (diag) diag[v] = dg;
}

// ---------------------------------------------------------------------------
// edge-midpoint energy and differential (the sum Barnes-Hut approximates)
// ---------------------------------------------------------------------------
// Per target I with d = x_I - x_J and weights l_J:
//  0 E = sum l_J k(d, T_I); 1 S = sum l_J (k_I + k_J); 2-4 G = sum l_J grad_d(k_I + k_J)
//  minus its T_I part, 5 Gt; 6-8 Hd, 9 Ht as in the trapezoid kernel.
constexpr int kMidSlotsUsed = 10;

template <typename R, int EC, bool BAND>
__global__ __launch_bounds__(kTile) void k_mid_pairs(
    const V4<R>* __restrict__ GA, const V4<R>* __restrict__ GB, const V4<R>* __restrict__ GT,
    const int2* __restrict__ edges, const int4* __restrict__ cinfo, int nE, int src_per_chunk, R half_alpha,
    R half_beta, R beta, double* __restrict__ part) {
  __shared__ V4<R> sX[kTile], sT[kTile];
  __shared__ int2 sE[kTile];
  __shared__ int4 sC[BAND ? kTile : 1];
  const int tid = threadIdx.x;
  const int I = blockIdx.x * kTile + tid;
  const bool act = I < nE;
  const int Ic = act ? I : nE - 1;
  const V4<R> a = GA[Ic], b = GB[Ic], t = GT[Ic];
  const R mx = R(0.5) * (a.x + b.x), my = R(0.5) * (a.y + b.y), mz = R(0.5) * (a.z + b.z);
  const int2 ei = act ? edges[Ic] : make_int2(-1, -2);
  int4 ci = make_int4(-1, 0, 0, 0);
  if constexpr (BAND) ci = act ? cinfo[Ic] : make_int4(-1, 0, 0, 0);
  double acc[kMidSlotsUsed];
#pragma unroll
  for (int k = 0; k < kMidSlotsUsed; ++k) acc[k] = 0.0;
  const int s0 = blockIdx.y * src_per_chunk;
  const int s1 = min(nE, s0 + src_per_chunk);
  for (int t0 = s0; t0 < s1; t0 += kTile) {
    __syncthreads();
    if (t0 + tid < s1) {
      const int j = t0 + tid;
      V4<R> ga = GA[j], gb = GB[j];
      sX[tid] = V4<R>{R(0.5) * (ga.x + gb.x), R(0.5) * (ga.y + gb.y), R(0.5) * (ga.z + gb.z), ga.w};
      sT[tid] = GT[j];
      sE[tid] = edges[j];
      if constexpr (BAND) sC[tid] = cinfo[j];
    }
    __syncthreads();
    const int cnt = min(kTile, s1 - t0);
    for (int u0 = 0; u0 < cnt; u0 += kSub) {
      const int u1 = min(cnt, u0 + kSub);
      R E = 0, S = 0, Gx = 0, Gy = 0, Gz = 0, Gt = 0, Hx = 0, Hy = 0, Hz = 0, Ht = 0;
      for (int u = u0; u < u1; ++u) {
        const V4<R> q = sX[u], qt = sT[u];
        bool skip;
        if constexpr (BAND) {
          skip = chain_near(ci, sC[u]);
        } else {
          const int2 ej = sE[u];
          skip = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
        }
        const R w = skip ? R(0) : q.w;
        tpe_vertex_pair<R, EC, true>(mx, my, mz, t.x, t.y, t.z, q.x, q.y, q.z, qt.x, qt.y, qt.z, skip, w, half_alpha,
                                     half_beta, beta, E, S, Gx, Gy, Gz, Gt, Hx, Hy, Hz, Ht);
      }
      acc[0] += (double)E; acc[1] += (double)S; acc[2] += (double)Gx; acc[3] += (double)Gy;
      acc[4] += (double)Gz; acc[5] += (double)Gt; acc[6] += (double)Hx; acc[7] += (double)Hy;
      acc[8] += (double)Hz; acc[9] += (double)Ht;
    }
  }
  if (act) {
    double* out = part + (size_t)blockIdx.y * kMidSlotsUsed * nE + I;
#pragma unroll
    for (int k = 0; k < kMidSlotsUsed; ++k) out[(size_t)k * nE] = acc[k];
  }
}

// FP64 near band of the edge-midpoint sum (the pairs the BAND kernel skips).
template <int EC>
__global__ void k_mid_band(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                           const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                           const int4* __restrict__ cinfo, const int* __restrict__ chain_edge, int nE,
                           double half_alpha, double half_beta, double beta, int chunk, double* __restrict__ part) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const V4<double> a = GA[I], b = GB[I], t = GT[I];
  const double mx = 0.5 * (a.x + b.x), my = 0.5 * (a.y + b.y), mz = 0.5 * (a.z + b.z);
  const int2 ei = edges[I];
  const int4 ci = cinfo[I];
  const int m = ci.z;
  int q0, q1;
  if (ci.w && m <= 2 * kBand + 1) {
    q0 = 0;
    q1 = m - 1;
  } else if (ci.w) {
    q0 = ci.y - kBand;
    q1 = ci.y + kBand;
  } else {
    q0 = max(0, ci.y - kBand);
    q1 = min(m - 1, ci.y + kBand);
  }
  double E = 0, S = 0, Gx = 0, Gy = 0, Gz = 0, Gt = 0, Hx = 0, Hy = 0, Hz = 0, Ht = 0;
  for (int q = q0; q <= q1; ++q) {
    const int J = chain_edge[ci.x + ((q % m) + m) % m];
    const int2 ej = edges[J];
    if ((ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y)) continue;
    const V4<double> qa = GA[J], qb = GB[J], qt = GT[J];
    tpe_vertex_pair<double, EC, true>(mx, my, mz, t.x, t.y, t.z, 0.5 * (qa.x + qb.x), 0.5 * (qa.y + qb.y),
                                      0.5 * (qa.z + qb.z), qt.x, qt.y, qt.z, false, qa.w, half_alpha, half_beta, beta,
                                      E, S, Gx, Gy, Gz, Gt, Hx, Hy, Hz, Ht);
  }
  const double v[kMidSlotsUsed] = {E, S, Gx, Gy, Gz, Gt, Hx, Hy, Hz, Ht};
  double* out = part + (size_t)chunk * kMidSlotsUsed * nE + I;
  for (int k = 0; k < kMidSlotsUsed; ++k) out[(size_t)k * nE] = v[k];
}

__global__ void k_mid_finalize(const double* __restrict__ part, int nchunk, int nE,
                               const double* __restrict__ gd_a, const double* __restrict__ gd_t,
                               double* __restrict__ edge_out, unsigned* __restrict__ status) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  double s[kMidSlotsUsed];
  for (int k = 0; k < kMidSlotsUsed; ++k) {
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += part[((size_t)c * kMidSlotsUsed + k) * nE + I];
    s[k] = v;
  }
  const double l = gd_a[4 * I + 3];
  bool fin = true;
  for (int k = 0; k < kMidSlotsUsed; ++k) fin &= isfinite(s[k]);
  if (!fin && isfinite(l) && l > 0.0) latch(status, kFlagPairOverflow);
  const double Tx = gd_t[4 * I], Ty = gd_t[4 * I + 1], Tz = gd_t[4 * I + 2];
  const double S = s[1];
  const double Hx = s[6] - s[9] * Tx, Hy = s[7] - s[9] * Ty, Hz = s[8] - s[9] * Tz;
  const double px = 0.5 * l * (s[2] - s[5] * Tx), py = 0.5 * l * (s[3] - s[5] * Ty),
               pz = 0.5 * l * (s[4] - s[5] * Tz);
  double* o = edge_out + 8 * (size_t)I;
  o[0] = l * s[0];
  o[1] = -Tx * S + px + 2.0 * Hx;
  o[2] = -Ty * S + py + 2.0 * Hy;
  o[3] = -Tz * S + pz + 2.0 * Hz;
  o[4] = Tx * S + px - 2.0 * Hx;
  o[5] = Ty * S + py - 2.0 * Hy;
  o[6] = Tz * S + pz - 2.0 * Hz;
}

// ---------------------------------------------------------------------------
// dense FP64 assembly (vertex-pair gather of the increment tables), any graph
// ---------------------------------------------------------------------------
// Off-diagonal entry (v, w):
//   sum over disjoint I at v, J at w of
//      -2 s_I(v) s_J(w) w_IJ <T_I,T_J> / (l_I l_J) - (w0_IJ + w0_JI) / 4
//   plus, when v and w are the two ends of an edge K,
//      -Wq_K / (2 l_K) + l_K P0_K / 16
// with s(i1) = -1, s(i2) = +1.  The diagonal is minus the row sum (A 1 = 0).
template <int EC>
__global__ void k_assemble(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                           const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                           const int* __restrict__ inc_off, const int* __restrict__ inc,
                           const double* __restrict__ edge_out, int nV, double half_expo,
                           double* __restrict__ A) {
  const int w_ = blockIdx.x * blockDim.x + threadIdx.x;
  const int v_ = blockIdx.y * blockDim.y + threadIdx.y;
  if (v_ >= nV || w_ >= nV) return;
  if (v_ == w_) return;
  double acc = 0.0;
  for (int kv = inc_off[v_]; kv < inc_off[v_ + 1]; ++kv) {
    const int I = inc[kv] >> 1;
    const double sv = (inc[kv] & 1) ? 1.0 : -1.0;
    const int2 ei = edges[I];
    const V4<double> ia = GA[I], ib = GB[I], ti = GT[I];
    for (int kw = inc_off[w_]; kw < inc_off[w_ + 1]; ++kw) {
      const int J = inc[kw] >> 1;
      const double sw = (inc[kw] & 1) ? 1.0 : -1.0;
      const int2 ej = edges[J];
      if (I == J) {
        // v and w are the two ends of edge I
        const double* o = edge_out + 8 * (size_t)I;  // (Wq, P0) stored at slots 0, 1
        acc += -o[0] / (2.0 * ia.w) + ia.w * o[1] / 16.0;
        continue;
      }
      if (ei.x == ej.x || ei.x == ej.y || ei.y == ej.x || ei.y == ej.y) continue;
      const V4<double> ja = GA[J], jb = GB[J], tj = GT[J];
      double rho = 0.0, rho0 = 0.0;
      const V4<double>* P[2] = {&ia, &ib};
      const V4<double>* Q[2] = {&ja, &jb};
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
          const double dx = P[x]->x - Q[y]->x, dy = P[x]->y - Q[y]->y, dz = P[x]->z - Q[y]->z;
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double rs = f_rsq<double>(r2), ri = rs * rs;
          const double p = pow_sigma<EC, double>(r2, rs, ri, half_expo);
          const double cI = cross_norm2<double>(ti.x, ti.y, ti.z, dx, dy, dz);
          const double cJ = cross_norm2<double>(tj.x, tj.y, tj.z, dx, dy, dz);
          rho += p;
          rho0 += p * (cI + cJ) * ri * ri;
        }
      const double wIJ = 0.25 * ia.w * ja.w * rho;
      const double w0s = 0.25 * ia.w * ja.w * rho0;
      const double tt = ti.x * tj.x + ti.y * tj.y + ti.z * tj.z;
      acc += -2.0 * sv * sw * wIJ * tt / (ia.w * ja.w) - 0.25 * w0s;
    }
  }
  A[(size_t)v_ * nV + w_] = acc;
}

__global__ void k_diag_rowsum(double* __restrict__ A, int nV) {
  __shared__ double sm[256];
  const int v = blockIdx.x;
  double s = 0.0;
  for (int w = threadIdx.x; w < nV; w += 256)
    if (w != v) s += A[(size_t)v * nV + w];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) A[(size_t)v * nV + v] = -sm[0];
}

// ---------------------------------------------------------------------------
// sphere-obstacle penalty (Sec. 7.1, surface potential; M a sphere)
// ---------------------------------------------------------------------------
// The surface integral of |x_M - y|^-p over a sphere of radius R and centre
// c, at a point y with r = |y - c| > R, integrates in closed form over the
// polar angle (u = r^2 + R^2 - 2 r R cos):
//   Psi(r) = (pi R / r) [u^q / q] from (r-R)^2 to (r+R)^2,  q = 1 - p/2
// (log for p = 2).  Per edge, with one midpoint sample: l_I Psi(|x_I - c|),
// whose endpoint derivatives are -+T_I Psi + l_I Psi'(r) (x_I - c) / (2 r).
// A midpoint on or inside the sphere makes the energy infinite.
__global__ void k_obstacle(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                           const V4<double>* __restrict__ GT, int nE, double cx, double cy, double cz, double R,
                           double p, double w, int grad, double* __restrict__ edge_out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const V4<double> a = GA[I], b = GB[I], t = GT[I];
  const double dx = 0.5 * (a.x + b.x) - cx, dy = 0.5 * (a.y + b.y) - cy, dz = 0.5 * (a.z + b.z) - cz;
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double l = a.w;
  double* o = edge_out + 8 * (size_t)I;
  if (!(r > R)) {
    o[0] += INFINITY;
    return;
  }
  const double hi = (r + R) * (r + R), lo = (r - R) * (r - R);
  double F, dF;
  if (p == 2.0) {
    F = log(hi / lo);
    dF = 2.0 / (r + R) - 2.0 / (r - R);
  } else {
    const double q = 1.0 - 0.5 * p;
    const double hq = pow(hi, q), lq = pow(lo, q);
    F = (hq - lq) / q;
    dF = 2.0 * (r + R) * hq / hi - 2.0 * (r - R) * lq / lo;
  }
  const double psi = M_PI * R * F / r;
  const double dpsi = M_PI * R * (dF / r - F / (r * r));
  o[0] += w * l * psi;
  if (!grad) return;
  const double f = w * 0.5 * l * dpsi / r;
  o[1] += -w * t.x * psi + f * dx;
  o[2] += -w * t.y * psi + f * dy;
  o[3] += -w * t.z * psi + f * dz;
  o[4] += w * t.x * psi + f * dx;
  o[5] += w * t.y * psi + f * dy;
  o[6] += w * t.z * psi + f * dz;
}

// ---------------------------------------------------------------------------
// penalties (Sec. 7.1): per edge I, with e = l T its edge vector,
//   total length   w_len l                    d/de = w_len T
//   field          w_field (l - (e.X)^2 / l)  d/de = w_field (T - 2 (T.X) X + (T.X)^2 T)
//   length diff.   half of (l_I - l_J)^2 at each endpoint v of degree two (J the other edge at v),
//                  d/de = 2 sum_v (l_I - l_J) T   (the J side comes from edge J's own thread)
// and d/d(gamma_i2) = d/de, d/d(gamma_i1) = -d/de.
// ---------------------------------------------------------------------------
__global__ void k_penalties(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GT,
                            const int2* __restrict__ edges, const int* __restrict__ inc_off,
                            const int* __restrict__ inc, int nE, double w_len, double w_diff, double w_field,
                            double X0, double X1, double X2, int grad, double* __restrict__ edge_out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const double l = GA[I].w;
  const V4<double> t = GT[I];
  double E = w_len * l, gl = w_len;  // gl: coefficient of T in d/de
  if (w_diff != 0.0) {
    const int2 e = edges[I];
    const int ends[2] = {e.x, e.y};
    for (int k = 0; k < 2; ++k) {
      const int v = ends[k];
      if (inc_off[v + 1] - inc_off[v] != 2) continue;
      const int J0 = inc[inc_off[v]] >> 1, J1 = inc[inc_off[v] + 1] >> 1;
      const int J = J0 == I ? J1 : J0;
      const double d = l - GA[J].w;
      E += 0.5 * w_diff * d * d;
      gl += 2.0 * w_diff * d;
    }
  }
  double g[3] = {gl * t.x, gl * t.y, gl * t.z};
  if (w_field != 0.0) {
    const double tx = t.x * X0 + t.y * X1 + t.z * X2;
    E += w_field * l * (1.0 - tx * tx);
    g[0] += w_field * (t.x - 2.0 * tx * X0 + tx * tx * t.x);
    g[1] += w_field * (t.y - 2.0 * tx * X1 + tx * tx * t.y);
    g[2] += w_field * (t.z - 2.0 * tx * X2 + tx * tx * t.z);
  }
  double* o = edge_out + 8 * (size_t)I;
  o[0] += E;
  if (!grad) return;
  for (int c = 0; c < 3; ++c) {
    o[1 + c] -= g[c];
    o[4 + c] += g[c];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

rc_status launch_penalties(const Curve& c, bool grad, hipStream_t s) {
  if (c.spot.on) RC_TRY(launch_surface_potential(c, grad, s));
  if (!c.pen.on) return RC_OK;
  const Penalties& p = c.pen;
  hipLaunchKernelGGL(k_penalties, dim3(cdiv(c.nE, 256)), dim3(256), 0, s, (const V4<double>*)c.gd.a,
                     (const V4<double>*)c.gd.t, (const int2*)c.edges, (const int*)c.inc_off, (const int*)c.inc, c.nE,
                     p.w_len, p.w_diff, p.w_field, p.X[0], p.X[1], p.X[2], grad ? 1 : 0, c.edge_out);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_geometry(const Curve& c, const double* gamma, rc_dtype prec, hipStream_t s) {
  // the FP64 copy is always kept (the finalize kernels read l_I and T_I from it), the FP32 one and the
  // vertex-pair geometry with it in the same launch
  const bool f32 = prec == RC_F32, vp = f32 && c.vp;
  const int n = vp ? std::max(c.nE, c.nV) : c.nE;
  hipLaunchKernelGGL(k_geometry, dim3(cdiv(n, 256)), dim3(256), 0, s, gamma, c.edges, c.nE, c.gd.a, c.gd.b, c.gd.t,
                     f32 ? c.gf.a : nullptr, f32 ? c.gf.b : nullptr, f32 ? c.gf.t : nullptr, c.inc_off, c.inc, c.nV,
                     vp ? c.vg[0] : nullptr, vp ? c.vg[1] : nullptr, vp ? c.vg[2] : nullptr,
                     vp ? c.vgd[0] : nullptr, vp ? c.vgd[1] : nullptr, vp ? c.vgd[2] : nullptr, c.status);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

template <typename R, int EC, bool GRAD>
static void run_tpe(const Curve& c, const EdgeGeom<R>& g, double alpha, double beta, hipStream_t s) {
  dim3 grid(cdiv(c.nE, kTile), c.nchunk);
  const bool timed = GRAD && c.timer && c.timer->on;
  const bool band = std::is_same<R, float>::value && c.chain;
  if (c.n_inst > 0) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, c.counter);
    if (timed) c.timer->mark(c.timer->tpe, s);
    if (band)
      hipLaunchKernelGGL((k_tpe_items<R, EC, GRAD, true>), dim3(c.persist_blocks), dim3(kTile), 0, s, g.a, g.b, g.t,
                         c.edges, c.cinfo, c.nE, c.items, c.n_items, c.counter, c.inst_of_edge, c.inst_mask,
                         R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);
    else
      hipLaunchKernelGGL((k_tpe_items<R, EC, GRAD, false>), dim3(c.persist_blocks), dim3(kTile), 0, s, g.a, g.b,
                         g.t, c.edges, c.cinfo, c.nE, c.items, c.n_items, c.counter, c.inst_of_edge, c.inst_mask,
                         R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);
    if (timed) c.timer->mark(c.timer->tpe, s);
    if (band)
      hipLaunchKernelGGL((k_tpe_band<EC, GRAD>), dim3(cdiv(c.nE, 64)), dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t,
                         c.edges, c.cinfo, c.chain_edge, c.nE, 0.5 * alpha, 0.5 * beta, beta, c.nchunk, c.inst_of_edge,
                         c.inst_mask, c.part);
    return;
  }
  if (band) {
    if (timed) c.timer->mark(c.timer->tpe, s);
    hipLaunchKernelGGL((k_tpe_pairs<R, EC, GRAD, true>), grid, dim3(kTile), 0, s, g.a, g.b, g.t, c.edges, c.cinfo,
                       c.nE, c.src_per_chunk, R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);
    if (timed) c.timer->mark(c.timer->tpe, s);
    hipLaunchKernelGGL((k_tpe_band<EC, GRAD>), dim3(cdiv(c.nE, 64)), dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t,
                       c.edges, c.cinfo, c.chain_edge, c.nE, 0.5 * alpha, 0.5 * beta, beta, c.nchunk, c.inst_of_edge,
                         c.inst_mask, c.part);
  } else {
    if (timed) c.timer->mark(c.timer->tpe, s);
    hipLaunchKernelGGL((k_tpe_pairs<R, EC, GRAD, false>), grid, dim3(kTile), 0, s, g.a, g.b, g.t, c.edges,
                       c.cinfo, c.nE, c.src_per_chunk, R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);
    if (timed) c.timer->mark(c.timer->tpe, s);
  }
}

template <typename R, bool GRAD>
static void dispatch_tpe(const Curve& c, const EdgeGeom<R>& g, double alpha, double beta, hipStream_t s) {
  switch (exp_case(alpha, beta)) {
    case kA2B4: run_tpe<R, kA2B4, GRAD>(c, g, alpha, beta, s); break;
    case kA2B45: run_tpe<R, kA2B45, GRAD>(c, g, alpha, beta, s); break;
    case kA3B6: run_tpe<R, kA3B6, GRAD>(c, g, alpha, beta, s); break;
    default: run_tpe<R, kGeneral, GRAD>(c, g, alpha, beta, s); break;
  }
}

rc_status launch_tpe(const Curve& c, double alpha, double beta, rc_dtype prec, bool grad,
                     double* energy, double* dE, hipStream_t s) {
  if (c.vp && prec == RC_F32 && alpha == 2.0 && c.n_inst == 0 && !c.obstacle.on) {
    // alpha = 2 chain graph: the vertex-pair form, its FP64 near band in chunk 0
    RC_TRY(launch_tpe_vp_pairs(c, beta, grad, s));  // the near band writes the edge records
    // without penalties the edge pass also takes the first pass of the total energy (the same sums in the
    // same order as sum_edge_slot)
    const bool fold = energy && !c.spot.on && !c.pen.on;
    RC_TRY(launch_tpe_vp_finish(c, beta, grad, dE, fold ? c.red : nullptr, s));
    if (fold) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, c.red, c.red_blocks, energy, c.status);
    else if (energy) sum_edge_slot(c, 0, energy, s);
    RC_HIP(hipGetLastError());
    return RC_OK;
  }
  if (prec == RC_F32) {
    if (grad) dispatch_tpe<float, true>(c, c.gf, alpha, beta, s);
    else dispatch_tpe<float, false>(c, c.gf, alpha, beta, s);
  } else {
    if (grad) dispatch_tpe<double, true>(c, c.gd, alpha, beta, s);
    else dispatch_tpe<double, false>(c, c.gd, alpha, beta, s);
  }
  RC_HIP(hipGetLastError());
  const int band_chunk = (prec == RC_F32 && c.chain) ? c.nchunk : -1;
  hipLaunchKernelGGL(k_tpe_finalize, dim3(cdiv(c.nE, 64)), dim3(256), 0, s, c.part, c.nchunk,
                     (const int*)(c.n_inst > 0 ? c.nch_e : nullptr), band_chunk, c.nE, grad ? 1 : 0,
                     (const double*)c.gd.a, (const double*)c.gd.t, c.edge_out, c.status);
  if (c.obstacle.on) {
    const Obstacle& o = c.obstacle;
    hipLaunchKernelGGL(k_obstacle, dim3(cdiv(c.nE, 256)), dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.nE, o.c[0],
                       o.c[1], o.c[2], o.R, o.p, o.w, grad ? 1 : 0, c.edge_out);
  }
  RC_TRY(launch_penalties(c, grad, s));
  if (grad && dE)
    hipLaunchKernelGGL(k_gather_vertex, dim3(cdiv(c.nV, 256)), dim3(256), 0, s, c.edge_out, c.inc_off,
                       c.inc, c.nV, dE, c.status);
  if (energy) sum_edge_slot(c, 0, energy, s);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

template <typename R, int EC>
static void run_sob(const Curve& c, const EdgeGeom<R>& g, V4<R>* const* rhs, double half_expo, hipStream_t s) {
  dim3 grid(cdiv(c.nE, kTile), c.nchunk);
  const bool timed = c.timer && c.timer->on;
  std::vector<hipEvent_t>* tv = timed ? (std::is_same<R, float>::value ? &c.timer->sob : &c.timer->sob64) : nullptr;
  if (c.n_inst > 0) hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, c.counter);
  if (timed) c.timer->mark(*tv, s);
  if (c.n_inst > 0)
    hipLaunchKernelGGL((k_sob_items<R, EC>), dim3(c.persist_blocks), dim3(kTile), 0, s, g.a, g.b, g.t, c.edges,
                       rhs[0], rhs[1], c.nE, c.items, c.n_items, c.counter, c.inst_of_edge, c.inst_mask,
                       R(half_expo), c.part);
  else
    hipLaunchKernelGGL((k_sob_pairs<R, EC>), grid, dim3(kTile), 0, s, g.a, g.b, g.t, c.edges, rhs[0], rhs[1],
                       c.nE, c.src_per_chunk, R(half_expo), c.part);
  if (timed) c.timer->mark(*tv, s);
}

template <typename R>
static void dispatch_sob(const Curve& c, const EdgeGeom<R>& g, V4<R>* const* rhs, double alpha, double beta,
                         hipStream_t s) {
  const double sigma = (beta - 1.0) / alpha - 1.0;
  const double half_expo = 0.5 * (2.0 * sigma + 1.0);
  switch (exp_case(alpha, beta)) {
    case kA2B4: run_sob<R, kA2B4>(c, g, rhs, half_expo, s); break;
    case kA2B45: run_sob<R, kA2B45>(c, g, rhs, half_expo, s); break;
    default: run_sob<R, kGeneral>(c, g, rhs, half_expo, s); break;
  }
}

rc_status launch_sobolev(const Curve& c, double alpha, double beta, rc_dtype prec, const double* X,
                         double* Y, double* diag, hipStream_t s) {
  dim3 g1(cdiv(c.nE, 256)), b1(256);
  if (prec == RC_F32) {
    hipLaunchKernelGGL(k_edge_rhs<float>, g1, b1, 0, s, X, c.edges, c.nE, c.rhs_f[0], c.rhs_f[1]);
    dispatch_sob<float>(c, c.gf, c.rhs_f, alpha, beta, s);
  } else {
    hipLaunchKernelGGL(k_edge_rhs<double>, g1, b1, 0, s, X, c.edges, c.nE, c.rhs_d[0], c.rhs_d[1]);
    dispatch_sob<double>(c, c.gd, c.rhs_d, alpha, beta, s);
  }
  RC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_edge_length<double>, g1, b1, 0, s, c.gd.a, c.nE, c.edge_out);
  hipLaunchKernelGGL(k_sob_finalize, dim3(cdiv(c.nE, 64)), dim3(256), 0, s, c.part, c.nchunk,
                     (const int*)(c.n_inst > 0 ? c.nch_e : nullptr), c.nE, X, c.edges, c.edge_out);
  hipLaunchKernelGGL(k_gather_sob, dim3(cdiv(c.nV, 256)), b1, 0, s, c.edge_out, c.inc_off, c.inc, c.nV, Y,
                     diag);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

template <typename R>
static void dispatch_mid(const Curve& c, const EdgeGeom<R>& g, double alpha, double beta, hipStream_t s) {
  dim3 grid(cdiv(c.nE, kTile), c.nchunk);
  const bool band = std::is_same<R, float>::value && c.chain;
#define RC_MID(EC)                                                                                             \
  if (band) {                                                                                                  \
    hipLaunchKernelGGL((k_mid_pairs<R, EC, true>), grid, dim3(kTile), 0, s, g.a, g.b, g.t, c.edges, c.cinfo,   \
                       c.nE, c.src_per_chunk, R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);                 \
    hipLaunchKernelGGL((k_mid_band<EC>), dim3(cdiv(c.nE, 64)), dim3(64), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges, \
                       c.cinfo, c.chain_edge, c.nE, 0.5 * alpha, 0.5 * beta, beta, c.nchunk, c.part);          \
  } else {                                                                                                     \
    hipLaunchKernelGGL((k_mid_pairs<R, EC, false>), grid, dim3(kTile), 0, s, g.a, g.b, g.t, c.edges, c.cinfo,  \
                       c.nE, c.src_per_chunk, R(0.5 * alpha), R(0.5 * beta), R(beta), c.part);                 \
  }
  switch (exp_case(alpha, beta)) {
    case kA2B4: RC_MID(kA2B4); break;
    case kA2B45: RC_MID(kA2B45); break;
    case kA3B6: RC_MID(kA3B6); break;
    default: RC_MID(kGeneral); break;
  }
#undef RC_MID
}

rc_status launch_midpoint(const Curve& c, double alpha, double beta, rc_dtype prec, double* energy,
                          double* dE, hipStream_t s) {
  if (prec == RC_F32) dispatch_mid<float>(c, c.gf, alpha, beta, s);
  else dispatch_mid<double>(c, c.gd, alpha, beta, s);
  RC_HIP(hipGetLastError());
  return finalize_midpoint(c, c.nchunk + ((prec == RC_F32 && c.chain) ? 1 : 0), energy, dE, s);
}

rc_status finalize_midpoint(const Curve& c, int nparts, double* energy, double* dE, hipStream_t s) {
  hipLaunchKernelGGL(k_mid_finalize, dim3(cdiv(c.nE, 256)), dim3(256), 0, s, c.part, nparts, c.nE,
                     (const double*)c.gd.a, (const double*)c.gd.t, c.edge_out, c.status);
  if (dE)
    hipLaunchKernelGGL(k_gather_vertex, dim3(cdiv(c.nV, 256)), dim3(256), 0, s, c.edge_out, c.inc_off,
                       c.inc, c.nV, dE, c.status);
  if (energy) sum_edge_slot(c, 0, energy, s);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// Per-edge (Wq, P0) of the operator kernel, stored in edge_out slots 0 and 1.
__global__ void k_pick_wq_p0(const double* __restrict__ part, int nchunk, const int* __restrict__ nch_e, int nE,
                             double* __restrict__ edge_out) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  double wq = 0.0, p0 = 0.0;
  const int nc = nch_e ? nch_e[I] : nchunk;
  for (int c = 0; c < nc; ++c) {
    wq += part[((size_t)c * kSobSlots + 0) * nE + I];
    p0 += part[((size_t)c * kSobSlots + 4) * nE + I];
  }
  edge_out[8 * (size_t)I] = wq;
  edge_out[8 * (size_t)I + 1] = p0;
}

// Zero right-hand sides by kernel (no memset nodes, so the call can be captured).
template <typename R>
__global__ void k_zero_rhs(V4<R>* __restrict__ a, V4<R>* __restrict__ b, int n) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n) return;
  a[I] = V4<R>{R(0), R(0), R(0), R(0)};
  b[I] = V4<R>{R(0), R(0), R(0), R(0)};
}

rc_status launch_edge_sums(const Curve& c, double alpha, double beta, rc_dtype prec, hipStream_t s) {
  dim3 g1(cdiv(c.nE, 256)), b1(256);
  if (prec == RC_F32) {
    hipLaunchKernelGGL(k_zero_rhs<float>, g1, b1, 0, s, c.rhs_f[0], c.rhs_f[1], c.nE);
    dispatch_sob<float>(c, c.gf, c.rhs_f, alpha, beta, s);
  } else {
    hipLaunchKernelGGL(k_zero_rhs<double>, g1, b1, 0, s, c.rhs_d[0], c.rhs_d[1], c.nE);
    dispatch_sob<double>(c, c.gd, c.rhs_d, alpha, beta, s);
  }
  hipLaunchKernelGGL(k_pick_wq_p0, g1, b1, 0, s, c.part, c.nchunk, (const int*)(c.n_inst > 0 ? c.nch_e : nullptr),
                     c.nE, c.edge_out);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_assemble_dense(const Curve& c, double alpha, double beta, double* A, hipStream_t s) {
  // the operator kernel's per-edge sums Wq and P0 do not depend on the input vector
  RC_TRY(launch_edge_sums(c, alpha, beta, RC_F64, s));
  const double sigma = (beta - 1.0) / alpha - 1.0;
  const double half_expo = 0.5 * (2.0 * sigma + 1.0);
  dim3 b2(16, 16), g2(cdiv(c.nV, 16), cdiv(c.nV, 16));
  switch (exp_case(alpha, beta)) {
    case kA2B4:
      hipLaunchKernelGGL(k_assemble<kA2B4>, g2, b2, 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges, c.inc_off, c.inc,
                         c.edge_out, c.nV, half_expo, A);
      break;
    case kA2B45:
      hipLaunchKernelGGL(k_assemble<kA2B45>, g2, b2, 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges, c.inc_off, c.inc,
                         c.edge_out, c.nV, half_expo, A);
      break;
    default:
      hipLaunchKernelGGL(k_assemble<kGeneral>, g2, b2, 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges, c.inc_off,
                         c.inc, c.edge_out, c.nV, half_expo, A);
      break;
  }
  hipLaunchKernelGGL(k_diag_rowsum, dim3(c.nV), dim3(256), 0, s, A, c.nV);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
