// Vertex-pair form of the alpha = 2 tangent-point energy and its differential
// for graphs of vertex degree <= 2 (closed loops and open paths), in FP32.
//
// For alpha = 2 the kernel's numerator is |T_I x d|^2 = |d|^2 - (T_I . d)^2,
// so the trapezoid sum of eq. DiscreteEnergy, regrouped by vertex pair
// (v, w) (v an endpoint of I, w of J), is
//   sum_{I at v} sum_{J at w} 1/4 l_I l_J |T_I x d|^2 |d|^-beta
//     = 1/4 q_v(d) Lambda_w |d|^-beta,
//   q_v(d) = sum_{I at v} l_I |T_I x d|^2 = Lambda_v |d|^2 - sum_{I at v} (u_I . d)^2,
// with d = g_v - g_w, Lambda_v = sum_{I at v} l_I and u_I = sqrt(l_I) T_I,
// exactly whenever every edge at v is disjoint from every edge at w, which
// holds for vertices more than two steps apart along their chain.  Vertex
// pairs at most kBand steps apart (those sharing an edge among them) are
// summed in FP64 by the near-band kernel in the edge-pair form, each of their
// edge pairs with the exact shared-vertex exclusion of Sec. 4.1.
//
// The differential (Sec. 4.1) of the far sum, gathered per target vertex v:
// d enters both ordered vertex pairs (v, w) and (w, v), so with
// p = |d|^-beta, M_v d = Lambda_v d - sum_I u_I (u_I . d) (= grad q_v / 2),
//   grad_{g_v} = 1/4 sum_w [2 p (Lambda_w M_v + Lambda_v M_w) d
//                           - beta p |d|^-2 (Lambda_w q_v + Lambda_v q_w) d],
// which needs, per target, the sums G1 = sum p Lambda_w d, H = sum p (M_w d
// - Lambda_w d) sign-flipped, G3 = sum p |d|^-2 (...) d, and the adjoints of
// the target's own u_I (sum p Lambda_w (u_I . d) d) and Lambda_v
// (sum p (Lambda_w |d|^2 + q_w)); an O(|E|) pass maps the adjoints through
// u_I = e_I / sqrt(l_I) and Lambda to the edge vectors e_I and the vertices.
//
// Per vertex pair that is about 93 FP32 flops and 2 transcendentals (beta =
// 4.5), against 213 executed flops per edge pair in the edge-pair form.

#include <climits>
#include <type_traits>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

static inline int vp_cdiv(int a, int b) { return (a + b - 1) / b; }

// The FP64 near band (vertex pairs at most kBand steps apart along a chain,
// which the FP32 kernel masks) in one launch of two parts: the pairs at
// least kVpMinDist apart in the vertex-pair form (every edge at v is then
// disjoint from every edge at w), kBandLanes lanes per target vertex; the
// pairs closer than that in the edge-pair form with the exact shared-vertex
// exclusion, kNearLanes lanes per target edge.
constexpr int kVpMinDist = 3;
constexpr int kBandLanes = 16;  // a power of two, <= 64
constexpr int kNearLanes = 8;   // a power of two, >= 2 (kVpMinDist - 1) + 3 edges of the window

// Same chain and at most K steps apart (cyclically on a loop).
__device__ __forceinline__ bool vert_near(int4 a, int4 b, int K = kBand) {
  if (a.x != b.x) return false;
  int d = abs(b.y - a.y);
  if (a.w) d = min(d, a.z - d);
  return d <= K;
}

// All ordered vertex pairs (v, w) more than kBand steps apart: a thread owns
// target v, the workgroup's 256 targets sweep the source range of chunk
// blockIdx.y staged in LDS tiles of 256 vertices, FP32 sums folded into FP64
// every kSub sources.  Slots: E, G1 (3), H (3), G3 (3), A0 (3), A1 (3), L,
// written to part[chunk][slot][v] rounded to FP32 (a chunk's sum carries the
// rounding of its FP32 sub-sums already; the chunks are added in FP64).
template <int EC, bool GRAD>
__global__ __launch_bounds__(kTile) void k_vp_pairs(const V4<float>* __restrict__ P, const V4<float>* __restrict__ U0,
                                                    const V4<float>* __restrict__ U1, const int4* __restrict__ vinfo,
                                                    int nV, int src_per_chunk, float half_beta, float beta,
                                                    float* __restrict__ part) {
  __shared__ V4<float> sP[kTile], sU0[kTile], sU1[kTile];
  __shared__ int4 sC[kTile];
  __shared__ int4 sRed[2][kTile / 64];
  __shared__ int2 sChain;
  const int tid = threadIdx.x;
  const int v0 = blockIdx.x * kTile;
  const int v = v0 + tid;
  const bool act = v < nV;
  const int vc = act ? v : v0;
  const V4<float> p = P[vc], a0 = U0[vc], a1 = U1[vc];
  const int4 ci = vinfo[vc];
  wave_range(ci, act, sRed[0]);
  if (tid == 0) sChain = make_int2(ci.z, ci.w);
  constexpr int NS = GRAD ? kVpSlots : 1;
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  const int s0 = blockIdx.y * src_per_chunk, s1 = min(nV, s0 + src_per_chunk);
  const float Lv = p.w;
  for (int t0 = s0; t0 < s1; t0 += kTile) {
    __syncthreads();
    const bool staged = t0 + tid < s1;
    const int4 cj = staged ? vinfo[t0 + tid] : make_int4(-1, 0, 0, 0);
    if (staged) {
      sP[tid] = P[t0 + tid];
      sU0[tid] = U0[t0 + tid];
      sU1[tid] = U1[t0 + tid];
      sC[tid] = cj;
    }
    wave_range(cj, staged, sRed[1]);
    __syncthreads();
    const int cnt = min(kTile, s1 - t0);
    // pairs are tested (and masked) one by one only where the tiles' chain
    // ranges cannot rule out a near pair
    const bool test = !tiles_far(range_of(sRed[0]), range_of(sRed[1]), sChain.x, sChain.y);
    for (int u0 = 0; u0 < cnt; u0 += kSub) {
      const int u1 = min(cnt, u0 + kSub);
      float E = 0.f, G1x = 0.f, G1y = 0.f, G1z = 0.f, Hx = 0.f, Hy = 0.f, Hz = 0.f, G3x = 0.f, G3y = 0.f,
            G3z = 0.f, A0x = 0.f, A0y = 0.f, A0z = 0.f, A1x = 0.f, A1y = 0.f, A1z = 0.f, L = 0.f;
      auto sweep = [&](auto tested) {
        for (int u = u0; u < u1; ++u) {
          const V4<float> q = sP[u], w0 = sU0[u], w1 = sU1[u];
          const float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
          float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
          bool skip = false;
          if constexpr (decltype(tested)::value) {
            skip = vert_near(ci, sC[u]);
            r2 = skip ? r2 + 1.f : r2;  // a masked pair (the target itself included) stays finite
          }
          const float tav = fmaf(a0.x, dx, fmaf(a0.y, dy, a0.z * dz));
          const float tbv = fmaf(a1.x, dx, fmaf(a1.y, dy, a1.z * dz));
          const float qv = fmaf(-tav, tav, fmaf(-tbv, tbv, Lv * r2));
          float ri, pb;
          tpe_powers<EC, float>(r2, half_beta, ri, pb);
          if constexpr (decltype(tested)::value) pb = skip ? 0.f : pb;
          const float a = pb * q.w;
          E = fmaf(a, qv, E);
          if constexpr (GRAD) {
            const float taw = fmaf(w0.x, dx, fmaf(w0.y, dy, w0.z * dz));
            const float tbw = fmaf(w1.x, dx, fmaf(w1.y, dy, w1.z * dz));
            const float qw = fmaf(-taw, taw, fmaf(-tbw, tbw, q.w * r2));
            G1x = fmaf(a, dx, G1x);
            G1y = fmaf(a, dy, G1y);
            G1z = fmaf(a, dz, G1z);
            const float b0 = pb * taw, b1 = pb * tbw;
            Hx = fmaf(b0, w0.x, fmaf(b1, w1.x, Hx));
            Hy = fmaf(b0, w0.y, fmaf(b1, w1.y, Hy));
            Hz = fmaf(b0, w0.z, fmaf(b1, w1.z, Hz));
            const float c = (pb * ri) * fmaf(q.w, qv, Lv * qw);
            G3x = fmaf(c, dx, G3x);
            G3y = fmaf(c, dy, G3y);
            G3z = fmaf(c, dz, G3z);
            const float e0 = a * tav, e1 = a * tbv;
            A0x = fmaf(e0, dx, A0x);
            A0y = fmaf(e0, dy, A0y);
            A0z = fmaf(e0, dz, A0z);
            A1x = fmaf(e1, dx, A1x);
            A1y = fmaf(e1, dy, A1y);
            A1z = fmaf(e1, dz, A1z);
            L = fmaf(pb, fmaf(q.w, r2, qw), L);
          }
        }
      };
      if (test) sweep(std::true_type{});
      else sweep(std::false_type{});
      acc[0] += (double)E;
      if constexpr (GRAD) {
        acc[1] += (double)G1x; acc[2] += (double)G1y; acc[3] += (double)G1z;
        acc[4] += (double)Hx; acc[5] += (double)Hy; acc[6] += (double)Hz;
        acc[7] += (double)G3x; acc[8] += (double)G3y; acc[9] += (double)G3z;
        acc[10] += (double)A0x; acc[11] += (double)A0y; acc[12] += (double)A0z;
        acc[13] += (double)A1x; acc[14] += (double)A1y; acc[15] += (double)A1z;
        acc[16] += (double)L;
      }
    }
  }
  if (act) {
    float* out = part + (size_t)blockIdx.y * NS * nV + v;
#pragma unroll
    for (int k = 0; k < NS; ++k) out[(size_t)k * nV] = (float)acc[k];
  }
}

// Near band, edge-pair part: for target edge I, every edge J of its chain at
// most KB + 1 steps away, in the edge-pair form with the exact shared-vertex
// exclusion, keeping only the vertex pairs at most KB steps apart.  LANES
// lanes per target edge (tg: the thread's index in this part), summed across
// the lanes by a fixed butterfly; writes the edge's record to edge_out
// (tpe_edge_record), to which the vertex sums are added later.
template <int EC, bool GRAD, int KB, int LANES>
__device__ __forceinline__ void near_edge_pairs(int tg, const V4<double>* __restrict__ GA,
                                                const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                                                const int4* __restrict__ cinfo, const int* __restrict__ chain_edge,
                                                const int4* __restrict__ vinfo, int nE, double half_beta,
                                                double beta, double* __restrict__ edge_out,
                                                unsigned* __restrict__ status) {
  const int I = tg / LANES, sub = tg % LANES;
  const bool valid = I < nE;
  double E = 0, S = 0, G1x = 0, G1y = 0, G1z = 0, G2x = 0, G2y = 0, G2z = 0;
  double Gt1 = 0, Gt2 = 0, Hx = 0, Hy = 0, Hz = 0;
  V4<double> a{0, 0, 0, 0}, t{0, 0, 0, 0};
  if (valid) {
    a = GA[I];
    t = GT[I];
    const int2 ei = edges[I];
    const int4 ci = cinfo[I];
    const int4 va = vinfo[ei.x], vb = vinfo[ei.y];
    const int m = ci.z;
    constexpr int W = KB + 1;
    int q0, q1;
    if (ci.w && m <= 2 * W + 1) {
      q0 = 0;
      q1 = m - 1;
    } else if (ci.w) {
      q0 = ci.y - W;
      q1 = ci.y + W;
    } else {
      q0 = max(0, ci.y - W);
      q1 = min(m - 1, ci.y + W);
    }
    for (int q = q0 + sub; q <= q1; q += LANES) {
      const int qq = ((q % m) + m) % m;
      const int J = chain_edge[ci.x + qq];
      const int2 ej = edges[J];
      const bool skip = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
      const int4 vc = vinfo[ej.x], ve = vinfo[ej.y];
      const int m4 = (vert_near(va, vc, KB) ? 1 : 0) | (vert_near(va, ve, KB) ? 2 : 0) |
                     (vert_near(vb, vc, KB) ? 4 : 0) | (vert_near(vb, ve, KB) ? 8 : 0);
      const V4<double> qa = GA[J], qt = GT[J];
      tpe_edge_pair<double, EC, GRAD, true, true>(a.x, a.y, a.z, t.x, t.y, t.z, a.w, qa.x, qa.y, qa.z, qt.x, qt.y,
                                                  qt.z, qa.w, skip ? 0.0 : 0.25 * qa.w, skip ? 1.0 : 0.0, 1.0,
                                                  half_beta, beta, E, S, G1x, G1y, G1z, Gt1, G2x, G2y, G2z, Gt2, Hx,
                                                  Hy, Hz, m4);
    }
  }
  auto red = [](double v) {  // butterfly over the group: the same sum, in the same order, on every lane
#pragma unroll
    for (int o = 1; o < LANES; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
  };
  constexpr int NS = GRAD ? kTpeSlots : 1;
  double v[kTpeSlots] = {E, S, G1x, G1y, G1z, G2x, G2y, G2z, Gt1, Gt2, Hx, Hy, Hz, 0.0};
#pragma unroll
  for (int k = 0; k < NS; ++k) v[k] = red(v[k]);
  if (GRAD) v[13] = t.x * v[10] + t.y * v[11] + t.z * v[12];  // T.H: H holds multiples of T
  if (!valid || sub != 0) return;
  tpe_edge_record(v, GRAD, a.w, t.x, t.y, t.z, edge_out + 8 * (size_t)I, status);
}

// Near band, vertex-pair part: for target vertex v, the vertices w of its
// chain with kVpMinDist <= distance <= kBand, in FP64 with the sums of
// k_vp_pairs (the same slots and arithmetic).  kBandLanes lanes per target
// vertex (tg: the thread's index in this part), summed across the lanes by
// a fixed butterfly; written to vband[slot][v] (zeros for a vertex without
// such pairs).
template <int EC, bool GRAD>
__device__ __forceinline__ void near_vertex_pairs(int tg, const V4<double>* __restrict__ P,
                                                  const V4<double>* __restrict__ U0,
                                                  const V4<double>* __restrict__ U1, const int4* __restrict__ vinfo,
                                                  const int* __restrict__ vchain, int nV, double half_beta,
                                                  double* __restrict__ vband) {
  const int v = tg / kBandLanes, sub = tg % kBandLanes;
  const bool valid = v < nV;
  constexpr int NS = GRAD ? kVpSlots : 1;
  double acc[kVpSlots];
#pragma unroll
  for (int k = 0; k < kVpSlots; ++k) acc[k] = 0.0;
  if (valid) {
    const int4 ci = vinfo[v];
    const int m = ci.z, pos = ci.y;
    int q0 = 0, n = 0;  // candidate positions q0 + j, j < n (mod m on a loop)
    if (ci.x < 0) n = 0;  // isolated vertex
    else if (ci.w && m <= 2 * kBand + 1) n = m;
    else if (ci.w) {
      q0 = pos - kBand;
      n = 2 * kBand + 1;
    } else {
      q0 = max(0, pos - kBand);
      n = min(m - 1, pos + kBand) - q0 + 1;
    }
    const V4<double> p = P[v], a0 = U0[v], a1 = U1[v];
    const double Lv = p.w;
    for (int j = sub; j < n; j += kBandLanes) {
      int q = q0 + j;
      if (ci.w) q = ((q % m) + m) % m;
      int dist = abs(q - pos);
      if (ci.w) dist = min(dist, m - dist);
      if (dist < kVpMinDist || dist > kBand) continue;
      const int w = vchain[ci.x + q];
      const V4<double> qp = P[w], w0 = U0[w], w1 = U1[w];
      const double dx = p.x - qp.x, dy = p.y - qp.y, dz = p.z - qp.z;
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double tav = fma(a0.x, dx, fma(a0.y, dy, a0.z * dz));
      const double tbv = fma(a1.x, dx, fma(a1.y, dy, a1.z * dz));
      const double qv = fma(-tav, tav, fma(-tbv, tbv, Lv * r2));
      double ri, pb;
      tpe_powers<EC, double>(r2, half_beta, ri, pb);
      const double a = pb * qp.w;
      acc[0] = fma(a, qv, acc[0]);
      if constexpr (GRAD) {
        const double taw = fma(w0.x, dx, fma(w0.y, dy, w0.z * dz));
        const double tbw = fma(w1.x, dx, fma(w1.y, dy, w1.z * dz));
        const double qw = fma(-taw, taw, fma(-tbw, tbw, qp.w * r2));
        acc[1] = fma(a, dx, acc[1]);
        acc[2] = fma(a, dy, acc[2]);
        acc[3] = fma(a, dz, acc[3]);
        const double b0 = pb * taw, b1 = pb * tbw;
        acc[4] = fma(b0, w0.x, fma(b1, w1.x, acc[4]));
        acc[5] = fma(b0, w0.y, fma(b1, w1.y, acc[5]));
        acc[6] = fma(b0, w0.z, fma(b1, w1.z, acc[6]));
        const double c = (pb * ri) * fma(qp.w, qv, Lv * qw);
        acc[7] = fma(c, dx, acc[7]);
        acc[8] = fma(c, dy, acc[8]);
        acc[9] = fma(c, dz, acc[9]);
        const double e0 = a * tav, e1 = a * tbv;
        acc[10] = fma(e0, dx, acc[10]);
        acc[11] = fma(e0, dy, acc[11]);
        acc[12] = fma(e0, dz, acc[12]);
        acc[13] = fma(e1, dx, acc[13]);
        acc[14] = fma(e1, dy, acc[14]);
        acc[15] = fma(e1, dz, acc[15]);
        acc[16] = fma(pb, fma(qp.w, r2, qw), acc[16]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int o = 1; o < kBandLanes; o <<= 1) acc[k] += __shfl_xor(acc[k], o, 64);
  if (!valid || sub != 0) return;
#pragma unroll
  for (int k = 0; k < NS; ++k) vband[(size_t)k * nV + v] = acc[k];
}

// The near band in one launch: workgroups [0, nbv) take the vertex-pair part,
// the rest the edge-pair part.
template <int EC, bool GRAD>
__global__ __launch_bounds__(256) void k_vp_near(const V4<double>* __restrict__ P, const V4<double>* __restrict__ U0,
                                                 const V4<double>* __restrict__ U1, const int* __restrict__ vchain,
                                                 int nV, int nbv, const V4<double>* __restrict__ GA,
                                                 const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                                                 const int4* __restrict__ cinfo, const int* __restrict__ chain_edge,
                                                 const int4* __restrict__ vinfo, int nE, double half_beta,
                                                 double beta, double* __restrict__ vband,
                                                 double* __restrict__ edge_out, unsigned* __restrict__ status) {
  if ((int)blockIdx.x < nbv)  // uniform over the workgroup
    near_vertex_pairs<EC, GRAD>(blockIdx.x * 256 + threadIdx.x, P, U0, U1, vinfo, vchain, nV, half_beta, vband);
  else
    near_edge_pairs<EC, GRAD, kVpMinDist - 1, kNearLanes>((blockIdx.x - nbv) * 256 + threadIdx.x, GA, GT, edges,
                                                          cinfo, chain_edge, vinfo, nE, half_beta, beta, edge_out,
                                                          status);
}

// FP64 u_I (the vertex's incident edges in incidence order) and Lambda_v.
__device__ __forceinline__ double vertex_u(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GT,
                                           const int* __restrict__ inc_off, const int* __restrict__ inc, int v,
                                           double (&u)[2][3]) {
  double lam = 0.0;
  const int k0 = inc_off[v], k1 = min(inc_off[v + 1], k0 + 2);
  for (int j = 0; j < 2; ++j) u[j][0] = u[j][1] = u[j][2] = 0.0;
  for (int k = k0; k < k1; ++k) {
    const int I = inc[k] >> 1;
    const V4<double> a = GA[I], t = GT[I];
    const double sl = sqrt(a.w);
    lam += a.w;
    u[k - k0][0] = sl * t.x;
    u[k - k0][1] = sl * t.y;
    u[k - k0][2] = sl * t.z;
  }
  return lam;
}

// Per vertex: sums the chunks and the FP64 near band and writes
// vout[v] = (E_v, direct gradient (3), dE/du_0 (3), dE/du_1 (3), dE/dLambda_v, 0).
// A thread per (slot, vertex) adds the slot's chunk partials in chunk order in
// FP64 (eight loads in flight; kVpSumV consecutive vertices make one 128-byte
// line per slot and chunk), then one thread per vertex finishes from LDS.
constexpr int kVpSumV = 32;
__global__ __launch_bounds__(kVpSumV* kVpSlots) void k_vp_sum(const float* __restrict__ part,
                                                              const double* __restrict__ vband, int nchunk, int NS,
                                                              int nV, double beta, const V4<double>* __restrict__ GA,
                                                              const V4<double>* __restrict__ GT,
                                                              const int* __restrict__ inc_off,
                                                              const int* __restrict__ inc, double* __restrict__ vout,
                                                              unsigned* __restrict__ status) {
  __shared__ double sm[kVpSlots][kVpSumV];
  const int j = threadIdx.x % kVpSumV, k = threadIdx.x / kVpSumV;  // k < NS (blockDim = kVpSumV NS)
  const int v = blockIdx.x * kVpSumV + j;
  if (v < nV) {
    const size_t stride = (size_t)NS * nV;
    const float* p = part + (size_t)k * nV + v;
    double a = 0.0;
    int c = 0;
    for (; c + 8 <= nchunk; c += 8) {
      float t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = p[(size_t)(c + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += (double)t[u];
    }
    for (; c < nchunk; ++c) a += (double)p[(size_t)c * stride];
    sm[k][j] = a + vband[(size_t)k * nV + v];  // then the FP64 near band
  }
  __syncthreads();
  if (k != 0 || v >= nV) return;
  const bool grad = NS > 1;
  double s[kVpSlots];
  bool fin = true;
#pragma unroll
  for (int q = 0; q < kVpSlots; ++q) {
    s[q] = q < NS ? sm[q][j] : 0.0;
    fin &= isfinite(s[q]);
  }
  if (!fin) latch(status, kFlagPairOverflow);
  double* o = vout + (size_t)kVpOut * v;
  o[0] = 0.25 * s[0];
  if (!grad) return;
  double u[2][3];
  const double lam = vertex_u(GA, GT, inc_off, inc, v, u);
  const double G1[3] = {s[1], s[2], s[3]}, H[3] = {s[4], s[5], s[6]}, G3[3] = {s[7], s[8], s[9]};
  const double c0 = u[0][0] * G1[0] + u[0][1] * G1[1] + u[0][2] * G1[2];
  const double c1 = u[1][0] * G1[0] + u[1][1] * G1[1] + u[1][2] * G1[2];
  for (int q = 0; q < 3; ++q) {
    const double MG1 = lam * G1[q] - u[0][q] * c0 - u[1][q] * c1;
    o[1 + q] = 0.25 * (2.0 * MG1 + 2.0 * lam * (G1[q] - H[q]) - beta * G3[q]);
    o[4 + q] = -0.5 * s[10 + q];
    o[7 + q] = -0.5 * s[13 + q];
  }
  o[10] = 0.25 * s[16];
  o[11] = 0.0;
}

// Per edge I = (i1, i2): adds to the edge's record (already holding its near
// band) the vertex energies it carries (each vertex's energy goes to the edge
// in its first incidence slot) and, with the differential, the partial of
// the vertex sums through e_I = g_i2 - g_i1: u_I = e_I / sqrt(l_I) enters
// as a u of both endpoints, l_I as a term of both Lambdas, so
//   dE/de_I = (I - T T^T / 2) (g_u(i1) + g_u(i2)) / sqrt(l_I) + (g_Lambda(i1) + g_Lambda(i2)) T.
// Returns the edge's energy.
__device__ __forceinline__ double vp_edge_one(const double* __restrict__ vout, const int2* __restrict__ edges,
                                              const int* __restrict__ inc_off, const int* __restrict__ inc,
                                              const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GT,
                                              int I, bool grad, double* __restrict__ edge_out) {
  const int2 e = edges[I];
  const int k1 = (inc[inc_off[e.x]] >> 1) == I ? 0 : 1;
  const int k2 = (inc[inc_off[e.y]] >> 1) == I ? 0 : 1;
  const double* o1 = vout + (size_t)kVpOut * e.x;
  const double* o2 = vout + (size_t)kVpOut * e.y;
  double* o = edge_out + 8 * (size_t)I;
  const double E = o[0] + ((k1 == 0 ? o1[0] : 0.0) + (k2 == 0 ? o2[0] : 0.0));
  o[0] = E;
  if (!grad) return E;
  const V4<double> a = GA[I], t = GT[I];
  double gu[3];
  for (int k = 0; k < 3; ++k) gu[k] = o1[4 + 3 * k1 + k] + o2[4 + 3 * k2 + k];
  const double gl = o1[10] + o2[10];
  const double tg = t.x * gu[0] + t.y * gu[1] + t.z * gu[2];
  const double isl = 1.0 / sqrt(a.w);
  const double de[3] = {(gu[0] - 0.5 * tg * t.x) * isl + gl * t.x, (gu[1] - 0.5 * tg * t.y) * isl + gl * t.y,
                        (gu[2] - 0.5 * tg * t.z) * isl + gl * t.z};
  for (int k = 0; k < 3; ++k) {
    o[1 + k] -= de[k];
    o[4 + k] += de[k];
  }
  return E;
}

// vp_edge_one over the edges, a grid-stride loop; with partial set, also the
// workgroup sums of the edge energies (the first pass of the fixed-order
// total energy: partial[b] = sum of the energies of the edges b 256 + t +
// k gridDim 256, by thread, then a tree over the 256 threads).
__global__ __launch_bounds__(256) void k_vp_edge(const double* __restrict__ vout, const int2* __restrict__ edges,
                                                 const int* __restrict__ inc_off, const int* __restrict__ inc,
                                                 const V4<double>* __restrict__ GA,
                                                 const V4<double>* __restrict__ GT, int nE, int grad,
                                                 double* __restrict__ edge_out, double* __restrict__ partial) {
  __shared__ double sm[256];
  double acc = 0.0;
  for (int I = blockIdx.x * 256 + threadIdx.x; I < nE; I += gridDim.x * 256)
    acc += vp_edge_one(vout, edges, inc_off, inc, GA, GT, I, grad != 0, edge_out);
  if (!partial) return;
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

// dE_v = the direct vertex gradient plus the endpoint partials of the edges at v.
__global__ void k_vp_gather(const double* __restrict__ vout, const double* __restrict__ edge_out,
                            const int* __restrict__ inc_off, const int* __restrict__ inc, int nV,
                            double* __restrict__ dE, unsigned* __restrict__ status) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  const double* ov = vout + (size_t)kVpOut * v;
  double gx = ov[1], gy = ov[2], gz = ov[3];
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int code = inc[k];
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

template <int EC, bool GRAD>
static void run_vp(const Curve& c, double beta, hipStream_t s) {
  const bool timed = GRAD && c.timer && c.timer->on;
  if (timed) c.timer->mark(c.timer->tpe, s);
  hipLaunchKernelGGL((k_vp_pairs<EC, GRAD>), dim3(vp_cdiv(c.nV, kTile), c.vchunk), dim3(kTile), 0, s,
                     (const V4<float>*)c.vg[0], (const V4<float>*)c.vg[1], (const V4<float>*)c.vg[2],
                     (const int4*)c.vinfo, c.nV, c.vsrc_per_chunk, (float)(0.5 * beta), (float)beta, c.vpart);
  if (timed) c.timer->mark(c.timer->tpe, s);
  const int nbv = vp_cdiv(c.nV, 256 / kBandLanes), nbe = vp_cdiv(c.nE, 256 / kNearLanes);
  hipLaunchKernelGGL((k_vp_near<EC, GRAD>), dim3(nbv + nbe), dim3(256), 0, s, (const V4<double>*)c.vgd[0],
                     (const V4<double>*)c.vgd[1], (const V4<double>*)c.vgd[2], (const int*)c.vchain, c.nV, nbv,
                     (const V4<double>*)c.gd.a, (const V4<double>*)c.gd.t, (const int2*)c.edges,
                     (const int4*)c.cinfo, (const int*)c.chain_edge, (const int4*)c.vinfo, c.nE, 0.5 * beta, beta,
                     c.vband, c.edge_out, c.status);
}

rc_status launch_tpe_vp_pairs(const Curve& c, double beta, bool grad, hipStream_t s) {
  switch (exp_case(2.0, beta)) {
    case kA2B4:
      if (grad) run_vp<kA2B4, true>(c, beta, s);
      else run_vp<kA2B4, false>(c, beta, s);
      break;
    case kA2B45:
      if (grad) run_vp<kA2B45, true>(c, beta, s);
      else run_vp<kA2B45, false>(c, beta, s);
      break;
    default:
      if (grad) run_vp<kGeneral, true>(c, beta, s);
      else run_vp<kGeneral, false>(c, beta, s);
      break;
  }
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_tpe_vp_finish(const Curve& c, double beta, bool grad, double* dE, double* energy_partial,
                               hipStream_t s) {
  const int NS = grad ? kVpSlots : 1;
  hipLaunchKernelGGL(k_vp_sum, dim3(vp_cdiv(c.nV, kVpSumV)), dim3(kVpSumV * NS), 0, s, (const float*)c.vpart,
                     (const double*)c.vband, c.vchunk, NS, c.nV, beta, (const V4<double>*)c.gd.a, (const V4<double>*)c.gd.t,
                     (const int*)c.inc_off, (const int*)c.inc, c.vout, c.status);
  hipLaunchKernelGGL(k_vp_edge, dim3(c.red_blocks), dim3(256), 0, s, (const double*)c.vout, (const int2*)c.edges,
                     (const int*)c.inc_off, (const int*)c.inc, (const V4<double>*)c.gd.a, (const V4<double>*)c.gd.t,
                     c.nE, grad ? 1 : 0, c.edge_out, energy_partial);
  RC_TRY(launch_penalties(c, grad, s));
  if (grad && dE)
    hipLaunchKernelGGL(k_vp_gather, dim3(vp_cdiv(c.nV, 256)), dim3(256), 0, s, (const double*)c.vout,
                       (const double*)c.edge_out, (const int*)c.inc_off, (const int*)c.inc, c.nV, dE, c.status);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
