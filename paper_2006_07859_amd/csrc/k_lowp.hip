// Assembled Sobolev block in 16-bit storage and its product with the three
// coordinate columns on the matrix cores.
//
// The block is A = B + B0 (Sec. 4.2.2-4.2.3) on a curve whose vertices have
// degree <= 2.  Entry (v, w), v != w, is the sum over disjoint edges I at v
// and J at w of
//     -1/2 s_I(v) s_J(w) rho_IJ <T_I, T_J>  -  l_I l_J rho0_IJ / 16
// (rho_IJ: the sum over the four vertex pairs of |d|^-(2 sigma + 1); rho0_IJ
// the same weighted by the low-order kernel k_{2,4} with T_I and with T_J),
// plus, when v and w are the two ends of an edge K,
//     -Wq_K / (2 l_K) + l_K P0_K / 16,
// with s(i1) = -1, s(i2) = +1 and Wq, P0 the per-edge sums of the operator
// kernel.  diag(A) = d_v = sum over edges I at v of Wq_I / (2 l_I) + l_I P0_I / 16.
//
// Storage: S = D^-1/2 A D^-1/2 (D = diag d) has unit diagonal and
// off-diagonal entries in [-1, 1], so it fits FP16 and BF16.  Entries whose
// vertices lie at most `band` steps apart along a chain are computed in FP64
// and kept in FP32 (2 band values per row); every other off-diagonal entry
// is computed in FP32 (from FP64 coordinate differences) and rounded to 16
// bits.  The diagonal is not stored:
// it is recomputed from the stored values as
//     sigma_v = -sum_{w != v} S^_vw sqrt(d_w) / sqrt(d_v)      (FP64 sums)
// so that the stored operator
//     A^ = D^1/2 (S^_off + diag sigma) D^1/2
// annihilates constants exactly as A does.
//
// Tile layout: the off-diagonal part is cut into tiles of 16 rows x 32
// columns, held in the operand order of v_mfma_f32_16x16x32_{bf16,f16}: lane
// l of a wave holds row l % 16, columns 8 (l / 16) .. 8 (l / 16) + 7 as one
// 16-byte vector, and a tile is those 64 vectors in lane order (1 KB).  Tiles
// of one row block are consecutive in column order.
//
// Product Y = A^ X for X in R^{n x 3}, in difference form (see the product
// section below): the B operand holds sqrt(d_w) (x_w - c) for a reference c
// near the rows, for FP16 scaled by a power of two into [-1, 1] (BF16 keeps
// FP32's exponent range and needs no scaling), and split
// into hi + lo 16-bit parts in columns 0-2 and 3-5, so one MFMA per A tile
// gives both halves; the FP32 accumulators of the two halves are added, the
// band and diagonal terms are applied in FP64, and the result is scaled back
// and by D^1/2 in FP64.  The product streams the tiles once and is bound by
// HBM bandwidth.
//
// The same pass can also keep every entry in FP32 (tiles of 16 x 32 floats,
// lane l holding row l % 16, columns 8 (l / 16) .. + 7), with its own
// recomputed diagonal; its product uses v_mfma_f32_16x16x4f32.  Rounding the
// far field to 16 bits perturbs the smooth eigenvectors of A by much more than
// their small eigenvalues once the curve is fine, so the 16-bit block serves
// the multigrid smoothers and the FP32 block the Krylov recurrence.

#include <algorithm>
#include <type_traits>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef f16x8 type; };

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(f16x8 a, f16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Canonical signed offset of w from v along their chain, or a value above
// any band when they are on different chains.  vinfo = (chain, position,
// vertex count, is loop); on a loop of m vertices the offset lies in
// (-m/2, m/2].
__device__ __forceinline__ int chain_offset(int4 a, int4 b) {
  if (a.x != b.x) return 1 << 30;
  int d = b.y - a.y;
  if (a.w) {
    const int m = a.z;
    d %= m;
    if (d < 0) d += m;
    if (2 * d > m) d -= m;
  }
  return d;
}

// d_v and sqrt(d_v) from the FP64 per-edge sums.
__global__ void k_lowp_dvec(const double* __restrict__ edge_out, const V4<double>* __restrict__ GA,
                            const int* __restrict__ inc_off, const int* __restrict__ inc, int n,
                            double* __restrict__ dvec, double* __restrict__ sqd) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double d = 0.0;
  for (int k = inc_off[v]; k < inc_off[v + 1]; ++k) {
    const int I = inc[k] >> 1;
    const double l = GA[I].w;
    d += edge_out[8 * (size_t)I] / (2.0 * l) + l * edge_out[8 * (size_t)I + 1] / 16.0;
  }
  dvec[v] = d;
  sqd[v] = d > 0.0 ? sqrt(d) : 1.0;
}

// Tiles: one thread per lane vector (8 entries of one row); a workgroup
// builds four consecutive column tiles of one row block, so its stores are
// contiguous.  grid = (row blocks, groups of 4 column tiles).  Each entry is
// evaluated once in FP32 and stored rounded to T and, when W32, also as the
// FP32 value itself.  rowpart / rowpart32 [group][v] get the FP64 sums over
// the group's columns of S^_vw sqrt(d_w) for the two stored versions.
template <typename T, int EC, bool W32>
__global__ __launch_bounds__(256) void k_assemble_lowp(
    const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB, const V4<double>* __restrict__ GT,
    const int2* __restrict__ edges, const int* __restrict__ inc_off, const int* __restrict__ inc,
    const double* __restrict__ edge_out, const double* __restrict__ sqd, const int4* __restrict__ vinfo, int band,
    int n, int nkt, float half_expo, typename Vec8<T>::type* __restrict__ tiles, float4* __restrict__ tiles32,
    double* __restrict__ rowpart, double* __restrict__ rowpart32) {
  __shared__ double part[2][256];
  const int rb = blockIdx.x;
  const int t = threadIdx.x / 64, l = threadIdx.x % 64;
  const int kt = blockIdx.y * 4 + t;
  const int v = rb * 16 + (l % 16);
  double rs = 0.0, rs32 = 0.0;
  if (kt < nkt) {
    typename Vec8<T>::type vec;
    float f[8];
    const bool vok = v < n;
    const double sv = vok ? sqd[v] : 1.0;
    const int4 iv = vok ? vinfo[v] : make_int4(-1, 0, 1, 0);
    const int w0 = kt * 32 + 8 * (l / 16);
#pragma unroll 1
    for (int j = 0; j < 8; ++j) {
      const int w = w0 + j;
      float sf = 0.f;
      if (vok && w < n && w != v) {
        const int off = chain_offset(iv, vinfo[w]);
        if (off < -band || off > band) {
          // evaluated with the smaller index first, so that S^ is exactly symmetric
          const float a = sobolev_entry<float, EC>(min(v, w), max(v, w), GA, GB, GT, edges, inc_off, inc, edge_out,
                                                half_expo);
          const double sw = sqd[w];
          sf = (float)((double)a / (sv * sw));
          const T r = (T)sf;
          rs += (double)(float)r * sw;
          rs32 += (double)sf * sw;
        }
      }
      vec[j] = (T)sf;
      f[j] = sf;
    }
    const size_t tile = (size_t)rb * nkt + kt;
    tiles[tile * 64 + l] = vec;
    if (W32) {
      tiles32[tile * 128 + l] = make_float4(f[0], f[1], f[2], f[3]);
      tiles32[tile * 128 + 64 + l] = make_float4(f[4], f[5], f[6], f[7]);
    }
  }
  part[0][threadIdx.x] = rs;
  part[1][threadIdx.x] = rs32;
  __syncthreads();
  if (threadIdx.x < 16) {
    // row threadIdx.x appears in lanes threadIdx.x + 16 g (g < 4) of each of the 4 tiles
    double a16 = 0.0, a32 = 0.0;
    for (int q = 0; q < 16; ++q) {
      a16 += part[0][q * 16 + threadIdx.x];
      a32 += part[1][q * 16 + threadIdx.x];
    }
    const int vv = rb * 16 + threadIdx.x;
    if (vv < n) {
      rowpart[(size_t)blockIdx.y * n + vv] = a16;
      if (W32) rowpart32[(size_t)blockIdx.y * n + vv] = a32;
    }
  }
}

// The same tiles for curves (vertex degree <= 2) from edge pairs: an entry
// S^_vw sums over the edges I at v and J at w, and each edge pair serves up
// to four entries, so the workgroup evaluates every distinct (row edge,
// column edge) pair of a 16 x 32 tile once into LDS, forms the 512 entries
// from the table, and the owning wave stores its lane vectors.  A vertex's
// incident edge is a repeat within the tile when its other end is an earlier
// vertex of the same tile, so the distinct edges are found by one ballot; the
// edges' geometry and the vertices' data are staged in LDS.  The pair terms
// are evaluated with the smaller edge first and an entry sums its terms with
// the smaller vertex's edges outermost, so that S^ is exactly symmetric.
// Column tiles per workgroup of the edge-pair assembly (the row side is set up once for them).
constexpr int kEpTiles = 8;

struct EpEdge {
  double a[3], b[3];  // end points
  float t[3], l;      // unit tangent, length
  float dg;           // the term of an entry whose two vertices are the ends of this edge
};

template <typename T, int EC, bool W32>
__global__ __launch_bounds__(256) void k_assemble_lowp_ep(
    const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB, const V4<double>* __restrict__ GT,
    const int2* __restrict__ edges, const int* __restrict__ inc_off, const int* __restrict__ inc,
    const double* __restrict__ edge_out, const double* __restrict__ sqd, const int4* __restrict__ vinfo, int band,
    int n, int nkt, float half_expo, typename Vec8<T>::type* __restrict__ tiles, float4* __restrict__ tiles32,
    double* __restrict__ rowpart, double* __restrict__ rowpart32) {
  __shared__ int sE[2][32][2];      // [rows / columns][vertex][slot] incident edge, -1: none
  __shared__ float sS[2][32][2];    // its sign s(v)
  __shared__ int sI[2][32][2];      // index in the distinct list
  __shared__ int slist[2][64], nlist[2];
  __shared__ EpEdge ed[2][64];      // distinct row / column edges
  __shared__ int4 vi[2][32];        // vinfo of the row / column vertices
  __shared__ double sq[2][32];      // sqrt(d) of the row / column vertices
  __shared__ float G[32][65], H[32][65];  // pair terms rho T_I.T_J and l_I l_J rho0
  __shared__ float E[16][33];             // the tile's entries
  __shared__ double part[2][256];
  const int rb = blockIdx.x, t = threadIdx.x, wave = t / 64, l = t % 64;
  // slots of the side's nv vertices from v0 (threads 0 .. 2 nv - 1 of wave 0), distinct edges by ballot
  auto side_setup = [&](int sd, int v0, int nv) {
    int e = -1, u = -1;
    float sg = 0.f;
    const int vl = l / 2, sl = l % 2, v = v0 + vl;
    if (wave == 0 && l < 2 * nv && v < n) {
      const int kk = inc_off[v] + sl;
      if (kk < inc_off[v + 1]) {
        e = inc[kk] >> 1;
        sg = (inc[kk] & 1) ? 1.f : -1.f;
        const int2 ev = edges[e];
        u = ev.x == v ? ev.y : ev.x;  // the edge's other end
      }
    }
    if (wave == 0) {
      const bool fresh = e >= 0 && !(u >= v0 && u < v);
      const unsigned long long bal = __ballot(fresh);
      const int idx = __popcll(bal & ((1ull << l) - 1ull));
      if (l < 2 * nv) {
        sE[sd][vl][sl] = e;
        sS[sd][vl][sl] = sg;
        sI[sd][vl][sl] = fresh ? idx : -1;
      }
      if (fresh) slist[sd][idx] = e;
      if (l == 0) nlist[sd] = __popcll(bal);
    }
    __syncthreads();
    if (wave == 0 && l < 2 * nv && e >= 0 && sI[sd][vl][sl] < 0) {  // a repeat takes the index at its other end
      const int ul = u - v0;
      sI[sd][vl][sl] = sE[sd][ul][0] == e ? sI[sd][ul][0] : sI[sd][ul][1];
    }
    if (t < nlist[sd]) {
      const int I = slist[sd][t];
      const V4<double> ga = GA[I], gb = GB[I], gt = GT[I];
      EpEdge x;
      x.a[0] = ga.x; x.a[1] = ga.y; x.a[2] = ga.z;
      x.b[0] = gb.x; x.b[1] = gb.y; x.b[2] = gb.z;
      x.t[0] = (float)gt.x; x.t[1] = (float)gt.y; x.t[2] = (float)gt.z;
      x.l = (float)ga.w;
      const double* o = edge_out + 8 * (size_t)I;  // (Wq, P0) in slots 0, 1
      x.dg = (float)(-o[0] / (2.0 * ga.w) + ga.w * o[1] / 16.0);
      ed[sd][t] = x;
    }
    if (t >= 128 && t < 128 + nv) {
      const int v2 = v0 + (t - 128);
      vi[sd][t - 128] = v2 < n ? vinfo[v2] : make_int4(-1, 0, 1, 0);
      sq[sd][t - 128] = v2 < n ? sqd[v2] : 1.0;
    }
    __syncthreads();
  };
  side_setup(0, rb * 16, 16);
  const int nr = nlist[0];
  double rs = 0.0, rs32 = 0.0;
  for (int q = 0; q < kEpTiles; ++q) {
    const int kt = blockIdx.y * kEpTiles + q;
    if (kt >= nkt) break;  // uniform
    side_setup(1, kt * 32, 32);
    const int nc = nlist[1];
    for (int p = t; p < nr * nc; p += 256) {
      const int a = p / nc, b = p % nc;
      const int I = slist[0][a], J = slist[1][b];
      float g = 0.f, h = 0.f;
      const int2 ei = edges[I], ej = edges[J];
      if (I != J && ei.x != ej.x && ei.x != ej.y && ei.y != ej.x && ei.y != ej.y) {
        const EpEdge& X = I < J ? ed[0][a] : ed[1][b];  // the smaller edge first
        const EpEdge& Y = I < J ? ed[1][b] : ed[0][a];
        // differences taken in FP64, then rounded
        float rho, rho0;
        sob_edge_pair_d<float, EC, false>(
            (float)(X.a[0] - Y.a[0]), (float)(X.a[1] - Y.a[1]), (float)(X.a[2] - Y.a[2]), (float)(X.a[0] - Y.b[0]),
            (float)(X.a[1] - Y.b[1]), (float)(X.a[2] - Y.b[2]), (float)(X.b[0] - Y.a[0]), (float)(X.b[1] - Y.a[1]),
            (float)(X.b[2] - Y.a[2]), X.t[0], X.t[1], X.t[2], X.l, Y.t[0], Y.t[1], Y.t[2], 0.f, half_expo, rho,
            rho0);
        g = rho * (X.t[0] * Y.t[0] + X.t[1] * Y.t[1] + X.t[2] * Y.t[2]);
        h = X.l * Y.l * rho0;
      }
      G[a][b] = g;
      H[a][b] = h;
    }
    __syncthreads();
    for (int p = t; p < 16 * 32; p += 256) {  // the tile's entries
      const int vl = p / 32, wl = p % 32;
      const int v = rb * 16 + vl, w = kt * 32 + wl;
      float sf = 0.f;
      if (v < n && w < n && v != w) {
        const int off = chain_offset(vi[0][vl], vi[1][wl]);
        if (off < -band || off > band) {
          float acc = 0.f;
          auto term = [&](int su, int sw) {
            const int I = sE[0][vl][su], J = sE[1][wl][sw];
            if (I < 0 || J < 0) return;
            const int a = sI[0][vl][su];
            if (I == J) {  // v and w are the two ends of edge I
              acc += ed[0][a].dg;
              return;
            }
            const int b = sI[1][wl][sw];
            acc += -0.5f * sS[0][vl][su] * sS[1][wl][sw] * G[a][b] - 0.0625f * H[a][b];
          };
          if (v < w) {
            term(0, 0); term(0, 1); term(1, 0); term(1, 1);
          } else {
            term(0, 0); term(1, 0); term(0, 1); term(1, 1);
          }
          sf = (float)((double)acc / (sq[0][vl] * sq[1][wl]));
        }
      }
      E[vl][wl] = sf;
    }
    __syncthreads();
    if (wave == q % 4) {  // the owning wave stores its lane vectors
      typename Vec8<T>::type vec;
      float f[8];
      const int vl = l % 16, c0 = 8 * (l / 16);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float sf = E[vl][c0 + j];
        const T r = (T)sf;
        vec[j] = r;
        f[j] = sf;
        if (sf != 0.f) {
          const double sw = sq[1][c0 + j];
          rs += (double)(float)r * sw;
          rs32 += (double)sf * sw;
        }
      }
      const size_t tile = (size_t)rb * nkt + kt;
      tiles[tile * 64 + l] = vec;
      if (W32) {
        tiles32[tile * 128 + l] = make_float4(f[0], f[1], f[2], f[3]);
        tiles32[tile * 128 + 64 + l] = make_float4(f[4], f[5], f[6], f[7]);
      }
    }
  }
  part[0][t] = rs;
  part[1][t] = rs32;
  __syncthreads();
  if (t < 16) {
    // row t appears in lanes t + 16 g (g < 4) of each of the 4 waves
    double a16 = 0.0, a32 = 0.0;
    for (int q = 0; q < 16; ++q) {
      a16 += part[0][q * 16 + t];
      a32 += part[1][q * 16 + t];
    }
    const int vv = rb * 16 + t;
    if (vv < n) {
      rowpart[(size_t)blockIdx.y * n + vv] = a16;
      if (W32) rowpart32[(size_t)blockIdx.y * n + vv] = a32;
    }
  }
}

// FP32 band: entries (v, w) with w at canonical chain offset o, 0 < |o| <= band,
// computed in FP64.  band_idx / band_val are [n][2 band]; slot o - 1 holds
// offset o > 0 and slot band - o - 1 offset o < 0; band_idx is -1 where the
// chain has no vertex at that offset.
template <int EC>
__global__ void k_lowp_band(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                            const V4<double>* __restrict__ GT, const int2* __restrict__ edges,
                            const int* __restrict__ inc_off, const int* __restrict__ inc,
                            const double* __restrict__ edge_out, const double* __restrict__ sqd,
                            const int* __restrict__ band_idx, int band, int n, double half_expo,
                            float* __restrict__ band_val, double* __restrict__ bandpart) {
  // 32 lanes per vertex: lane q computes slots q, q + 32, ..., and the row sum
  // is reduced over the lanes in a fixed order
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = g / 32, q = g % 32;
  const int nb = 2 * band;
  double rs = 0.0;
  if (v < n)
    for (int qq = q; qq < nb; qq += 32) {
      const int w = band_idx[(size_t)v * nb + qq];
      float val = 0.f;
      if (w >= 0) {
        const double a =
            sobolev_entry<double, EC>(min(v, w), max(v, w), GA, GB, GT, edges, inc_off, inc, edge_out, half_expo);
        val = (float)(a / (sqd[v] * sqd[w]));
        rs += (double)val * sqd[w];
      }
      band_val[(size_t)v * nb + qq] = val;
    }
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) rs += __shfl_xor(rs, off, 32);
  if (v < n && q == 0) bandpart[v] = rs;
}

// sigma_off_v = -(sum of the tile row parts) / sqrt(d_v): the diagonal that
// balances the entries kept in the tiles; diag_out = d_v (sigma_off_v +
// sigma_band_v), the diagonal of the whole stored operator.
__global__ void k_lowp_sigma(const double* __restrict__ rowpart, int ngroups, const double* __restrict__ bandpart,
                             const double* __restrict__ sqd, int n, double* __restrict__ sigma_off,
                             double* __restrict__ diag_out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double s = 0.0;
  for (int g = 0; g < ngroups; ++g) s += rowpart[(size_t)g * n + v];
  const double r = sqd[v];
  sigma_off[v] = -s / r;
  if (diag_out) diag_out[v] = -r * (s + (bandpart ? bandpart[v] : 0.0));
}

// ---------------------------------------------------------------------------
// product in difference form
// ---------------------------------------------------------------------------
// With sigma = sigma_off + sigma_band and sum_w S^_vw sqrt(d_w) = -sigma_v sqrt(d_v),
//   (A^ X)_v / sqrt(d_v) = sum_{w in tiles} S^_vw sqrt(d_w) (x_w - c)
//                        + sigma_off_v sqrt(d_v) (x_v - c)
//                        + sum_{w in band} S^_vw sqrt(d_w) (x_w - x_v)
// for any reference c; c is x at the first vertex of v's group of 64 rows.
// For a smooth X the terms are then of the size of the result instead of
// sqrt(d) |x|, so the FP32 accumulation and the 16-bit B operand do not lose
// the result to cancellation.  The B operand sqrt(d_w) (x_w - c) is formed in
// the product kernel from p_w = sqrt(d_w) (x_w - c_kt) (c_kt: x at the first
// vertex of column tile kt) plus sqrt(d_w) (c_kt - c), each part accurate
// relative to its own size.

// cref[kt][3] = x at vertex min(32 kt, n - 1); p[kt][3][32] and sqdf[kt][32] in FP32.
__global__ void k_lowp_prep(const double* __restrict__ X, const double* __restrict__ sqd, int n, int nkt,
                            double* __restrict__ cref, float* __restrict__ p, float* __restrict__ sqdf) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (kt, c, j)
  if (idx >= nkt * 96) return;
  const int kt = idx / 96, c = (idx / 32) % 3, j = idx % 32;
  const int w = kt * 32 + j;
  const int w0 = min(kt * 32, n - 1);
  const double cr = X[3 * w0 + c];
  if (j == 0) cref[kt * 3 + c] = cr;
  float pv = 0.f;
  if (w < n) pv = (float)(sqd[w] * (X[3 * w + c] - cr));
  p[idx] = pv;
  if (c == 0) sqdf[kt * 32 + j] = w < n ? (float)sqd[w] : 0.f;
}

// The parts of the operand that depend on the assembly only: sqdf, and p = 0
// for the padding columns w >= n (an operand written by another launch covers
// the vertices w < n).
__global__ void k_lowp_prep_static(const double* __restrict__ sqd, int n, int nkt, float* __restrict__ p,
                                   float* __restrict__ sqdf) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (kt, c, j)
  if (idx >= nkt * 96) return;
  const int kt = idx / 96, c = (idx / 32) % 3, j = idx % 32;
  const int w = kt * 32 + j;
  if (w >= n) p[idx] = 0.f;
  if (c == 0) sqdf[kt * 32 + j] = w < n ? (float)sqd[w] : 0.f;
}

// out[0] = 2 max|x| max sqrt(d): a bound of |sqrt(d_w) (x_w - c)| (one workgroup).
__global__ __launch_bounds__(1024) void k_lowp_absmax(const double* __restrict__ X, const double* __restrict__ sqd,
                                                      int n, double* __restrict__ out) {
  __shared__ double sx[1024], sd[1024];
  double mx = 0.0, md = 0.0;
  for (int i = threadIdx.x; i < 3 * n; i += 1024) mx = fmax(mx, fabs(X[i]));
  for (int i = threadIdx.x; i < n; i += 1024) md = fmax(md, sqd[i]);
  sx[threadIdx.x] = mx;
  sd[threadIdx.x] = md;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      sx[threadIdx.x] = fmax(sx[threadIdx.x], sx[threadIdx.x + k]);
      sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 2.0 * sx[0] * sd[0];
}

// Power-of-two factor that brings the bound into [0.5, 1): keeps the 16-bit
// B operand inside the FP16 range whatever the scale of X and D.
__device__ __forceinline__ double x_scale(const double* mx) {
  if (!mx) return 1.0;  // BF16 operands: FP32's exponent range, no scaling needed
  const double m = mx[0];
  if (!(m > 0.0) || !isfinite(m)) return 1.0;
  int e;
  frexp(m, &e);
  return ldexp(1.0, -e);
}

// B values of lane (group g = l / 16, component c) for column tile kt:
// b_j = sqrt(d_w) (x_w - c_rg) for w = 32 kt + 8 g + j.
struct BSrc {
  float4 p0, p1, s0, s1;
  double ck;
};
__device__ __forceinline__ BSrc load_b(const float4* __restrict__ P, const float4* __restrict__ SQ,
                                       const double* __restrict__ cref, int kt, int c, int g) {
  BSrc b;
  const size_t pb = ((size_t)kt * 3 + c) * 8 + 2 * g;
  b.p0 = P[pb];
  b.p1 = P[pb + 1];
  b.s0 = SQ[(size_t)kt * 8 + 2 * g];
  b.s1 = SQ[(size_t)kt * 8 + 2 * g + 1];
  b.ck = cref[kt * 3 + c];
  return b;
}
__device__ __forceinline__ void b_values(const BSrc& s, double crg, float scale, float* b) {
  const float dc = (float)(s.ck - crg);
  b[0] = fmaf(s.s0.x, dc, s.p0.x) * scale;
  b[1] = fmaf(s.s0.y, dc, s.p0.y) * scale;
  b[2] = fmaf(s.s0.z, dc, s.p0.z) * scale;
  b[3] = fmaf(s.s0.w, dc, s.p0.w) * scale;
  b[4] = fmaf(s.s1.x, dc, s.p1.x) * scale;
  b[5] = fmaf(s.s1.y, dc, s.p1.y) * scale;
  b[6] = fmaf(s.s1.z, dc, s.p1.z) * scale;
  b[7] = fmaf(s.s1.w, dc, s.p1.w) * scale;
}

// part[split][v][3] = sum over the split's column tiles of S^_vw sqrt(d_w) (x_w - c_rg) sc.
// One wave per (group of RB row blocks, split); four waves per workgroup.
// The loads for column tile kt + 1 are issued before the MFMAs of tile kt.
// B operand: columns 0-2 hi, 3-5 lo parts of the three components.
template <typename T, int RB>
__global__ __launch_bounds__(256, 4) void k_lowp_gemv(const typename Vec8<T>::type* __restrict__ tiles,
                                                   const float4* __restrict__ P, const float4* __restrict__ SQ,
                                                   const double* __restrict__ cref, const double* __restrict__ mx,
                                                   int n, int nrb, int nkt, int nsplit, int per,
                                                   float* __restrict__ part) {
  typedef typename Vec8<T>::type V;
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  const int l = threadIdx.x % 64;
  const int nrg = (nrb + RB - 1) / RB;
  if (wave >= nrg * nsplit) return;
  const int rg = wave / nsplit, sp = wave % nsplit;
  const int rb0 = rg * RB;
  const int k0 = sp * per, k1 = min(nkt, k0 + per);
  const int col = l % 16, g = l / 16, c = col % 3;
  const bool act = col < 6, hi = col < 3;
  const float scale = (float)x_scale(mx);
  const double crg = cref[(rb0 / 2) * 3 + c];  // first vertex of the group: 16 rb0 = 32 (rb0 / 2)
  f32x4 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
  const V* rows[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) rows[r] = tiles + (size_t)min(rb0 + r, nrb - 1) * nkt * 64 + l;
  if (k0 < k1) {
    V a[RB];
    BSrc bs = load_b(P, SQ, cref, k0, c, g);
#pragma unroll
    for (int r = 0; r < RB; ++r) a[r] = __builtin_nontemporal_load(&rows[r][(size_t)k0 * 64]);
    for (int kt = k0; kt < k1; ++kt) {
      V an[RB];
      BSrc bn;
      const bool more = kt + 1 < k1;
      if (more) {
        bn = load_b(P, SQ, cref, kt + 1, c, g);
#pragma unroll
        for (int r = 0; r < RB; ++r) an[r] = __builtin_nontemporal_load(&rows[r][(size_t)(kt + 1) * 64]);
      }
      float bv[8];
      b_values(bs, crg, scale, bv);
      V b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const T th = (T)bv[j];
        const T v = hi ? th : (T)(bv[j] - (float)th);
        b[j] = act ? v : (T)0.f;
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r] = mfma16(a[r], b, acc[r]);
      if (more) {
#pragma unroll
        for (int r = 0; r < RB; ++r) a[r] = an[r];
        bs = bn;
      }
    }
  }
  // lane l holds D[4 (l / 16) + j][l % 16]: columns 0-2 (hi) and 3-5 (lo)
#pragma unroll
  for (int r = 0; r < RB; ++r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float lo = __shfl_down(acc[r][j], 3, 16);
      const int v = (rb0 + r) * 16 + 4 * (l / 16) + j;
      if (hi && rb0 + r < nrb && v < n) part[((size_t)sp * n + v) * 3 + col] = acc[r][j] + lo;
    }
  }
}

// FP32 version: a 16 x 32 tile is eight v_mfma_f32_16x16x4f32 products; in
// product i lane l supplies A[l % 16][8 (l / 16) + i] and B row 8 (l / 16) + i
// of column l % 16 (columns 0-2 used), so the eight products together contract
// all 32 columns.  A tile is stored as two lane-contiguous halves (every
// lane's entries 0-3, then every lane's entries 4-7), so each of the two
// 16-byte loads of a wave covers whole cache lines; like the 16-bit tiles,
// the FP32 tiles are read once per product with streaming (nontemporal) loads.
template <int RB>
__global__ __launch_bounds__(256, 4) void k_lowp_gemv32(const float4* __restrict__ tiles, const float4* __restrict__ P,
                                                     const float4* __restrict__ SQ, const double* __restrict__ cref,
                                                     int n, int nrb, int nkt, int nsplit, int per,
                                                     float* __restrict__ part) {
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  const int l = threadIdx.x % 64;
  const int nrg = (nrb + RB - 1) / RB;
  if (wave >= nrg * nsplit) return;
  const int rg = wave / nsplit, sp = wave % nsplit;
  const int rb0 = rg * RB;
  const int k0 = sp * per, k1 = min(nkt, k0 + per);
  const int col = l % 16, g = l / 16, c = col % 3;
  const bool act = col < 3;
  const double crg = cref[(rb0 / 2) * 3 + c];
  f32x4 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float4* rows[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) rows[r] = tiles + (size_t)min(rb0 + r, nrb - 1) * nkt * 128 + l;
  for (int kt = k0; kt < k1; ++kt) {
    const BSrc bs = load_b(P, SQ, cref, kt, c, g);
    f32x4 a0[RB], a1[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      a0[r] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(&rows[r][(size_t)kt * 128]));
      a1[r] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(&rows[r][(size_t)kt * 128 + 64]));
    }
    float b[8];
    b_values(bs, crg, 1.f, b);
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = act ? b[j] : 0.f;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[r].x, b[0], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[r].y, b[1], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[r].z, b[2], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[r].w, b[3], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[r].x, b[4], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[r].y, b[5], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[r].z, b[6], acc[r], 0, 0, 0);
      acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[r].w, b[7], acc[r], 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int v = (rb0 + r) * 16 + 4 * (l / 16) + j;
      if (act && rb0 + r < nrb && v < n) part[((size_t)sp * n + v) * 3 + col] = acc[r][j];
    }
  }
}

// Y_v = sqrt(d_v) [ sum_splits part / sc + sigma_off_v sqrt(d_v) (x_v - c)
//                  + sum_band S^_vw sqrt(d_w) (x_w - x_v) ]   (FP64; sc = 1 when mx is null)
// 32 lanes per vertex (two vertices per wave): lanes stride over the splits'
// partial sums and the band entries, then a shuffle reduction over the 32.
__global__ __launch_bounds__(256) void k_lowp_finish(const float* __restrict__ part, int nsplit,
                                                     const double* __restrict__ mx, const int* __restrict__ band_idx,
                                                     const float* __restrict__ band_val, int band,
                                                     const double* __restrict__ sigma_off,
                                                     const double* __restrict__ sqd, const double* __restrict__ X,
                                                     int n, const double* __restrict__ base, double alpha,
                                                     double* __restrict__ Y) {
  const int h = threadIdx.x % 32;
  const int v = (blockIdx.x * 256 + threadIdx.x) / 32;
  const bool act = v < n;
  const int vv = act ? v : 0;
  const double isc = mx ? 1.0 / x_scale(mx) : 1.0;  // a power of two: exact
  const double x0 = X[3 * vv], x1 = X[3 * vv + 1], x2 = X[3 * vv + 2];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int p = h; p < nsplit; p += 32) {
    const float* q = part + ((size_t)p * n + vv) * 3;
    s0 += (double)q[0] * isc;
    s1 += (double)q[1] * isc;
    s2 += (double)q[2] * isc;
  }
  const int nb = 2 * band;
  for (int q = h; q < nb; q += 32) {
    const int w = band_idx[(size_t)vv * nb + q];
    if (w >= 0) {
      const double bw = (double)band_val[(size_t)vv * nb + q] * sqd[w];
      s0 += bw * (X[3 * w] - x0);
      s1 += bw * (X[3 * w + 1] - x1);
      s2 += bw * (X[3 * w + 2] - x2);
    }
  }
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 32);
    s1 += __shfl_xor(s1, off, 32);
    s2 += __shfl_xor(s2, off, 32);
  }
  if (act && h < 3) {
    const double sv = sqd[v];
    const double xc = h == 0 ? x0 : h == 1 ? x1 : x2;
    const double cr = X[3 * ((v / 64) * 64) + h];
    const double sh = h == 0 ? s0 : h == 1 ? s1 : s2;
    const double y = sv * (sh + sigma_off[v] * sv * (xc - cr));
    Y[3 * v + h] = base ? base[3 * v + h] + alpha * y : y;  // Y = base + alpha (A X) (Y may alias base)
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
constexpr int kLowpRB = 4;  // row blocks per wave in the products (the reference group is 64 rows)
// Waves per product launch (measured at 16k and 32k vertices: the streamed
// 16-bit tiles reach the highest HBM rate with about 2,048 long-running waves,
// the FP32 tiles with about 3,072).
constexpr int kLowpWaves16 = 2048, kLowpWaves32 = 3072;

rc_status LowpOp::ensure(const Curve& c, int fmt_, int band_, bool with32_) {
  if (!c.chain) {
    set_error("the assembled operator needs every vertex to have degree <= 2");
    return RC_ERR_UNSUPPORTED;
  }
  if (fmt_ != 1 && fmt_ != 2) {
    set_error("assembled operator format must be 1 (BF16) or 2 (FP16)");
    return RC_ERR_ARG;
  }
  if (band_ < 0 || band_ > kLowpMaxBand) {
    set_error("assembled operator band must lie in [0, 64]");
    return RC_ERR_ARG;
  }
  if (tiles && n == c.nV && fmt == fmt_ && band == band_ && with32 == with32_) return RC_OK;
  release();
  n = c.nV;
  fmt = fmt_;
  band = band_;
  with32 = with32_;
  nrb = cdiv(n, 16);
  nkt = cdiv(n, 32);
  ngroups = cdiv(nkt, 4);
  // column tiles split so that each product launches about kLowpWaves16 (kLowpWaves32) waves
  const int nrg = cdiv(nrb, kLowpRB);
  nsplit = std::max(1, std::min({64, nkt, cdiv(kLowpWaves16, nrg)}));
  per = cdiv(nkt, nsplit);
  nsplit = cdiv(nkt, per);
  nsplit32 = std::max(1, std::min({64, nkt, cdiv(kLowpWaves32, nrg)}));
  per32 = cdiv(nkt, nsplit32);
  nsplit32 = cdiv(nkt, per32);
  const size_t nb = (size_t)2 * band;
  auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess; };
  bool ok = al(&tiles, (size_t)nrb * nkt * 1024) && al((void**)&rowpart, sizeof(double) * (size_t)ngroups * n) &&
            al((void**)&dvec, sizeof(double) * n) && al((void**)&sqd, sizeof(double) * n) &&
            al((void**)&sigma, sizeof(double) * n) && al((void**)&bandpart, sizeof(double) * n) &&
            al((void**)&pbuf, sizeof(float) * 96 * (size_t)nkt) && al((void**)&sqdf, sizeof(float) * 32 * (size_t)nkt) &&
            al((void**)&cref, sizeof(double) * 3 * (size_t)nkt) &&
            al((void**)&part, sizeof(float) * 3 * (size_t)n * std::max(nsplit, nsplit32)) && al((void**)&mx, sizeof(double) * 2) &&
            al((void**)&vinfo, sizeof(int4) * (size_t)n) && al((void**)&band_idx, sizeof(int) * nb * n) &&
            al((void**)&band_val, sizeof(float) * nb * n);
  if (ok && with32)
    ok = al(&tiles32, (size_t)nrb * nkt * 2048) && al((void**)&rowpart32, sizeof(double) * (size_t)ngroups * n) &&
         al((void**)&sigma32, sizeof(double) * n);
  if (!ok) {
    set_error("allocation of the assembled operator failed");
    release();
    return RC_ERR_NOMEM;
  }
  // chain position of every vertex and the band's neighbour table
  std::vector<int4> hv(n);
  for (int v = 0; v < n; ++v) hv[v] = make_int4(-1 - v, 0, 1, 0);
  std::vector<Chain> chains = chains_of(c);
  for (size_t k = 0; k < chains.size(); ++k) {
    const Chain& ch = chains[k];
    const int m = (int)ch.verts.size();
    for (int p = 0; p < m; ++p) hv[ch.verts[p]] = make_int4((int)k, p, m, ch.loop ? 1 : 0);
  }
  std::vector<int> hb(nb * n, -1);
  for (size_t k = 0; k < chains.size() && band > 0; ++k) {
    const Chain& ch = chains[k];
    const int m = (int)ch.verts.size();
    for (int p = 0; p < m; ++p) {
      const int v = ch.verts[p];
      for (int o = -band; o <= band; ++o) {
        if (o == 0) continue;
        int q = p + o;
        if (ch.loop) {
          // keep o only where it is the canonical offset, in (-m/2, m/2]
          if (2 * o > m || 2 * o <= -m) continue;
          q = ((q % m) + m) % m;
        } else if (q < 0 || q >= m) {
          continue;
        }
        if (q == p) continue;
        hb[(size_t)v * nb + (o > 0 ? o - 1 : band - o - 1)] = ch.verts[q];
      }
    }
  }
  if (hipMemcpy(vinfo, hv.data(), sizeof(int4) * n, hipMemcpyHostToDevice) != hipSuccess ||
      (nb && hipMemcpy(band_idx, hb.data(), sizeof(int) * nb * n, hipMemcpyHostToDevice) != hipSuccess)) {
    set_error("upload of the band table failed");
    release();
    return RC_ERR_HIP;
  }
  return RC_OK;
}

void LowpOp::release() {
  void* ps[] = {tiles, tiles32, rowpart, rowpart32, dvec, sqd, sigma, sigma32, bandpart, pbuf, sqdf, cref,
                part, mx, vinfo, band_idx, band_val};
  for (void* p : ps)
    if (p) hipFree(p);
  tiles = tiles32 = nullptr;
  rowpart = rowpart32 = dvec = sqd = sigma = sigma32 = bandpart = mx = cref = nullptr;
  pbuf = sqdf = part = band_val = nullptr;
  vinfo = nullptr;
  band_idx = nullptr;
  n = 0;
  ready = false;
}

template <typename T, int EC>
static void assemble_t(const Curve& c, LowpOp& op, float half_expo, hipStream_t s) {
  typedef typename Vec8<T>::type V;
  dim3 grid(op.nrb, op.ngroups);
  const dim3 grid_ep(op.nrb, cdiv(op.nkt, kEpTiles));
  op.ngroups_used = c.max_degree <= 2 ? (int)grid_ep.y : op.ngroups;
  if (c.max_degree <= 2 && op.with32)
    hipLaunchKernelGGL((k_assemble_lowp_ep<T, EC, true>), grid_ep, dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges,
                       c.inc_off, c.inc, c.edge_out, op.sqd, op.vinfo, op.band, op.n, op.nkt, half_expo,
                       (V*)op.tiles, (float4*)op.tiles32, op.rowpart, op.rowpart32);
  else if (c.max_degree <= 2)
    hipLaunchKernelGGL((k_assemble_lowp_ep<T, EC, false>), grid_ep, dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges,
                       c.inc_off, c.inc, c.edge_out, op.sqd, op.vinfo, op.band, op.n, op.nkt, half_expo,
                       (V*)op.tiles, (float4*)nullptr, op.rowpart, (double*)nullptr);
  else if (op.with32)
    hipLaunchKernelGGL((k_assemble_lowp<T, EC, true>), grid, dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges,
                       c.inc_off, c.inc, c.edge_out, op.sqd, op.vinfo, op.band, op.n, op.nkt, half_expo,
                       (V*)op.tiles, (float4*)op.tiles32, op.rowpart, op.rowpart32);
  else
    hipLaunchKernelGGL((k_assemble_lowp<T, EC, false>), grid, dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges,
                       c.inc_off, c.inc, c.edge_out, op.sqd, op.vinfo, op.band, op.n, op.nkt, half_expo,
                       (V*)op.tiles, (float4*)nullptr, op.rowpart, (double*)nullptr);
  if (op.band > 0)
    hipLaunchKernelGGL((k_lowp_band<EC>), dim3(cdiv(op.n * 32, 256)), dim3(256), 0, s, c.gd.a, c.gd.b, c.gd.t, c.edges,
                       c.inc_off, c.inc, c.edge_out, op.sqd, op.band_idx, op.band, op.n, (double)half_expo,
                       op.band_val, op.bandpart);
}

template <typename T>
static void assemble_fmt(const Curve& c, LowpOp& op, double alpha, double beta, hipStream_t s) {
  const double sg = (beta - 1.0) / alpha - 1.0;
  const float half_expo = (float)(0.5 * (2.0 * sg + 1.0));
  switch (exp_case(alpha, beta)) {
    case kA2B4: assemble_t<T, kA2B4>(c, op, half_expo, s); break;
    case kA2B45: assemble_t<T, kA2B45>(c, op, half_expo, s); break;
    default: assemble_t<T, kGeneral>(c, op, half_expo, s); break;
  }
}

rc_status launch_assemble_lowp(const Curve& c, LowpOp& op, int fmt, int band, bool with32, double alpha,
                               double beta, double* diag_out, hipStream_t s) {
  RC_TRY(op.ensure(c, fmt, band, with32));
  // FP64 per-edge sums Wq, P0 (edge_out slots 0, 1) from the FP64 geometry
  RC_TRY(launch_edge_sums(c, alpha, beta, RC_F64, s));
  hipLaunchKernelGGL(k_lowp_dvec, dim3(cdiv(op.n, 256)), dim3(256), 0, s, c.edge_out, c.gd.a, c.inc_off, c.inc,
                     op.n, op.dvec, op.sqd);
  if (fmt == 1) assemble_fmt<__bf16>(c, op, alpha, beta, s);
  else assemble_fmt<_Float16>(c, op, alpha, beta, s);
  const double* bp = op.band > 0 ? op.bandpart : nullptr;
  hipLaunchKernelGGL(k_lowp_sigma, dim3(cdiv(op.n, 256)), dim3(256), 0, s, op.rowpart, op.ngroups_used, bp, op.sqd,
                     op.n, op.sigma, diag_out);
  if (with32)
    hipLaunchKernelGGL(k_lowp_sigma, dim3(cdiv(op.n, 256)), dim3(256), 0, s, op.rowpart32, op.ngroups_used, bp, op.sqd,
                       op.n, op.sigma32, (double*)nullptr);
  hipLaunchKernelGGL(k_lowp_prep_static, dim3(cdiv(op.nkt * 96, 256)), dim3(256), 0, s, op.sqd, op.n, op.nkt, op.pbuf,
                     op.sqdf);
  RC_HIP(hipGetLastError());
  op.ready = true;
  return RC_OK;
}

static void prep(const LowpOp& op, const double* X, hipStream_t s) {
  hipLaunchKernelGGL(k_lowp_prep, dim3(cdiv(op.nkt * 96, 256)), dim3(256), 0, s, X, op.sqd, op.n, op.nkt, op.cref,
                     op.pbuf, op.sqdf);
}

template <typename T>
static void apply16(const LowpOp& op, const double* X, double* Y, hipStream_t s, KernelTimer* timer,
                    const double* base, double alpha, bool prepped) {
  typedef typename Vec8<T>::type V;
  // FP16 operands need the power-of-two scaling into range; BF16 ones do not
  const double* mx = std::is_same<T, _Float16>::value ? (const double*)op.mx : nullptr;
  if (mx) hipLaunchKernelGGL(k_lowp_absmax, dim3(1), dim3(1024), 0, s, X, op.sqd, op.n, op.mx);
  if (!prepped) prep(op, X, s);
  const int waves = cdiv(op.nrb, kLowpRB) * op.nsplit;
  if (timer) timer->mark(timer->lowp, s);
  hipLaunchKernelGGL((k_lowp_gemv<T, kLowpRB>), dim3(cdiv(waves, 4)), dim3(256), 0, s, (const V*)op.tiles,
                     (const float4*)op.pbuf, (const float4*)op.sqdf, (const double*)op.cref, mx, op.n, op.nrb,
                     op.nkt, op.nsplit, op.per, op.part);
  if (timer) timer->mark(timer->lowp, s);
  hipLaunchKernelGGL(k_lowp_finish, dim3(cdiv(op.n, 8)), dim3(256), 0, s, op.part, op.nsplit, mx, op.band_idx,
                     op.band_val, op.band, op.sigma, op.sqd, X, op.n, base, alpha, Y);
}

rc_status launch_lowp_apply(const LowpOp& op, const double* X, double* Y, hipStream_t s, KernelTimer* timer,
                            const double* base, double alpha, bool prepped) {
  if (!op.ready) {
    set_error("the assembled operator has not been built");
    return RC_ERR_ARG;
  }
  KernelTimer* t = (timer && timer->on) ? timer : nullptr;
  if (op.fmt == 1) apply16<__bf16>(op, X, Y, s, t, base, alpha, prepped);
  else apply16<_Float16>(op, X, Y, s, t, base, alpha, prepped);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_lowp_apply32(const LowpOp& op, const double* X, double* Y, hipStream_t s, KernelTimer* timer) {
  if (!op.ready || !op.with32) {
    set_error("the assembled FP32 operator has not been built");
    return RC_ERR_ARG;
  }
  KernelTimer* t = (timer && timer->on) ? timer : nullptr;
  prep(op, X, s);
  const int waves = cdiv(op.nrb, kLowpRB) * op.nsplit32;
  if (t) t->mark(t->asm32, s);
  hipLaunchKernelGGL((k_lowp_gemv32<kLowpRB>), dim3(cdiv(waves, 4)), dim3(256), 0, s, (const float4*)op.tiles32,
                     (const float4*)op.pbuf, (const float4*)op.sqdf, (const double*)op.cref, op.n, op.nrb, op.nkt,
                     op.nsplit32, op.per32, op.part);
  if (t) t->mark(t->asm32, s);
  hipLaunchKernelGGL(k_lowp_finish, dim3(cdiv(op.n, 8)), dim3(256), 0, s, op.part, op.nsplit32,
                     (const double*)nullptr, op.band_idx, op.band_val, op.band, op.sigma32, op.sqd, X, op.n,
                     (const double*)nullptr, 1.0, Y);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
