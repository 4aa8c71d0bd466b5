// Bounding volume hierarchy over tangent-points and the Barnes-Hut energy and
// differential (paper App. B.1).
//
// Build (on the device, level by level, one workgroup per node):
//   every edge I is the tangent-point p_I = (T_I, x_I) in R^6 (App. B.1.1).
//   A node with more than `leaf` edges is split: on each of the six axes a
//   balanced plane is found from a 64-bin histogram of the node's points, the
//   two child boxes that plane would produce are measured, and the axis whose
//   split minimises diam(left)^2 + diam(right)^2 (6-D box diameters) wins.
//   The node's index range is then partitioned stably in place, so every node
//   owns a contiguous range of the edge permutation.  Child slots come from a
//   prefix sum over the level, so the layout is deterministic.
// Node data (App. B.1.1): mass L = sum l_I, centre xbar = sum l_I x_I / L,
//   mean tangent Tbar = sum l_I T_I / L, and the half-diagonals r_x, r_T of
//   the node's spatial and tangential boxes.
// Traversal (App. B.1.2): targets are processed in BVH order so that a wave's
//   64 targets are neighbours; the wave walks the tree as one packet with an
//   LDS stack of (node, lane mask).  For each lane the node is admissible when
//   r_x < theta |x_I - xbar| and r_T < theta (eq. BarnesHutCondition); then the
//   cluster term uses (xbar, Tbar, L) in place of a source edge (eq. BVHNodeTPE
//   and the differential formula of App. B.1.2).  At a leaf the remaining lanes
//   sum the exact edge-midpoint pairs, omitting edges that share a vertex.

#include <algorithm>
#include <vector>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

static inline int cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr int kBvhThreads = 256;
constexpr int kBins = 64;
constexpr int kStack = 64;
// top-level split over many workgroups: levels of at most kBigMaxNodes nodes
// whose mean size is at least kBigNode, in chunks of kBigChunk positions
constexpr int kBigMaxNodes = 1024, kBigNode = 2048, kBigChunk = 4096, kBigWords = 640;

// tangent-points, SoA [6][nE]: T (3) then midpoint x (3); perm (when given) reset to the identity
__global__ void k_tangent_points(const V4<float>* __restrict__ GA, const V4<float>* __restrict__ GB,
                                 const V4<float>* __restrict__ GT, int nE, float* __restrict__ pts,
                                 int* __restrict__ perm) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const V4<float> a = GA[I], b = GB[I], t = GT[I];
  pts[I] = t.x;
  pts[nE + I] = t.y;
  pts[2 * (size_t)nE + I] = t.z;
  pts[3 * (size_t)nE + I] = 0.5f * (a.x + b.x);
  pts[4 * (size_t)nE + I] = 0.5f * (a.y + b.y);
  pts[5 * (size_t)nE + I] = 0.5f * (a.z + b.z);
  if (perm) perm[I] = I;
}

__device__ __forceinline__ float block_min(float v, float* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBvhThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fminf(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  float r = sm[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ float block_max(float v, float* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBvhThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  float r = sm[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ int bin_of(float x, float lo, float inv_w) {
  int b = (int)((x - lo) * inv_w);
  return min(kBins - 1, max(0, b));
}

// One workgroup per node of the level [lb, lb + count).  node = (start, count,
// left child, number of left edges after the split).  split[i] = 1 if split.
__global__ __launch_bounds__(kBvhThreads) void k_bvh_split(const float* __restrict__ pts, int nE,
                                                            int4* __restrict__ node, int lb, int* __restrict__ perm,
                                                            int* __restrict__ scratch, int leaf,
                                                            int* __restrict__ split) {
  __shared__ float smf[kBvhThreads];
  __shared__ int smi[kBvhThreads];
  __shared__ unsigned hist[6][kBins];
  __shared__ float lo[6], hi[6];
  __shared__ int cut[6], nleft[6];
  __shared__ float cost[6];
  __shared__ int best;
  const int bid = blockIdx.x;
  int4 nd = node[lb + bid];
  const int s = nd.x, n = nd.y;
  const int tid = threadIdx.x;
  if (n <= leaf) {
    if (tid == 0) {
      split[bid] = 0;
      node[lb + bid] = make_int4(s, n, -1, 0);
    }
    return;
  }
  // bounding box on the six axes
  for (int a = 0; a < 6; ++a) {
    float mn = INFINITY, mx = -INFINITY;
    for (int i = tid; i < n; i += kBvhThreads) {
      const float v = pts[(size_t)a * nE + perm[s + i]];
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
    mn = block_min(mn, smf);
    mx = block_max(mx, smf);
    if (tid == 0) {
      lo[a] = mn;
      hi[a] = mx;
    }
  }
  for (int i = tid; i < 6 * kBins; i += kBvhThreads) hist[i / kBins][i % kBins] = 0u;
  __syncthreads();
  // histograms
  for (int i = tid; i < n; i += kBvhThreads) {
    const int I = perm[s + i];
    for (int a = 0; a < 6; ++a) {
      const float w = hi[a] - lo[a];
      if (!(w > 0.f)) continue;
      atomicAdd(&hist[a][bin_of(pts[(size_t)a * nE + I], lo[a], kBins / w)], 1u);
    }
  }
  __syncthreads();
  // balanced cut per axis: first bin boundary where the running count reaches n/2
  if (tid < 6) {
    const int a = tid;
    int run = 0, c = -1, nl = 0;
    if (hi[a] - lo[a] > 0.f) {
      for (int b = 0; b < kBins - 1; ++b) {
        run += (int)hist[a][b];
        if (run >= n / 2) {
          c = b + 1;
          nl = run;
          break;
        }
      }
      if (c > 0 && (nl == 0 || nl == n)) c = -1;
    }
    cut[a] = c;
    nleft[a] = nl;
  }
  __syncthreads();
  // cost of each candidate: squared diameters of the two child boxes
  for (int a = 0; a < 6; ++a) {
    if (cut[a] < 0) {
      if (tid == 0) cost[a] = INFINITY;
      continue;
    }
    const float inv_w = kBins / (hi[a] - lo[a]);
    float lmn[6], lmx[6], rmn[6], rmx[6];
    for (int d = 0; d < 6; ++d) {
      lmn[d] = rmn[d] = INFINITY;
      lmx[d] = rmx[d] = -INFINITY;
    }
    for (int i = tid; i < n; i += kBvhThreads) {
      const int I = perm[s + i];
      const bool left = bin_of(pts[(size_t)a * nE + I], lo[a], inv_w) < cut[a];
      for (int d = 0; d < 6; ++d) {
        const float v = pts[(size_t)d * nE + I];
        if (left) {
          lmn[d] = fminf(lmn[d], v);
          lmx[d] = fmaxf(lmx[d], v);
        } else {
          rmn[d] = fminf(rmn[d], v);
          rmx[d] = fmaxf(rmx[d], v);
        }
      }
    }
    float dl = 0.f, dr = 0.f;
    for (int d = 0; d < 6; ++d) {
      const float a0 = block_min(lmn[d], smf), a1 = block_max(lmx[d], smf);
      const float b0 = block_min(rmn[d], smf), b1 = block_max(rmx[d], smf);
      dl += (a1 - a0) * (a1 - a0);
      dr += (b1 - b0) * (b1 - b0);
    }
    if (tid == 0) cost[a] = dl + dr;
  }
  __syncthreads();
  if (tid == 0) {
    int b = -1;
    for (int a = 0; a < 6; ++a)
      if (cut[a] >= 0 && (b < 0 || cost[a] < cost[b])) b = a;
    best = b;
  }
  __syncthreads();
  const int a = best;
  const int nl = (a >= 0) ? nleft[a] : n / 2;  // no usable plane: split the range in halves
  const float inv_w = (a >= 0) ? kBins / (hi[a] - lo[a]) : 0.f;
  // stable partition of perm[s, s+n) into scratch, then copy back
  int lbase = 0, rbase = 0;
  for (int c0 = 0; c0 < n; c0 += kBvhThreads) {
    const int i = c0 + tid;
    int flag = 0, I = -1;
    if (i < n) {
      I = perm[s + i];
      flag = (a >= 0) ? (bin_of(pts[(size_t)a * nE + I], lo[a], inv_w) < cut[a]) : (i < nl);
    }
    // exclusive scan of flags within the chunk
    smi[tid] = flag;
    __syncthreads();
    for (int off = 1; off < kBvhThreads; off <<= 1) {
      const int v = (tid >= off) ? smi[tid - off] : 0;
      __syncthreads();
      smi[tid] += v;
      __syncthreads();
    }
    const int incl = smi[tid];
    const int total = smi[kBvhThreads - 1];
    const int cnt = min(kBvhThreads, n - c0);
    if (i < n) {
      if (flag) scratch[s + lbase + incl - 1] = I;
      else scratch[s + nl + rbase + (i - c0) - incl] = I;
    }
    lbase += total;
    rbase += cnt - total;
    __syncthreads();
  }
  for (int i = tid; i < n; i += kBvhThreads) perm[s + i] = scratch[s + i];
  if (tid == 0) {
    split[bid] = 1;
    node[lb + bid] = make_int4(s, n, 0, nl);
  }
}

// ---------------------------------------------------------------------------
// The same split for the top levels (few nodes, many edges each) over many
// workgroups: a node's range is cut into chunks of kBigChunk positions, and
// every quantity the single-workgroup split takes (the six-axis box, the
// per-axis histograms, the two child boxes of each candidate cut) is a
// minimum, maximum or integer count, accumulated by chunk with atomics, so
// the split (cut, axis, stable partition) is exactly that of k_bvh_split.
// Floats take part in integer min / max through an order-preserving map.
// Per node (kBigWords ints): box [6][2], hist [6][kBins], cand [6][2][6][2],
// cut [6], nleft [6], plan (axis, left count, lo bits, inv_w bits).
// ---------------------------------------------------------------------------
constexpr int oBox = 0, oHist = oBox + 12, oCand = oHist + 6 * kBins, oCut = oCand + 144, oNl = oCut + 6,
              oPlan = oNl + 6;
static_assert(oPlan + 4 <= kBigWords, "per-node words of the top-level split");

__device__ __forceinline__ int fkey(float f) {
  const int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float fval(int k) { return __int_as_float(k >= 0 ? k : k ^ 0x7FFFFFFF); }

__device__ __forceinline__ float wave_min(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// chunk c = (node of the level, first position in the node, positions, 0)
__global__ void k_big_init(int* __restrict__ big, int count) {
  int* w = big + (size_t)kBigWords * blockIdx.x;
  for (int i = threadIdx.x; i < kBigWords; i += blockDim.x) {
    int v = 0;
    if (i < oHist) v = (i % 2 == 0) ? fkey(INFINITY) : fkey(-INFINITY);
    else if (i >= oCand && i < oCut) v = ((i - oCand) % 2 == 0) ? fkey(INFINITY) : fkey(-INFINITY);
    w[i] = v;
  }
}

__global__ __launch_bounds__(kBvhThreads) void k_big_bounds(const float* __restrict__ pts, int nE,
                                                             const int4* __restrict__ node, int lb,
                                                             const int* __restrict__ perm,
                                                             const int4* __restrict__ chunks, int* __restrict__ big) {
  const int4 ch = chunks[blockIdx.x];
  const int s = node[lb + ch.x].x + ch.y;
  int* w = big + (size_t)kBigWords * ch.x;
  for (int a = 0; a < 6; ++a) {
    float mn = INFINITY, mx = -INFINITY;
    for (int i = threadIdx.x; i < ch.z; i += kBvhThreads) {
      const float v = pts[(size_t)a * nE + perm[s + i]];
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if (threadIdx.x % 64 == 0) {
      atomicMin(w + oBox + 2 * a, fkey(mn));
      atomicMax(w + oBox + 2 * a + 1, fkey(mx));
    }
  }
}

__global__ __launch_bounds__(kBvhThreads) void k_big_hist(const float* __restrict__ pts, int nE,
                                                           const int4* __restrict__ node, int lb,
                                                           const int* __restrict__ perm,
                                                           const int4* __restrict__ chunks, int* __restrict__ big) {
  __shared__ unsigned hist[6][kBins];
  const int4 ch = chunks[blockIdx.x];
  const int s = node[lb + ch.x].x + ch.y;
  int* w = big + (size_t)kBigWords * ch.x;
  for (int i = threadIdx.x; i < 6 * kBins; i += kBvhThreads) hist[i / kBins][i % kBins] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < ch.z; i += kBvhThreads) {
    const int I = perm[s + i];
    for (int a = 0; a < 6; ++a) {
      const float lo = fval(w[oBox + 2 * a]), hi = fval(w[oBox + 2 * a + 1]);
      const float wd = hi - lo;
      if (!(wd > 0.f)) continue;
      atomicAdd(&hist[a][bin_of(pts[(size_t)a * nE + I], lo, kBins / wd)], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 6 * kBins; i += kBvhThreads)
    if (hist[i / kBins][i % kBins]) atomicAdd(w + oHist + i, (int)hist[i / kBins][i % kBins]);
}

// per node: the balanced cut of each axis (as k_bvh_split)
__global__ void k_big_cut(const int4* __restrict__ node, int lb, int* __restrict__ big) {
  const int a = threadIdx.x;
  if (a >= 6) return;
  int* w = big + (size_t)kBigWords * blockIdx.x;
  const int n = node[lb + blockIdx.x].y;
  const float lo = fval(w[oBox + 2 * a]), hi = fval(w[oBox + 2 * a + 1]);
  int run = 0, c = -1, nl = 0;
  if (hi - lo > 0.f) {
    for (int b = 0; b < kBins - 1; ++b) {
      run += w[oHist + a * kBins + b];
      if (run >= n / 2) {
        c = b + 1;
        nl = run;
        break;
      }
    }
    if (c > 0 && (nl == 0 || nl == n)) c = -1;
  }
  w[oCut + a] = c;
  w[oNl + a] = nl;
}

// the two child boxes of candidate axis blockIdx.y on the chunk's positions
__global__ __launch_bounds__(kBvhThreads) void k_big_cand(const float* __restrict__ pts, int nE,
                                                           const int4* __restrict__ node, int lb,
                                                           const int* __restrict__ perm,
                                                           const int4* __restrict__ chunks, int* __restrict__ big) {
  const int4 ch = chunks[blockIdx.x];
  const int a = blockIdx.y;
  int* w = big + (size_t)kBigWords * ch.x;
  const int cut = w[oCut + a];
  if (cut < 0) return;  // uniform per workgroup
  const int s = node[lb + ch.x].x + ch.y;
  const float lo = fval(w[oBox + 2 * a]), hi = fval(w[oBox + 2 * a + 1]);
  const float inv_w = kBins / (hi - lo);
  float lmn[6], lmx[6], rmn[6], rmx[6];
  for (int d = 0; d < 6; ++d) {
    lmn[d] = rmn[d] = INFINITY;
    lmx[d] = rmx[d] = -INFINITY;
  }
  for (int i = threadIdx.x; i < ch.z; i += kBvhThreads) {
    const int I = perm[s + i];
    const bool left = bin_of(pts[(size_t)a * nE + I], lo, inv_w) < cut;
    for (int d = 0; d < 6; ++d) {
      const float v = pts[(size_t)d * nE + I];
      if (left) {
        lmn[d] = fminf(lmn[d], v);
        lmx[d] = fmaxf(lmx[d], v);
      } else {
        rmn[d] = fminf(rmn[d], v);
        rmx[d] = fmaxf(rmx[d], v);
      }
    }
  }
  int* cw = w + oCand + a * 24;
  for (int d = 0; d < 6; ++d) {
    const float a0 = wave_min(lmn[d]), a1 = wave_max(lmx[d]), b0 = wave_min(rmn[d]), b1 = wave_max(rmx[d]);
    if (threadIdx.x % 64 == 0) {
      atomicMin(cw + 2 * d, fkey(a0));
      atomicMax(cw + 2 * d + 1, fkey(a1));
      atomicMin(cw + 12 + 2 * d, fkey(b0));
      atomicMax(cw + 12 + 2 * d + 1, fkey(b1));
    }
  }
}

// per split node: costs, the chosen axis, the node record and the partition plan
__global__ void k_big_choose_split(int4* __restrict__ node, int lb, int* __restrict__ big, int* __restrict__ split) {
  if (threadIdx.x != 0) return;
  const int k = blockIdx.x;
  if (!split[k]) return;  // a leaf of this level, written by the host
  int* w = big + (size_t)kBigWords * k;
  const int4 nd = node[lb + k];
  int b = -1;
  float cb = 0.f;
  for (int a = 0; a < 6; ++a) {
    if (w[oCut + a] < 0) continue;
    const int* cw = w + oCand + a * 24;
    float dl = 0.f, dr = 0.f;
    for (int d = 0; d < 6; ++d) {
      const float a0 = fval(cw[2 * d]), a1 = fval(cw[2 * d + 1]);
      const float b0 = fval(cw[12 + 2 * d]), b1 = fval(cw[12 + 2 * d + 1]);
      dl += (a1 - a0) * (a1 - a0);
      dr += (b1 - b0) * (b1 - b0);
    }
    const float c = dl + dr;
    if (b < 0 || c < cb) {
      b = a;
      cb = c;
    }
  }
  const int nl = (b >= 0) ? w[oNl + b] : nd.y / 2;  // no usable plane: the range in halves
  w[oPlan] = b;
  w[oPlan + 1] = nl;
  if (b >= 0) {
    const float lo = fval(w[oBox + 2 * b]), hi = fval(w[oBox + 2 * b + 1]);
    w[oPlan + 2] = __float_as_int(lo);
    w[oPlan + 3] = __float_as_int(kBins / (hi - lo));
  }
  split[k] = 1;
  node[lb + k] = make_int4(nd.x, nd.y, 0, nl);
}

__device__ __forceinline__ int big_left(const float* __restrict__ pts, int nE, const int* w, int I, int pos) {
  const int b = w[oPlan];
  if (b < 0) return pos < w[oPlan + 1];
  return bin_of(pts[(size_t)b * nE + I], __int_as_float(w[oPlan + 2]), __int_as_float(w[oPlan + 3])) < w[oCut + b];
}

// left positions per chunk into chunks[c].w
__global__ __launch_bounds__(kBvhThreads) void k_big_count(const float* __restrict__ pts, int nE,
                                                            const int4* __restrict__ node, int lb,
                                                            const int* __restrict__ perm, int4* __restrict__ chunks,
                                                            const int* __restrict__ big) {
  __shared__ int sm[kBvhThreads / 64];
  const int4 ch = chunks[blockIdx.x];
  const int s = node[lb + ch.x].x + ch.y;
  const int* w = big + (size_t)kBigWords * ch.x;
  int cnt = 0;
  for (int i = threadIdx.x; i < ch.z; i += kBvhThreads) cnt += big_left(pts, nE, w, perm[s + i], ch.y + i);
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < kBvhThreads / 64; ++k) t += sm[k];
    chunks[blockIdx.x].w = t;
  }
}

// stable partition of the chunk's positions into scratch: its left ones after
// the left ones of the node's earlier chunks, its right ones likewise after nl
__global__ __launch_bounds__(kBvhThreads) void k_big_scatter(const float* __restrict__ pts, int nE,
                                                              const int4* __restrict__ node, int lb,
                                                              const int* __restrict__ perm,
                                                              const int4* __restrict__ chunks,
                                                              const int* __restrict__ big, int* __restrict__ scratch) {
  __shared__ int smi[kBvhThreads];
  __shared__ int base_l;
  const int4 ch = chunks[blockIdx.x];
  const int4 nd = node[lb + ch.x];
  const int* w = big + (size_t)kBigWords * ch.x;
  const int nl = w[oPlan + 1];
  const int tid = threadIdx.x;
  if (tid == 0) {  // left positions of the node's chunks before this one (they precede it in the table)
    int t = 0;
    for (int c = blockIdx.x - 1; c >= 0 && chunks[c].x == ch.x; --c) t += chunks[c].w;
    base_l = t;
  }
  __syncthreads();
  int lbase = base_l, rbase = ch.y - base_l;
  for (int c0 = 0; c0 < ch.z; c0 += kBvhThreads) {
    const int i = c0 + tid;
    int flag = 0, I = -1;
    if (i < ch.z) {
      I = perm[nd.x + ch.y + i];
      flag = big_left(pts, nE, w, I, ch.y + i);
    }
    smi[tid] = flag;
    __syncthreads();
    for (int off = 1; off < kBvhThreads; off <<= 1) {
      const int v = (tid >= off) ? smi[tid - off] : 0;
      __syncthreads();
      smi[tid] += v;
      __syncthreads();
    }
    const int incl = smi[tid];
    const int total = smi[kBvhThreads - 1];
    const int cnt = min(kBvhThreads, ch.z - c0);
    if (i < ch.z) {
      if (flag) scratch[nd.x + lbase + incl - 1] = I;
      else scratch[nd.x + nl + rbase + (i - c0) - incl] = I;
    }
    lbase += total;
    rbase += cnt - total;
    __syncthreads();
  }
}

__global__ void k_big_copy(const int4* __restrict__ node, int lb, const int4* __restrict__ chunks,
                           const int* __restrict__ scratch, int* __restrict__ perm) {
  const int4 ch = chunks[blockIdx.x];
  const int s = node[lb + ch.x].x + ch.y;
  for (int i = threadIdx.x; i < ch.z; i += blockDim.x) perm[s + i] = scratch[s + i];
}

// Children of the level's split nodes: slots le + 2 * (rank among split nodes).
__global__ void k_bvh_children(int4* __restrict__ node, int lb, int count, const int* __restrict__ split, int le,
                               int* __restrict__ next_count) {
  __shared__ int sm[1024];
  int base = 0;
  for (int c0 = 0; c0 < count; c0 += 1024) {
    const int i = c0 + threadIdx.x;
    const int f = (i < count) ? split[i] : 0;
    sm[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int v = (threadIdx.x >= off) ? sm[threadIdx.x - off] : 0;
      __syncthreads();
      sm[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) {
      const int rank = base + sm[threadIdx.x] - 1;
      const int4 nd = node[lb + i];
      const int left = le + 2 * rank;
      node[left] = make_int4(nd.x, nd.w, -1, 0);
      node[left + 1] = make_int4(nd.x + nd.w, nd.y - nd.w, -1, 0);
      node[lb + i] = make_int4(nd.x, nd.y, left, nd.w);
    }
    base += sm[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) next_count[0] = 2 * base;
}

// Node data: na = (xbar, L), nb = (Tbar, |Tbar|^2), nr = (r_x, r_T).
__global__ __launch_bounds__(kBvhThreads) void k_bvh_props(const float* __restrict__ pts,
                                                            const V4<float>* __restrict__ GA, int nE,
                                                            const int4* __restrict__ node,
                                                            const int* __restrict__ perm, float4* __restrict__ na,
                                                            float4* __restrict__ nb, float2* __restrict__ nr) {
  __shared__ float smf[kBvhThreads];
  const int4 nd = node[blockIdx.x];
  const int s = nd.x, n = nd.y;
  float sl = 0.f, sx[3] = {0, 0, 0}, st[3] = {0, 0, 0};
  float mn[6], mx[6];
  for (int d = 0; d < 6; ++d) {
    mn[d] = INFINITY;
    mx[d] = -INFINITY;
  }
  for (int i = threadIdx.x; i < n; i += kBvhThreads) {
    const int I = perm[s + i];
    const float l = GA[I].w;
    sl += l;
    for (int d = 0; d < 3; ++d) {
      const float t = pts[(size_t)d * nE + I], x = pts[(size_t)(3 + d) * nE + I];
      st[d] += l * t;
      sx[d] += l * x;
    }
    for (int d = 0; d < 6; ++d) {
      const float v = pts[(size_t)d * nE + I];
      mn[d] = fminf(mn[d], v);
      mx[d] = fmaxf(mx[d], v);
    }
  }
  float vals[7] = {sl, sx[0], sx[1], sx[2], st[0], st[1], st[2]};
  float red[7];
  for (int k = 0; k < 7; ++k) {
    smf[threadIdx.x] = vals[k];
    __syncthreads();
    for (int w = kBvhThreads / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) smf[threadIdx.x] += smf[threadIdx.x + w];
      __syncthreads();
    }
    red[k] = smf[0];
    __syncthreads();
  }
  float ext[6];
  for (int d = 0; d < 6; ++d) ext[d] = block_max(mx[d], smf) - block_min(mn[d], smf);
  if (threadIdx.x == 0) {
    const float L = red[0], iL = 1.f / L;
    const float tx = red[4] * iL, ty = red[5] * iL, tz = red[6] * iL;
    na[blockIdx.x] = make_float4(red[1] * iL, red[2] * iL, red[3] * iL, L);
    nb[blockIdx.x] = make_float4(tx, ty, tz, tx * tx + ty * ty + tz * tz);
    const float rT = 0.5f * sqrtf(ext[0] * ext[0] + ext[1] * ext[1] + ext[2] * ext[2]);
    const float rx = 0.5f * sqrtf(ext[3] * ext[3] + ext[4] * ext[4] + ext[5] * ext[5]);
    nr[blockIdx.x] = make_float2(rx, rT);
  }
}

__global__ void k_invperm(const int* __restrict__ perm, int nE, int* __restrict__ inv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nE) inv[perm[i]] = i;
}

// Chain-near test (same chain, at most kBand apart): such pairs are summed in
// FP64, where FP32 would lose their small offsets perpendicular to T.
__device__ __forceinline__ bool bh_chain_near(int4 ci, int4 cj) {
  int dd = abs(cj.y - ci.y);
  dd = ci.w ? min(dd, ci.z - dd) : dd;
  return (cj.x == ci.x) & (dd <= kBand);
}

// Barnes-Hut traversal: 10 accumulators per target in the edge-midpoint layout
// (E, S, G(3), Gt, Hd(3), Ht), written to part[slot][I].
// A cluster that holds an edge sharing a vertex with the target is never
// admissible for it (its pair with that edge is omitted from the energy), so
// every lane keeps the BVH positions of its neighbouring edges (at most
// kMaxNbr; the launcher checks the vertex degrees).
constexpr int kMaxNbr = 6;

template <int EC, bool BAND>
__global__ __launch_bounds__(256) void k_bh_traverse(
    const V4<float>* __restrict__ GA, const V4<float>* __restrict__ GB, const V4<float>* __restrict__ GT,
    const V4<double>* __restrict__ DA, const V4<double>* __restrict__ DB, const V4<double>* __restrict__ DT,
    const int2* __restrict__ edges, const int* __restrict__ inc_off, const int* __restrict__ inc,
    const int4* __restrict__ cinfo, int nE, const int* __restrict__ perm, const int* __restrict__ invperm,
    const int4* __restrict__ node, const float4* __restrict__ na, const float4* __restrict__ nb,
    const float2* __restrict__ nr, float theta, float half_alpha, float half_beta, float beta,
    double* __restrict__ part, unsigned long long* __restrict__ work) {
  __shared__ int st_node[4][kStack];
  __shared__ unsigned long long st_mask[4][kStack];
  __shared__ unsigned long long blk_work[2];
  if (threadIdx.x < 2) blk_work[threadIdx.x] = 0ull;
  __syncthreads();
  const int w = threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const bool act = t < nE;
  const int I = act ? perm[t] : perm[nE - 1];
  const V4<float> a = GA[I], b = GB[I], tt = GT[I];
  const float mxI = 0.5f * (a.x + b.x), myI = 0.5f * (a.y + b.y), mzI = 0.5f * (a.z + b.z);
  const int2 ei = edges[I];
  int nbr[kMaxNbr];
  int nn = 0;
  for (int v = 0; v < 2; ++v) {
    const int vert = v ? ei.y : ei.x;
    for (int q = inc_off[vert]; q < inc_off[vert + 1]; ++q) {
      const int J = inc[q] >> 1;
      if (J != I && nn < kMaxNbr) nbr[nn++] = invperm[J];
    }
  }
  int4 ci = make_int4(-1, 0, 0, 0);
  double pxd = 0, pyd = 0, pzd = 0, txd = 0, tyd = 0, tzd = 0;
  if constexpr (BAND) {
    ci = cinfo[I];
    const V4<double> da = DA[I], db = DB[I], dt = DT[I];
    pxd = 0.5 * (da.x + db.x);
    pyd = 0.5 * (da.y + db.y);
    pzd = 0.5 * (da.z + db.z);
    txd = dt.x;
    tyd = dt.y;
    tzd = dt.z;
  }
  double acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  unsigned far_n = 0, near_n = 0;
  const unsigned long long me = 1ull << lane;
  const unsigned long long all = __ballot(act);
  if (lane == 0) {
    st_node[w][0] = 0;
    st_mask[w][0] = all;
  }
  int sp = 1;
  __builtin_amdgcn_wave_barrier();
  while (sp > 0) {
    --sp;
    const int B = __builtin_amdgcn_readfirstlane(st_node[w][sp]);
    const unsigned long long m = st_mask[w][sp];
    __builtin_amdgcn_wave_barrier();
    const int4 nd = node[B];
    const float4 ca = na[B], cb = nb[B];
    const float2 cr = nr[B];
    const bool mine = (m & me) != 0;
    const float dx = mxI - ca.x, dy = myI - ca.y, dz = mzI - ca.z;
    const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
    bool holds_nbr = false;
    for (int q = 0; q < nn; ++q) holds_nbr |= (nbr[q] >= nd.x) & (nbr[q] < nd.x + nd.y);
    const bool adm = mine && !holds_nbr && (cr.x < theta * dist) && (cr.y < theta);
    const unsigned long long admm = __ballot(adm);
    if (adm) {
      float E = 0, S = 0, Gx = 0, Gy = 0, Gz = 0, Gt = 0, Hx = 0, Hy = 0, Hz = 0, Ht = 0;
      tpe_vertex_pair<float, EC, true>(mxI, myI, mzI, tt.x, tt.y, tt.z, ca.x, ca.y, ca.z, cb.x, cb.y, cb.z, false,
                                        ca.w, half_alpha, half_beta, beta, E, S, Gx, Gy, Gz, Gt, Hx, Hy, Hz, Ht,
                                        cb.w);
      acc[0] += E; acc[1] += S; acc[2] += Gx; acc[3] += Gy; acc[4] += Gz;
      acc[5] += Gt; acc[6] += Hx; acc[7] += Hy; acc[8] += Hz; acc[9] += Ht;
      ++far_n;
    }
    const unsigned long long rem = m & ~admm;
    if (rem == 0ull) continue;
    if (nd.z < 0) {
      // leaf: exact edge-midpoint pairs for the lanes still active; chain-near
      // pairs in FP64
      const bool on = (rem & me) != 0;
      float E = 0, S = 0, Gx = 0, Gy = 0, Gz = 0, Gt = 0, Hx = 0, Hy = 0, Hz = 0, Ht = 0;
      double dE = 0, dS = 0, dGx = 0, dGy = 0, dGz = 0, dGt = 0, dHx = 0, dHy = 0, dHz = 0, dHt = 0;
      for (int j = 0; j < nd.y; ++j) {
        const int J = perm[nd.x + j];
        const int2 ej = edges[J];
        const bool excl = (ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y);
        bool near64 = false;
        if constexpr (BAND) near64 = bh_chain_near(ci, cinfo[J]);
        if (near64) {
          const V4<double> qa = DA[J], qb = DB[J], qt = DT[J];
          const double wgt = (on && !excl) ? qa.w : 0.0;
          tpe_vertex_pair<double, EC, true>(pxd, pyd, pzd, txd, tyd, tzd, 0.5 * (qa.x + qb.x), 0.5 * (qa.y + qb.y),
                                            0.5 * (qa.z + qb.z), qt.x, qt.y, qt.z, J == I, wgt, (double)half_alpha,
                                            (double)half_beta, (double)beta, dE, dS, dGx, dGy, dGz, dGt, dHx, dHy,
                                            dHz, dHt);
        } else {
          const V4<float> qa = GA[J], qb = GB[J], qt = GT[J];
          const float wgt = (on && !excl) ? qa.w : 0.f;
          tpe_vertex_pair<float, EC, true>(mxI, myI, mzI, tt.x, tt.y, tt.z, 0.5f * (qa.x + qb.x),
                                            0.5f * (qa.y + qb.y), 0.5f * (qa.z + qb.z), qt.x, qt.y, qt.z, J == I, wgt,
                                            half_alpha, half_beta, beta, E, S, Gx, Gy, Gz, Gt, Hx, Hy, Hz, Ht);
        }
      }
      if (on) {
        acc[0] += E + dE; acc[1] += S + dS; acc[2] += Gx + dGx; acc[3] += Gy + dGy; acc[4] += Gz + dGz;
        acc[5] += Gt + dGt; acc[6] += Hx + dHx; acc[7] += Hy + dHy; acc[8] += Hz + dHz; acc[9] += Ht + dHt;
        near_n += nd.y;
      }
    } else if (sp + 2 <= kStack) {
      if (lane == 0) {
        st_node[w][sp] = nd.z + 1;
        st_mask[w][sp] = rem;
        st_node[w][sp + 1] = nd.z;
        st_mask[w][sp + 1] = rem;
      }
      __builtin_amdgcn_wave_barrier();
      sp += 2;
    }
  }
  if (act) {
#pragma unroll
    for (int k = 0; k < 10; ++k) part[(size_t)k * nE + I] = acc[k];
  }
  atomicAdd(&blk_work[0], (unsigned long long)far_n);
  atomicAdd(&blk_work[1], (unsigned long long)near_n);
  __syncthreads();
  if (threadIdx.x == 0 && work) {
    atomicAdd(&work[0], blk_work[0]);
    atomicAdd(&work[1], blk_work[1]);
  }
}

rc_status Bvh::ensure(int nE_) {
  if (nE == nE_ && perm) return RC_OK;
  release();
  nE = nE_;
  cap = 2 * nE + 2;
  auto al = [](void** p, size_t bytes) {
    return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess;
  };
  if (!al((void**)&perm, sizeof(int) * nE) || !al((void**)&scratch, sizeof(int) * nE) ||
      !al((void**)&pts, sizeof(float) * 6 * (size_t)nE) || !al((void**)&node, sizeof(int4) * cap) ||
      !al((void**)&na, sizeof(float4) * cap) || !al((void**)&nb, sizeof(float4) * cap) ||
      !al((void**)&nr, sizeof(float2) * cap) || !al((void**)&split, sizeof(int) * cap) ||
      !al((void**)&counter, sizeof(int) * 4) || !al((void**)&work, sizeof(unsigned long long) * 2) ||
      !al((void**)&big, sizeof(int) * kBigWords * kBigMaxNodes) ||
      !al((void**)&chunks, sizeof(int4) * (nE / kBigChunk + 2 * kBigMaxNodes))) {
    set_error("BVH allocation failed");
    return RC_ERR_NOMEM;
  }
  return RC_OK;
}

void Bvh::release() {
  void* ps[] = {perm, scratch, pts, node, na, nb, nr, split, counter, work, big, chunks};
  for (void* p : ps)
    if (p) hipFree(p);
  perm = scratch = split = counter = big = nullptr;
  chunks = nullptr;
  pts = nullptr;
  node = nullptr;
  na = nb = nullptr;
  nr = nullptr;
  work = nullptr;
  nE = 0;
}

// One top level by chunks (see k_big_*): nodes of at most `leaf` edges
// become leaves as in k_bvh_split; the others are split by the chunked kernels.
static rc_status split_top_level(Bvh& bvh, int nE, int lb, int count, int leaf, hipStream_t s) {
  std::vector<int4> nodes(count);
  RC_HIP(hipMemcpyAsync(nodes.data(), bvh.node + lb, sizeof(int4) * count, hipMemcpyDeviceToHost, s));
  RC_HIP(hipStreamSynchronize(s));
  std::vector<int4> chunks;
  std::vector<int> flags(count, 0);
  for (int k = 0; k < count; ++k) {
    if (nodes[k].y <= leaf) {
      nodes[k] = make_int4(nodes[k].x, nodes[k].y, -1, 0);
      continue;
    }
    flags[k] = 1;
    for (int o = 0; o < nodes[k].y; o += kBigChunk) chunks.push_back(make_int4(k, o, std::min(kBigChunk, nodes[k].y - o), 0));
  }
  if ((int)chunks.size() > nE / kBigChunk + 2 * kBigMaxNodes) {
    set_error("BVH top-level chunk table overflow");
    return RC_ERR_HIP;
  }
  // leaves of this level are written here; split nodes by k_big_choose
  RC_HIP(hipMemcpyAsync(bvh.split, flags.data(), sizeof(int) * count, hipMemcpyHostToDevice, s));
  for (int k = 0; k < count; ++k)
    if (!flags[k]) RC_HIP(hipMemcpyAsync(bvh.node + lb + k, &nodes[k], sizeof(int4), hipMemcpyHostToDevice, s));
  const int nc = (int)chunks.size();
  if (nc > 0) {
    RC_HIP(hipMemcpyAsync(bvh.chunks, chunks.data(), sizeof(int4) * nc, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_big_init, dim3(count), dim3(256), 0, s, bvh.big, count);
    hipLaunchKernelGGL(k_big_bounds, dim3(nc), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                       bvh.chunks, bvh.big);
    hipLaunchKernelGGL(k_big_hist, dim3(nc), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                       bvh.chunks, bvh.big);
    hipLaunchKernelGGL(k_big_cut, dim3(count), dim3(64), 0, s, bvh.node, lb, bvh.big);
    hipLaunchKernelGGL(k_big_cand, dim3(nc, 6), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                       bvh.chunks, bvh.big);
    // only the split nodes (a leaf has no chunks; its block exits on its flag)
    hipLaunchKernelGGL(k_big_choose_split, dim3(count), dim3(64), 0, s, bvh.node, lb, bvh.big, bvh.split);
    hipLaunchKernelGGL(k_big_count, dim3(nc), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                       bvh.chunks, bvh.big);
    hipLaunchKernelGGL(k_big_scatter, dim3(nc), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                       bvh.chunks, bvh.big, bvh.scratch);
    hipLaunchKernelGGL(k_big_copy, dim3(nc), dim3(256), 0, s, bvh.node, lb, bvh.chunks, bvh.scratch, bvh.perm);
  }
  RC_HIP(hipGetLastError());
  // the host copies above read `nodes` and `flags`: finish them before the vectors go
  RC_HIP(hipStreamSynchronize(s));
  return RC_OK;
}

rc_status build_bvh(const Curve& c, Bvh& bvh, int leaf, hipStream_t s) {
  const int nE = c.nE;
  RC_TRY(bvh.ensure(nE));
  hipLaunchKernelGGL(k_tangent_points, dim3(cdiv(nE, 256)), dim3(256), 0, s, c.gf.a, c.gf.b, c.gf.t, nE, bvh.pts,
                     bvh.perm);
  const int4 root = make_int4(0, nE, -1, 0);
  RC_HIP(hipMemcpyAsync(bvh.node, &root, sizeof(int4), hipMemcpyHostToDevice, s));
  int lb = 0, count = 1, levels = 0;
  while (count > 0) {
    if (lb + 3 * count > bvh.cap || levels > kStack - 4) {
      set_error("BVH deeper or larger than expected");
      return RC_ERR_HIP;
    }
    if (count <= kBigMaxNodes && nE / count >= kBigNode) {
      RC_TRY(split_top_level(bvh, nE, lb, count, leaf, s));
    } else {
      hipLaunchKernelGGL(k_bvh_split, dim3(count), dim3(kBvhThreads), 0, s, bvh.pts, nE, bvh.node, lb, bvh.perm,
                         bvh.scratch, leaf, bvh.split);
    }
    hipLaunchKernelGGL(k_bvh_children, dim3(1), dim3(1024), 0, s, bvh.node, lb, count, bvh.split, lb + count,
                       bvh.counter);
    int next = 0;
    RC_HIP(hipMemcpyAsync(&next, bvh.counter, sizeof(int), hipMemcpyDeviceToHost, s));
    RC_HIP(hipStreamSynchronize(s));
    lb += count;
    count = next;
    ++levels;
  }
  bvh.n_nodes = lb;
  bvh.depth = levels;
  hipLaunchKernelGGL(k_bvh_props, dim3(bvh.n_nodes), dim3(kBvhThreads), 0, s, bvh.pts, c.gf.a, nE, bvh.node,
                     bvh.perm, bvh.na, bvh.nb, bvh.nr);
  hipLaunchKernelGGL(k_invperm, dim3(cdiv(nE, 256)), dim3(256), 0, s, bvh.perm, nE, bvh.scratch);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

// Re-fit (the remark of the paper's conclusion on small time steps): the tree of the last build
// keeps its nodes and their edge sets, and only the node data (centre, length, mean tangent, radii)
// are recomputed from the current edges, in one launch; the admissibility test then reads the
// re-fitted radii, so the traversal stays valid, and its clusters only grow looser as the curve
// moves away from the built one.
rc_status refit_bvh(const Curve& c, Bvh& bvh, hipStream_t s) {
  const int nE = c.nE;
  if (bvh.n_nodes <= 0 || bvh.nE != nE) {
    set_error("BVH re-fit: no tree built for this curve");
    return RC_ERR_ARG;
  }
  hipLaunchKernelGGL(k_tangent_points, dim3(cdiv(nE, 256)), dim3(256), 0, s, c.gf.a, c.gf.b, c.gf.t, nE, bvh.pts,
                     (int*)nullptr);
  hipLaunchKernelGGL(k_bvh_props, dim3(bvh.n_nodes), dim3(kBvhThreads), 0, s, bvh.pts, c.gf.a, nE, bvh.node,
                     bvh.perm, bvh.na, bvh.nb, bvh.nr);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

rc_status launch_bh(const Curve& c, Bvh& bvh, double alpha, double beta, double theta, int leaf, double* energy,
                    double* dE, hipStream_t s, bool refit) {
  const int nE = c.nE;
  if (c.max_degree > 4) {
    set_error("Barnes-Hut needs vertex degree <= 4 (a target keeps at most 6 neighbouring edges)");
    return RC_ERR_UNSUPPORTED;
  }
  if (refit) RC_TRY(refit_bvh(c, bvh, s));
  else RC_TRY(build_bvh(c, bvh, leaf, s));
  RC_HIP(hipMemsetAsync(bvh.work, 0, sizeof(unsigned long long) * 2, s));
  const float ha = (float)(0.5 * alpha), hb = (float)(0.5 * beta), bb = (float)beta, th = (float)theta;
  dim3 g(cdiv(nE, 256)), b(256);
  const bool timed = c.timer && c.timer->on;
  if (timed) c.timer->mark(c.timer->bh, s);
#define RC_BH(EC, BAND)                                                                                            \
  hipLaunchKernelGGL((k_bh_traverse<EC, BAND>), g, b, 0, s, c.gf.a, c.gf.b, c.gf.t, c.gd.a, c.gd.b, c.gd.t, c.edges, \
                     c.inc_off, c.inc, c.cinfo, nE, bvh.perm, bvh.scratch, bvh.node, bvh.na, bvh.nb, bvh.nr, th, ha, \
                     hb, bb, c.part, bvh.work)
#define RC_BH2(EC) \
  if (c.chain) RC_BH(EC, true); else RC_BH(EC, false)
  switch (exp_case(alpha, beta)) {
    case kA2B4: RC_BH2(kA2B4); break;
    case kA2B45: RC_BH2(kA2B45); break;
    case kA3B6: RC_BH2(kA3B6); break;
    default: RC_BH2(kGeneral); break;
  }
#undef RC_BH2
#undef RC_BH
  if (timed) c.timer->mark(c.timer->bh, s);
  RC_HIP(hipGetLastError());
  return finalize_midpoint(c, 1, energy, dE, s);
}

}  // namespace rc
