// Block cluster tree and the 0th-order hierarchical product with the Sobolev
// operator in its kernel-matrix form (App. B.2, App. B.3.4).
//
// A = B + B0 written with edge-by-edge kernel matrices (eqs.
// LowOrderDecomposition, LowOrderKernel):
//   B0 u = E^T (diag(K 1) - K) E u,  K_IJ = (k_{2,2s'}(x_I, x_J, T_I) + k_{2,2s'}(x_J, x_I, T_J)) l_I l_J,
//   B u  = D^T (diag(H 1) - H) D u,  H_IJ = 2 |x_I - x_J|^-(2 sigma + 1) l_I l_J,
// with 2s' = 2 sigma + 5, E the vertex-to-edge average, D the edge
// derivative (D u)_I = (u_i2 - u_i1) / l_I T_I, pairs sharing a vertex left
// out.  The products K psi and H psi are approximated on a block cluster tree:
// blocks (T, S) of BVH nodes, split recursively from (root, root); a block is
// a leaf when it is admissible (eq. BCTAdmissibilityTest:
// max(r_x^T, r_x^S) < theta |c_T - c_S| and max(r_T^T, r_T^S) < theta) or when
// both nodes are BVH leaves; otherwise the larger of the two internal nodes
// (both when both are internal) is split.  An admissible block is the rank-1
// block L_T k(p_T, p_S) L_S^T with the nodes' tangent-points p = (c, Tbar) and
// edge-length vectors L; an inadmissible leaf block is summed exactly, in
// FP64, over its edge pairs.  The condition and the kernels are symmetric in
// (T, S), so the approximate matrices are symmetric.
//
// Product (all sums in FP64, in fixed orders): per-edge right-hand sides
// psi_J = l_J (1, (E u)_J, s_J^c T_J) (13 values, s^c = (u^c_j2 - u^c_j1) / l_J),
// per-node sums Psi_S (contiguous ranges of the BVH permutation, summed bottom-up), per target
// node the admissible blocks' Phi_T = sum_S k(p_T, p_S) Psi_S, pushed down to
// every edge through its ancestors, the exact near blocks per target leaf,
// then the diagonal and off-diagonal parts combined and gathered to vertices.

#include <algorithm>
#include <vector>

#include "pair_math.h"
#include "rc_internal.h"

namespace rc {

static inline int bct_cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr int kPsi = 13;   // 1, E u (3), s^c T (9); times l_J
constexpr int kPhi = 14;   // K: 1, E u (3); H: 1, s^c T (9)
constexpr int kEv = 14;    // per-edge values: w (3), z (9), K1, H1

// Per edge J at BVH position p: psi[p][0..12].
__global__ void k_bct_rhs(const double* __restrict__ X, const int2* __restrict__ edges,
                          const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GT,
                          const int* __restrict__ perm, int nE, double* __restrict__ psi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nE) return;
  const int J = perm[p];
  const int2 e = edges[J];
  const double l = GA[J].w;
  const V4<double> t = GT[J];
  double* o = psi + (size_t)kPsi * p;
  o[0] = l;
  for (int c = 0; c < 3; ++c) {
    const double a = X[3 * e.x + c], b = X[3 * e.y + c];
    o[1 + c] = l * 0.5 * (a + b);
    const double sl = (b - a);  // l * s^c
    o[4 + 3 * c] = sl * t.x;
    o[5 + 3 * c] = sl * t.y;
    o[6 + 3 * c] = sl * t.z;
  }
}

// Psi_S = sum of psi over the node's range, bottom-up: a leaf sums its edges
// in order, an internal node adds its two children (left + right).  The
// schedule is built with the tree: the nodes of each subtree below a cut depth
// go to one workgroup, deepest first, one segment per depth (a barrier
// between segments); the nodes above the cut are a last workgroup of their own,
// run by a second launch.
__global__ __launch_bounds__(256) void k_bct_sums(const int* __restrict__ wseg, const int2* __restrict__ seg,
                                                  const int* __restrict__ ord, int w0, const int4* __restrict__ node,
                                                  const double* __restrict__ psi, double* __restrict__ Psi) {
  const int w = w0 + blockIdx.x;
  for (int g = wseg[w]; g < wseg[w + 1]; ++g) {
    const int2 sg = seg[g];
    const int items = (sg.y - sg.x) * kPsi;
    for (int i = threadIdx.x; i < items; i += blockDim.x) {
      const int n = ord[sg.x + i / kPsi], k = i % kPsi;
      const int4 nd = node[n];
      double a = 0.0;
      if (nd.z < 0)
        for (int q = 0; q < nd.y; ++q) a += psi[(size_t)kPsi * (nd.x + q) + k];
      else
        a = Psi[(size_t)kPsi * nd.z + k] + Psi[(size_t)kPsi * (nd.z + 1) + k];
      Psi[(size_t)kPsi * n + k] = a;
    }
    __syncthreads();  // this depth's sums are read by the next segment
  }
}

// The two kernels between tangent-points (x, T) and (y, U), d = x - y:
// klo = (|T x d|^2 + |U x d|^2) |d|^-(2 sigma + 5), khi = 2 |d|^-(2 sigma + 1);
// the powers of |d|^2 as in the operator's FP64 pair kernel (sob_powers).
template <int EC>
__device__ __forceinline__ void bct_kernels(double dx, double dy, double dz, double tx, double ty, double tz,
                                            double ux, double uy, double uz, double half_expo, double& klo,
                                            double& khi) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double cx = ty * dz - tz * dy, cy = tz * dx - tx * dz, cz = tx * dy - ty * dx;
  const double ex = uy * dz - uz * dy, ey = uz * dx - ux * dz, ez = ux * dy - uy * dx;
  double ri, p;
  sob_powers<EC, double>(r2, half_expo, ri, p);  // ri = |d|^-2, p = |d|^-(2 sigma + 1)
  khi = 2.0 * p;
  klo = (cx * cx + cy * cy + cz * cz + ex * ex + ey * ey + ez * ez) * p * ri * ri;
}

// Phi_T = sum over the admissible blocks (T, S) of klo(T, S) (Psi_S[0..3]) and
// khi(T, S) (Psi_S[0], Psi_S[4..12]); one wave per node, its lanes striding
// over the node's blocks, then a fixed-order wave reduction.
template <int EC>
__global__ __launch_bounds__(256) void k_bct_far(const int* __restrict__ far_off, const int* __restrict__ far_src,
                                                 const float4* __restrict__ na, const float4* __restrict__ nb,
                                                 const double* __restrict__ Psi, int n_nodes, double half_expo,
                                                 double* __restrict__ Phi) {
  const int T = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
  if (T >= n_nodes) return;  // uniform per wave
  double a[kPhi];
  for (int k = 0; k < kPhi; ++k) a[k] = 0.0;
  const float4 ct = na[T], tt = nb[T];
  for (int q = far_off[T] + lane; q < far_off[T + 1]; q += 64) {
    const int S = far_src[q];
    const float4 cs = na[S], ts = nb[S];
    double klo, khi;
    bct_kernels<EC>((double)ct.x - cs.x, (double)ct.y - cs.y, (double)ct.z - cs.z, tt.x, tt.y, tt.z, ts.x, ts.y,
                    ts.z, half_expo, klo, khi);
    const double* P = Psi + (size_t)kPsi * S;
    for (int k = 0; k < 4; ++k) a[k] += klo * P[k];
    a[4] += khi * P[0];
    for (int k = 0; k < 9; ++k) a[5 + k] += khi * P[4 + k];
  }
#pragma unroll
  for (int k = 0; k < kPhi; ++k)
    for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_xor(a[k], o);
  if (lane < kPhi) {
    double v = a[0];
#pragma unroll
    for (int k = 1; k < kPhi; ++k) v = lane == k ? a[k] : v;
    Phi[(size_t)kPhi * T + lane] = v;
  }
}

// phi[p] = l_J (sum of Phi over the ancestors of position p, root included).
__global__ void k_bct_down(const int4* __restrict__ node, const double* __restrict__ Phi,
                           const V4<double>* __restrict__ GA, const int* __restrict__ perm, int nE,
                           double* __restrict__ phi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nE) return;
  double a[kPhi];
  for (int k = 0; k < kPhi; ++k) a[k] = 0.0;
  int B = 0;
  while (true) {
    for (int k = 0; k < kPhi; ++k) a[k] += Phi[(size_t)kPhi * B + k];
    const int4 nd = node[B];
    if (nd.z < 0) break;
    const int4 left = node[nd.z];
    B = (p < left.x + left.y) ? nd.z : nd.z + 1;
  }
  const double l = GA[perm[p]].w;
  for (int k = 0; k < kPhi; ++k) phi[(size_t)kPhi * p + k] = l * a[k];
}

// Exact near blocks.  A task is a target leaf T (at most 32 edges) with a
// run of at most kTaskBlocks of its near source leaves; a leaf with a longer
// near list is split over several tasks (workgroups), whose partial sums go
// to their own slots and are added in task order afterwards.  Per round the
// workgroup stages up to eight source leaves as one flat list of at most 256
// source edges in LDS; a thread per target edge in each of eight groups of 32
// sweeps its group's equal share of that list; the eight partial sums are
// added in group order.
constexpr int kNearGroups = 8;
constexpr int kTaskRounds = 4;
constexpr int kTaskBlocks = kNearGroups * kTaskRounds;
constexpr int kStage = kNearGroups * 32;
constexpr int kSrcVals = 6 + kPsi;  // x (3), T (3), psi
template <int EC>
__global__ __launch_bounds__(256) void k_bct_near(const int4* __restrict__ task, const int* __restrict__ near_src,
                                                  const int* __restrict__ leaf_node, const int4* __restrict__ node,
                                                  const int* __restrict__ perm, const int2* __restrict__ edges,
                                                  const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                                                  const V4<double>* __restrict__ GT, const double* __restrict__ psi,
                                                  double half_expo, double* __restrict__ phi,
                                                  double* __restrict__ part) {
  static_assert(kNearGroups * 32 * kPhi <= kStage * kSrcVals, "the group sums reuse the staging memory");
  __shared__ double sd[kStage * kSrcVals];
  __shared__ int2 se[kStage];
  __shared__ int soff[kNearGroups + 1], sbeg[kNearGroups];
  const int4 tk = task[blockIdx.x];  // (leaf index, first block, end block, partial slot or -1)
  const int4 tn = node[leaf_node[tk.x]];
  const int grp = threadIdx.x / 32, tid = threadIdx.x % 32;
  const bool act = tid < tn.y;
  const int p = tn.x + (act ? tid : 0);
  const int I = perm[p];
  const V4<double> a = GA[I], b = GB[I], t = GT[I];
  const double x0 = 0.5 * (a.x + b.x), x1 = 0.5 * (a.y + b.y), x2 = 0.5 * (a.z + b.z);
  const int2 ei = edges[I];
  double acc[kPhi];
  for (int k = 0; k < kPhi; ++k) acc[k] = 0.0;
  for (int q = tk.y; q < tk.z; q += kNearGroups) {
    const int nb = min(kNearGroups, tk.z - q);
    __syncthreads();  // the previous round's list is no longer read
    if (threadIdx.x == 0) {
      int o = 0;
      for (int j = 0; j < nb; ++j) {
        const int4 sn = node[near_src[q + j]];
        soff[j] = o;
        sbeg[j] = sn.x;
        o += sn.y;
      }
      soff[nb] = o;
    }
    __syncthreads();
    const int m = soff[nb];  // <= 8 leaves of <= 32 edges
    if ((int)threadIdx.x < m) {
      int j = 0;
      while ((int)threadIdx.x >= soff[j + 1]) ++j;
      const int pj = sbeg[j] + (int)threadIdx.x - soff[j];
      const int J = perm[pj];
      const V4<double> qa = GA[J], qb = GB[J], qt = GT[J];
      double* d = sd + kSrcVals * threadIdx.x;
      d[0] = 0.5 * (qa.x + qb.x);
      d[1] = 0.5 * (qa.y + qb.y);
      d[2] = 0.5 * (qa.z + qb.z);
      d[3] = qt.x;
      d[4] = qt.y;
      d[5] = qt.z;
      for (int k = 0; k < kPsi; ++k) d[6 + k] = psi[(size_t)kPsi * pj + k];
      se[threadIdx.x] = edges[J];
    }
    __syncthreads();
    const int share = (m + kNearGroups - 1) / kNearGroups;
    const int u1 = min(m, (grp + 1) * share);
    if (act)
      for (int u = grp * share; u < u1; ++u) {
        const int2 ej = se[u];
        if ((ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y)) continue;
        const double* d = sd + kSrcVals * u;
        double klo, khi;
        bct_kernels<EC>(x0 - d[0], x1 - d[1], x2 - d[2], t.x, t.y, t.z, d[3], d[4], d[5], half_expo, klo, khi);
        for (int k = 0; k < 4; ++k) acc[k] += klo * d[6 + k];
        acc[4] += khi * d[6];
        for (int k = 0; k < 9; ++k) acc[5 + k] += khi * d[10 + k];
      }
  }
  __syncthreads();
  double* red = sd;  // [group][target][kPhi]
  for (int k = 0; k < kPhi; ++k) red[(threadIdx.x) * kPhi + k] = acc[k];
  __syncthreads();
  if (grp == 0 && act) {
    for (int k = 0; k < kPhi; ++k) {
      double v = red[tid * kPhi + k];
      for (int g = 1; g < kNearGroups; ++g) v += red[(g * 32 + tid) * kPhi + k];
      if (tk.w < 0)
        phi[(size_t)kPhi * p + k] += a.w * v;
      else
        part[((size_t)tk.w * 32 + tid) * kPhi + k] = v;
    }
  }
}

// Leaves whose near list spans several tasks: phi += l_I (sum of the tasks'
// partial sums, in task order).  red[r] = (leaf index, first slot, slots).
__global__ void k_bct_near_sum(const int4* __restrict__ red, int n_red, const int* __restrict__ leaf_node,
                               const int4* __restrict__ node, const int* __restrict__ perm,
                               const V4<double>* __restrict__ GA, const double* __restrict__ part,
                               double* __restrict__ phi) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_red * 32) return;
  const int4 r = red[i / 32];
  const int tid = i % 32;
  const int4 tn = node[leaf_node[r.x]];
  if (tid >= tn.y) return;
  const int p = tn.x + tid;
  const double l = GA[perm[p]].w;
  for (int k = 0; k < kPhi; ++k) {
    double v = 0.0;
    int j = 0;
    for (; j + 8 <= r.z; j += 8) {  // eight loads in flight, added in slot order
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = part[((size_t)(r.y + j + u) * 32 + tid) * kPhi + k];
#pragma unroll
      for (int u = 0; u < 8; ++u) v += t[u];
    }
    for (; j < r.z; ++j) v += part[((size_t)(r.y + j) * 32 + tid) * kPhi + k];
    phi[(size_t)kPhi * p + k] += l * v;
  }
}

// Per edge: the kernel-matrix form's edge values (B0 part w (3), B part z^c (3 x 3))
// and the row sums: out[I] = (w (3), z (9), (K1)_I, (H1)_I) with
// w = (K1) (E u) - K E u and z^c = (H1) s^c T - H (s^c T).
__global__ void k_bct_edge_vals(const double* __restrict__ phi, const int* __restrict__ perm, const double* __restrict__ X,
                                const int2* __restrict__ edges, const V4<double>* __restrict__ GA,
                                const V4<double>* __restrict__ GT, int nE, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nE) return;
  const int I = perm[p];
  const int2 e = edges[I];
  const double l = GA[I].w;
  const V4<double> t = GT[I];
  const double* f = phi + (size_t)kPhi * p;
  double* o = out + kEv * (size_t)I;
  o[12] = f[0];
  o[13] = f[4];
  const double tv[3] = {t.x, t.y, t.z};
  for (int c = 0; c < 3; ++c) {
    const double a = X[3 * e.x + c], b = X[3 * e.y + c];
    o[c] = f[0] * 0.5 * (a + b) - f[1 + c];
    const double s = (b - a) / l;
    for (int k = 0; k < 3; ++k) o[3 + 3 * c + k] = f[4] * s * tv[k] - f[5 + 3 * c + k];
  }
}

// Y_v = sum over incident edges of E^T w (1/2 w) and D^T z (+-T.z / l); with
// diag, the diagonal of the same operator: the diagonal of E^T (diag(K1) - K) E
// is 1/4 sum_{I at v} (K1)_I and that of D^T (diag(H1) - H) D is
// sum_{I at v} (H1)_I / l_I^2 (K and H vanish on pairs sharing v).
__global__ void k_bct_gather(const double* __restrict__ ev, const int* __restrict__ inc_off,
                             const int* __restrict__ inc, const V4<double>* __restrict__ GA,
                             const V4<double>* __restrict__ GT, int nV, double* __restrict__ Y,
                             double* __restrict__ diag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nV) return;
  double y[3] = {0.0, 0.0, 0.0}, dg = 0.0;
  for (int q = inc_off[v]; q < inc_off[v + 1]; ++q) {
    const int code = inc[q], I = code >> 1;
    const double sg = (code & 1) ? 1.0 : -1.0;
    const double* o = ev + kEv * (size_t)I;
    const double l = GA[I].w;
    const V4<double> t = GT[I];
    for (int c = 0; c < 3; ++c) {
      const double tz = t.x * o[3 + 3 * c] + t.y * o[4 + 3 * c] + t.z * o[5 + 3 * c];
      y[c] += 0.5 * o[c] + sg * tz / l;
    }
    dg += 0.25 * o[12] + o[13] / (l * l);
  }
  for (int c = 0; c < 3; ++c) Y[3 * v + c] = y[c];
  if (diag) diag[v] = dg;
}

// ---------------------------------------------------------------------------
// host side: block lists from the BVH's node data
// ---------------------------------------------------------------------------
rc_status Bct::ensure(int nE_, int nodes_) {
  if (nE == nE_ && cap_nodes >= nodes_ && psi) return RC_OK;
  release();
  auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess; };
  if (!al((void**)&psi, sizeof(double) * kPsi * (size_t)nE_) || !al((void**)&phi, sizeof(double) * kPhi * (size_t)nE_) ||
      !al((void**)&ev, sizeof(double) * kEv * (size_t)nE_) || !al((void**)&Psi, sizeof(double) * kPsi * (size_t)nodes_) ||
      !al((void**)&Phi, sizeof(double) * kPhi * (size_t)nodes_)) {
    release();
    set_error("allocation of the block cluster tree failed");
    return RC_ERR_NOMEM;
  }
  nE = nE_;
  cap_nodes = nodes_;
  return RC_OK;
}

void Bct::release() {
  void* ps[] = {psi, phi, ev, Psi, Phi, part, far_off, far_src, near_off, near_src, leaf_node, wseg, ord, task, red, seg};
  for (void* p : ps)
    if (p) hipFree(p);
  psi = phi = ev = Psi = Phi = part = nullptr;
  far_off = far_src = near_off = near_src = leaf_node = wseg = ord = nullptr;
  task = red = nullptr;
  seg = nullptr;
  nE = cap_nodes = n_far = n_near = n_leaves = n_tasks = n_red = n_sub = 0;
  near_pairs = 0;
  ready = false;
}

rc_status build_bct(const Curve& c, Bvh& bvh, Bct& bct, double theta, int leaf, hipStream_t s) {
  RC_TRY(build_bvh(c, bvh, leaf, s));
  const int nn = bvh.n_nodes;
  std::vector<int4> node(nn);
  std::vector<float4> na(nn);
  std::vector<float2> nr(nn);
  RC_HIP(hipMemcpyAsync(node.data(), bvh.node, sizeof(int4) * nn, hipMemcpyDeviceToHost, s));
  RC_HIP(hipMemcpyAsync(na.data(), bvh.na, sizeof(float4) * nn, hipMemcpyDeviceToHost, s));
  RC_HIP(hipMemcpyAsync(nr.data(), bvh.nr, sizeof(float2) * nn, hipMemcpyDeviceToHost, s));
  RC_HIP(hipStreamSynchronize(s));
  // split (root, root) breadth first; blocks go to the target node's lists
  std::vector<std::vector<int>> far(nn), nearl(nn);
  std::vector<int2> cur{make_int2(0, 0)}, next;
  long long pairs = 0;
  const float th = (float)theta;
  while (!cur.empty()) {
    next.clear();
    for (const int2 blk : cur) {
      const int T = blk.x, S = blk.y;
      const float4 ct = na[T], cs = na[S];
      const float dx = ct.x - cs.x, dy = ct.y - cs.y, dz = ct.z - cs.z;
      const float dist = std::sqrt(dx * dx + dy * dy + dz * dz);
      const bool adm = T != S && std::max(nr[T].x, nr[S].x) < th * dist && std::max(nr[T].y, nr[S].y) < th;
      if (adm) {
        far[T].push_back(S);
        continue;
      }
      const bool lt = node[T].z < 0, ls = node[S].z < 0;
      if (lt && ls) {
        nearl[T].push_back(S);
        pairs += (long long)node[T].y * node[S].y;
        continue;
      }
      // split the internal side(s): both when both are internal
      const int t0 = lt ? T : node[T].z, t1 = lt ? T : node[T].z + 1;
      const int s0 = ls ? S : node[S].z, s1 = ls ? S : node[S].z + 1;
      next.push_back(make_int2(t0, s0));
      if (s1 != s0) next.push_back(make_int2(t0, s1));
      if (t1 != t0) {
        next.push_back(make_int2(t1, s0));
        if (s1 != s0) next.push_back(make_int2(t1, s1));
      }
    }
    cur.swap(next);
  }
  std::vector<int> foff(nn + 1, 0), fsrc, noff(1, 0), nsrc, lnode;
  for (int T = 0; T < nn; ++T) {
    foff[T + 1] = foff[T] + (int)far[T].size();
    fsrc.insert(fsrc.end(), far[T].begin(), far[T].end());
    if (node[T].z < 0) {
      lnode.push_back(T);
      nsrc.insert(nsrc.end(), nearl[T].begin(), nearl[T].end());
      noff.push_back((int)nsrc.size());
    }
  }
  // node-sum schedule: depths (children follow their parents in node order),
  // the cut at the first depth with at least 256 nodes, one workgroup per
  // subtree below it and a last one for the nodes above it
  std::vector<int> depth(nn, 0), sub(nn, -1), per_depth;
  for (int T = 0; T < nn; ++T) {
    if ((int)per_depth.size() <= depth[T]) per_depth.resize(depth[T] + 1, 0);
    ++per_depth[depth[T]];
    if (node[T].z >= 0) depth[node[T].z] = depth[node[T].z + 1] = depth[T] + 1;
  }
  const int maxd = (int)per_depth.size() - 1;
  int cut = maxd + 1;
  for (int d = 0; d <= maxd; ++d)
    if (per_depth[d] >= 256) {
      cut = d;
      break;
    }
  int nsub = 0;
  for (int T = 0; T < nn; ++T) {
    if (depth[T] == cut) sub[T] = nsub++;
    if (node[T].z >= 0 && sub[T] >= 0) sub[node[T].z] = sub[node[T].z + 1] = sub[T];
  }
  std::vector<std::vector<std::vector<int>>> by(nsub + 1, std::vector<std::vector<int>>(maxd + 1));
  for (int T = 0; T < nn; ++T) by[sub[T] >= 0 ? sub[T] : nsub][depth[T]].push_back(T);
  std::vector<int> wseg(1, 0), ord;
  std::vector<int2> segs;
  for (int w = 0; w <= nsub; ++w) {
    for (int d = maxd; d >= 0; --d)
      if (!by[w][d].empty()) {
        segs.push_back(make_int2((int)ord.size(), (int)(ord.size() + by[w][d].size())));
        ord.insert(ord.end(), by[w][d].begin(), by[w][d].end());
      }
    wseg.push_back((int)segs.size());
  }
  // near tasks: leaves with more than kTaskBlocks near blocks first, split
  // into runs with a partial slot each; then one task per remaining leaf
  std::vector<int4> tasks, reds;
  int slots = 0;
  const int nl = (int)lnode.size();
  for (int li = 0; li < nl; ++li) {
    const int q0 = noff[li], q1 = noff[li + 1];
    if (q1 - q0 <= kTaskBlocks) continue;
    const int nt = (q1 - q0 + kTaskBlocks - 1) / kTaskBlocks;
    reds.push_back(make_int4(li, slots, nt, 0));
    for (int j = 0; j < nt; ++j)
      tasks.push_back(make_int4(li, q0 + j * kTaskBlocks, std::min(q1, q0 + (j + 1) * kTaskBlocks), slots++));
  }
  for (int li = 0; li < nl; ++li)
    if (noff[li + 1] > noff[li] && noff[li + 1] - noff[li] <= kTaskBlocks)
      tasks.push_back(make_int4(li, noff[li], noff[li + 1], -1));
  RC_TRY(bct.ensure(c.nE, nn));
  void* ps[] = {bct.far_off, bct.far_src, bct.near_off, bct.near_src, bct.leaf_node, bct.wseg, bct.ord,
                bct.task, bct.red, bct.part, bct.seg};
  for (void* p : ps)
    if (p) hipFree(p);
  bct.far_off = bct.far_src = bct.near_off = bct.near_src = bct.leaf_node = bct.wseg = bct.ord = nullptr;
  bct.task = bct.red = nullptr;
  bct.seg = nullptr;
  bct.part = nullptr;
  auto up = [&](auto** dst, const auto& v) -> rc_status {
    using T = typename std::decay_t<decltype(v)>::value_type;
    if (hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(v.size(), 1)) != hipSuccess) {
      set_error("allocation of the block lists failed");
      return RC_ERR_NOMEM;
    }
    if (!v.empty()) RC_HIP(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return RC_OK;
  };
  RC_TRY(up(&bct.far_off, foff));
  RC_TRY(up(&bct.far_src, fsrc));
  RC_TRY(up(&bct.near_off, noff));
  RC_TRY(up(&bct.near_src, nsrc));
  RC_TRY(up(&bct.leaf_node, lnode));
  RC_TRY(up(&bct.task, tasks));
  RC_TRY(up(&bct.red, reds));
  RC_TRY(up(&bct.wseg, wseg));
  RC_TRY(up(&bct.seg, segs));
  RC_TRY(up(&bct.ord, ord));
  bct.n_sub = nsub;
  if (hipMalloc((void**)&bct.part, sizeof(double) * kPhi * 32 * std::max(slots, 1)) != hipSuccess) {
    set_error("allocation of the block lists failed");
    return RC_ERR_NOMEM;
  }
  bct.n_nodes = nn;
  bct.n_far = (int)fsrc.size();
  bct.n_near = (int)nsrc.size();
  bct.n_leaves = nl;
  bct.n_tasks = (int)tasks.size();
  bct.n_red = (int)reds.size();
  bct.near_pairs = pairs;
  bct.theta = theta;
  bct.ready = true;
  return RC_OK;
}

rc_status launch_bct_apply(const Curve& c, const Bvh& bvh, Bct& bct, double alpha, double beta, const double* X,
                           double* Y, hipStream_t s, double* diag) {
  if (!bct.ready) {
    set_error("block cluster tree not built");
    return RC_ERR_ARG;
  }
  const int nE = c.nE;
  const double sigma = (beta - 1.0) / alpha - 1.0;
  const double half_expo = 0.5 * (2.0 * sigma + 1.0);
  const V4<double>*GA = c.gd.a, *GB = c.gd.b, *GT = c.gd.t;
  hipLaunchKernelGGL(k_bct_rhs, dim3(bct_cdiv(nE, 256)), dim3(256), 0, s, X, (const int2*)c.edges, GA, GT,
                     (const int*)bvh.perm, nE, bct.psi);
  if (bct.n_sub > 0)
    hipLaunchKernelGGL(k_bct_sums, dim3(bct.n_sub), dim3(256), 0, s, (const int*)bct.wseg, (const int2*)bct.seg,
                       (const int*)bct.ord, 0, (const int4*)bvh.node, (const double*)bct.psi, bct.Psi);
  hipLaunchKernelGGL(k_bct_sums, dim3(1), dim3(256), 0, s, (const int*)bct.wseg, (const int2*)bct.seg,
                     (const int*)bct.ord, bct.n_sub, (const int4*)bvh.node, (const double*)bct.psi, bct.Psi);
  auto far_near = [&](auto ec) {
    constexpr int EC = decltype(ec)::value;
    hipLaunchKernelGGL((k_bct_far<EC>), dim3(bct_cdiv(bct.n_nodes, 4)), dim3(256), 0, s, (const int*)bct.far_off,
                       (const int*)bct.far_src, (const float4*)bvh.na, (const float4*)bvh.nb,
                       (const double*)bct.Psi, bct.n_nodes, half_expo, bct.Phi);
    hipLaunchKernelGGL(k_bct_down, dim3(bct_cdiv(nE, 256)), dim3(256), 0, s, (const int4*)bvh.node,
                       (const double*)bct.Phi, GA, (const int*)bvh.perm, nE, bct.phi);
    if (bct.n_tasks > 0)
      hipLaunchKernelGGL((k_bct_near<EC>), dim3(bct.n_tasks), dim3(256), 0, s, (const int4*)bct.task,
                         (const int*)bct.near_src, (const int*)bct.leaf_node, (const int4*)bvh.node,
                         (const int*)bvh.perm, (const int2*)c.edges, GA, GB, GT, (const double*)bct.psi, half_expo,
                         bct.phi, bct.part);
    if (bct.n_red > 0)
      hipLaunchKernelGGL(k_bct_near_sum, dim3(bct_cdiv(bct.n_red * 32, 256)), dim3(256), 0, s, (const int4*)bct.red,
                         bct.n_red, (const int*)bct.leaf_node, (const int4*)bvh.node, (const int*)bvh.perm, GA,
                         (const double*)bct.part, bct.phi);
  };
  switch (exp_case(alpha, beta)) {
    case kA2B4: far_near(std::integral_constant<int, kA2B4>{}); break;
    case kA2B45: far_near(std::integral_constant<int, kA2B45>{}); break;
    default: far_near(std::integral_constant<int, kGeneral>{}); break;
  }
  hipLaunchKernelGGL(k_bct_edge_vals, dim3(bct_cdiv(nE, 256)), dim3(256), 0, s, (const double*)bct.phi,
                     (const int*)bvh.perm, X, (const int2*)c.edges, GA, GT, nE, bct.ev);
  hipLaunchKernelGGL(k_bct_gather, dim3(bct_cdiv(c.nV, 256)), dim3(256), 0, s, (const double*)bct.ev,
                     (const int*)c.inc_off, (const int*)c.inc, GA, GT, c.nV, Y, diag);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
