// Triangulated-surface potential (Sec. 7.1, surface potential): the double
// integral of |x_M - gamma|^-(beta - alpha) over the curve and a triangulated
// surface M, with one sample per edge (midpoint x_I, weight l_I) and one per
// triangle (centroid c_T, weight A_T):
//   E_M = sum_I l_I phi(x_I),   phi(x) = sum_T A_T |c_T - x|^-p,
// and its differential: at the edge's ends -+T_I phi(x_I) + (l_I / 2) grad phi,
// grad phi(x) = p sum_T A_T |c_T - x|^(-p-2) (c_T - x).
//
// The surface does not move, so its tree is built once on the host: median
// splits of the triangle centroids along the longest side of their bounding
// box, leaves of at most 8 triangles, each node with its area-weighted centre
// c_B, total area A_B and the radius r_B of a sphere around c_B holding all of
// its triangles.  One thread per edge walks the tree depth first: a node with
// r_B < theta |c_B - x_I| contributes A_B |c_B - x_I|^-p (the Barnes-Hut
// far-field rule of App. B.1 for this potential), a leaf otherwise sums its
// triangles; theta = 0 sums every triangle (the oracle's definition exactly).
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "rc_internal.h"

namespace rc {

namespace {

constexpr int kSpLeaf = 8;    // triangles per leaf at most
constexpr int kSpStack = 64;  // traversal stack (the tree's depth + 1 at most; checked at build)

struct __align__(16) SpNode {
  double cx, cy, cz, area, radius;
  int child;  // leaf: first triangle; inner node: first of its two children (stored together)
  int count;  // triangles of a leaf, 0 for an inner node
};

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// the node's contribution A |d|^-p and its gradient term p A |d|^(-p-2) d, d = c - x
__device__ __forceinline__ void sp_term(double A, double dx, double dy, double dz, double p, double& phi,
                                        double& g0, double& g1, double& g2) {
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double q = A * pow(d2, -0.5 * p);
  const double f = p * q / d2;
  phi += q;
  g0 += f * dx;
  g1 += f * dy;
  g2 += f * dz;
}

__global__ void k_surface_potential(const V4<double>* __restrict__ GA, const V4<double>* __restrict__ GB,
                                    const V4<double>* __restrict__ GT, int nE, const SpNode* __restrict__ nodes,
                                    const double* __restrict__ tris, double p, double w, double theta2, int grad,
                                    double* __restrict__ edge_out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const V4<double> a = GA[I], b = GB[I], t = GT[I];
  const double x0 = 0.5 * (a.x + b.x), x1 = 0.5 * (a.y + b.y), x2 = 0.5 * (a.z + b.z);
  double phi = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
  int stack[kSpStack];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const SpNode nd = nodes[stack[--sp]];
    const double dx = nd.cx - x0, dy = nd.cy - x1, dz = nd.cz - x2;
    if (nd.radius * nd.radius < theta2 * (dx * dx + dy * dy + dz * dz)) {  // far: the node as one sample
      sp_term(nd.area, dx, dy, dz, p, phi, g0, g1, g2);
    } else if (nd.count > 0) {  // a near leaf: its triangles
      for (int k = nd.child; k < nd.child + nd.count; ++k) {
        const double* tr = tris + 4 * (size_t)k;
        sp_term(tr[3], tr[0] - x0, tr[1] - x1, tr[2] - x2, p, phi, g0, g1, g2);
      }
    } else {
      stack[sp++] = nd.child;
      stack[sp++] = nd.child + 1;
    }
  }
  const double l = a.w;
  double* o = edge_out + 8 * (size_t)I;
  o[0] += w * l * phi;
  if (!grad) return;
  const double h = 0.5 * w * l;
  const double tp0 = w * t.x * phi, tp1 = w * t.y * phi, tp2 = w * t.z * phi;
  o[1] += -tp0 + h * g0;
  o[2] += -tp1 + h * g1;
  o[3] += -tp2 + h * g2;
  o[4] += tp0 + h * g0;
  o[5] += tp1 + h * g1;
  o[6] += tp2 + h * g2;
}

}  // namespace

void SurfacePotential::release() {
  if (nodes) hipFree(nodes);
  if (tris) hipFree(tris);
  nodes = nullptr;
  tris = nullptr;
  on = false;
  n_nodes = nF = depth = 0;
}

rc_status build_surface_potential(SurfacePotential& sp, const double* P_h, int nP, const int* F_h, int nF) {
  std::vector<double> c(3 * (size_t)nF), A(nF);
  for (int f = 0; f < nF; ++f) {
    const double* v[3] = {P_h + 3 * (size_t)F_h[3 * f], P_h + 3 * (size_t)F_h[3 * f + 1],
                          P_h + 3 * (size_t)F_h[3 * f + 2]};
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    A[f] = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int k = 0; k < 3; ++k) c[3 * f + k] = (v[0][k] + v[1][k] + v[2][k]) / 3.0;
  }
  (void)nP;
  std::vector<int> idx(nF);
  for (int f = 0; f < nF; ++f) idx[f] = f;
  std::vector<SpNode> nodes(1);
  int depth = 0;
  std::function<void(int, int, int, int)> fill = [&](int slot, int lo, int hi, int d) {
    depth = std::max(depth, d);
    double area = 0.0, m[3] = {0.0, 0.0, 0.0}, lo3[3] = {INFINITY, INFINITY, INFINITY},
           hi3[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = lo; k < hi; ++k) {
      const int f = idx[k];
      area += A[f];
      for (int q = 0; q < 3; ++q) {
        m[q] += A[f] * c[3 * f + q];
        lo3[q] = std::min(lo3[q], c[3 * f + q]);
        hi3[q] = std::max(hi3[q], c[3 * f + q]);
      }
    }
    double ctr[3];
    for (int q = 0; q < 3; ++q) ctr[q] = area > 0.0 ? m[q] / area : 0.5 * (lo3[q] + hi3[q]);
    double r2 = 0.0;
    for (int k = lo; k < hi; ++k)
      for (int j = 0; j < 3; ++j) {
        const double* v = P_h + 3 * (size_t)F_h[3 * idx[k] + j];
        const double d0 = v[0] - ctr[0], d1 = v[1] - ctr[1], d2 = v[2] - ctr[2];
        r2 = std::max(r2, d0 * d0 + d1 * d1 + d2 * d2);
      }
    SpNode nd{ctr[0], ctr[1], ctr[2], area, std::sqrt(r2), lo, hi - lo};
    if (hi - lo <= kSpLeaf) {
      nodes[slot] = nd;
      return;
    }
    int ax = 0;
    for (int q = 1; q < 3; ++q)
      if (hi3[q] - lo3[q] > hi3[ax] - lo3[ax]) ax = q;
    const int mid = lo + (hi - lo) / 2;
    std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi,
                     [&](int f, int g) { return c[3 * f + ax] < c[3 * g + ax]; });
    const int ch = (int)nodes.size();
    nodes.resize(ch + 2);
    nd.child = ch;
    nd.count = 0;
    nodes[slot] = nd;
    fill(ch, lo, mid, d + 1);
    fill(ch + 1, mid, hi, d + 1);
  };
  fill(0, 0, nF, 0);
  if (depth + 2 > kSpStack) {
    set_error("surface potential: triangle tree too deep");
    return RC_ERR_UNSUPPORTED;
  }
  std::vector<double> tr(4 * (size_t)nF);
  for (int k = 0; k < nF; ++k) {
    const int f = idx[k];
    tr[4 * k] = c[3 * f];
    tr[4 * k + 1] = c[3 * f + 1];
    tr[4 * k + 2] = c[3 * f + 2];
    tr[4 * k + 3] = A[f];
  }
  sp.release();
  RC_HIP(hipMalloc(&sp.nodes, sizeof(SpNode) * nodes.size()));
  RC_HIP(hipMalloc((void**)&sp.tris, sizeof(double) * tr.size()));
  RC_HIP(hipMemcpy(sp.nodes, nodes.data(), sizeof(SpNode) * nodes.size(), hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(sp.tris, tr.data(), sizeof(double) * tr.size(), hipMemcpyHostToDevice));
  sp.n_nodes = (int)nodes.size();
  sp.nF = nF;
  sp.depth = depth;
  return RC_OK;
}

rc_status launch_surface_potential(const Curve& c, bool grad, hipStream_t s) {
  const SurfacePotential& sp = c.spot;
  hipLaunchKernelGGL(k_surface_potential, dim3(cdiv(c.nE, 128)), dim3(128), 0, s, (const V4<double>*)c.gd.a,
                     (const V4<double>*)c.gd.b, (const V4<double>*)c.gd.t, c.nE, (const SpNode*)sp.nodes, sp.tris,
                     sp.p, sp.w, sp.theta * sp.theta, grad ? 1 : 0, c.edge_out);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
