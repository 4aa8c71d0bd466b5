// Curve record: topology, incidence and the device buffers of one level.

#include <algorithm>
#include <cstring>

#include "rc_internal.h"

namespace rc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

template <typename T>
static rc_status dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * n);
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    return RC_ERR_NOMEM;
  }
  return RC_OK;
}

// Chains of a degree <= 2 graph: vertex and edge sequences of every component.
std::vector<Chain> chains_of(const Curve& c) {
  std::vector<Chain> out;
  std::vector<char> used(c.nE, 0), seen(c.nV, 0);
  auto other = [&](int I, int v) { return c.h_edges[2 * I] == v ? c.h_edges[2 * I + 1] : c.h_edges[2 * I]; };
  auto next_edge = [&](int v, int prevI) {
    for (int k = c.h_inc_off[v]; k < c.h_inc_off[v + 1]; ++k) {
      int I = c.h_inc[k] >> 1;
      if (I != prevI && !used[I]) return I;
    }
    return -1;
  };
  // open paths start at degree-1 vertices
  for (int pass = 0; pass < 2; ++pass) {
    for (int v0 = 0; v0 < c.nV; ++v0) {
      const int deg = c.h_inc_off[v0 + 1] - c.h_inc_off[v0];
      if (seen[v0] || deg == 0) continue;
      if (pass == 0 && deg != 1) continue;
      Chain ch;
      ch.verts.push_back(v0);
      seen[v0] = 1;
      int v = v0, prevI = -1;
      while (true) {
        int I = next_edge(v, prevI);
        if (I < 0) break;
        used[I] = 1;
        ch.edges.push_back(I);
        int w = other(I, v);
        if (w == v0) {
          ch.loop = true;
          break;
        }
        ch.verts.push_back(w);
        seen[w] = 1;
        v = w;
        prevI = I;
      }
      out.push_back(std::move(ch));
    }
  }
  return out;
}


rc_status Curve::init(int nV_, int nE_, const int* edges_h) {
  nV = nV_;
  nE = nE_;
  h_edges.assign(edges_h, edges_h + 2 * (size_t)nE);
  // incidence CSR, entries 2*edge + endpoint
  std::vector<int> deg(nV, 0);
  for (int I = 0; I < nE; ++I) {
    deg[h_edges[2 * I]]++;
    deg[h_edges[2 * I + 1]]++;
  }
  h_inc_off.assign(nV + 1, 0);
  for (int v = 0; v < nV; ++v) h_inc_off[v + 1] = h_inc_off[v] + deg[v];
  h_inc.assign(2 * (size_t)nE, 0);
  std::vector<int> fill(h_inc_off.begin(), h_inc_off.end() - 1);
  for (int I = 0; I < nE; ++I)
    for (int a = 0; a < 2; ++a) h_inc[fill[h_edges[2 * I + a]]++] = 2 * I + a;
  max_degree = nV ? *std::max_element(deg.begin(), deg.end()) : 0;
  chain = max_degree <= 2;

  // source chunks: enough workgroups to fill 256 CUs several times over
  const int tblocks = (nE + kTile - 1) / kTile;
  nchunk = std::max(1, std::min(tblocks, (2048 + tblocks - 1) / tblocks));
  src_per_chunk = (nE + nchunk - 1) / nchunk;
  red_blocks = std::max(1, std::min(256, (nE + 255) / 256));

  RC_TRY(dmalloc(&edges, nE));
  RC_TRY(dmalloc(&inc_off, nV + 1));
  RC_TRY(dmalloc(&inc, 2 * (size_t)nE));
  RC_HIP(hipMemcpy(edges, h_edges.data(), sizeof(int) * 2 * nE, hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(inc_off, h_inc_off.data(), sizeof(int) * (nV + 1), hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(inc, h_inc.data(), sizeof(int) * 2 * nE, hipMemcpyHostToDevice));
  RC_TRY(dmalloc(&gf.a, nE));
  RC_TRY(dmalloc(&gf.b, nE));
  RC_TRY(dmalloc(&gf.t, nE));
  RC_TRY(dmalloc(&gd.a, nE));
  RC_TRY(dmalloc(&gd.b, nE));
  RC_TRY(dmalloc(&gd.t, nE));
  for (int k = 0; k < 2; ++k) {
    RC_TRY(dmalloc(&rhs_f[k], nE));
    RC_TRY(dmalloc(&rhs_d[k], nE));
  }
  const int slots = std::max(kTpeSlots, std::max(kSobSlots, 10));
  RC_TRY(dmalloc(&part, (size_t)(nchunk + 1) * slots * nE));  // + one chunk for the FP64 near band
  RC_TRY(dmalloc(&edge_out, 8 * (size_t)nE));
  RC_TRY(dmalloc(&red, 256));
  // chain position of every edge: near pairs along a chain are evaluated in FP64
  if (chain) {
    std::vector<Chain> chs = chains_of(*this);
    std::vector<int4> info(nE, make_int4(-1, 0, 0, 0));
    std::vector<int> order;
    for (int q = 0; q < (int)chs.size(); ++q) {
      const int start = (int)order.size();
      const int m = (int)chs[q].edges.size();
      for (int p = 0; p < m; ++p) {
        info[chs[q].edges[p]] = make_int4(start, p, m, chs[q].loop ? 1 : 0);
        order.push_back(chs[q].edges[p]);
      }
    }
    RC_TRY(dmalloc(&cinfo, nE));
    RC_TRY(dmalloc(&chain_edge, nE));
    RC_HIP(hipMemcpy(cinfo, info.data(), sizeof(int4) * nE, hipMemcpyHostToDevice));
    RC_HIP(hipMemcpy(chain_edge, order.data(), sizeof(int) * nE, hipMemcpyHostToDevice));
  }
  return RC_OK;
}

void Curve::release() {
  void* ptrs[] = {edges, inc_off, inc, gf.a, gf.b, gf.t, gd.a, gd.b, gd.t,
                  rhs_f[0], rhs_f[1], rhs_d[0], rhs_d[1], part, edge_out, red, cinfo, chain_edge};
  for (void* p : ptrs)
    if (p) hipFree(p);
  edges = nullptr;
  inc_off = inc = nullptr;
  gf = EdgeGeom<float>();
  gd = EdgeGeom<double>();
  rhs_f[0] = rhs_f[1] = nullptr;
  rhs_d[0] = rhs_d[1] = nullptr;
  part = edge_out = red = nullptr;
  cinfo = nullptr;
  chain_edge = nullptr;
}

}  // namespace rc
