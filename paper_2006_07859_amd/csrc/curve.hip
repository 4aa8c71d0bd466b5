// Curve record: topology, incidence and the device buffers of one level.

#include <algorithm>
#include <cstring>
#include <string>

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

// Chains of a degree <= 2 graph: vertex and edge sequences of every component
// (of the kept edges' subgraph when keep is given).
std::vector<Chain> chains_of(const Curve& c, const std::vector<char>* keep) {
  std::vector<Chain> out;
  std::vector<char> used(c.nE, 0), seen(c.nV, 0);
  if (keep)
    for (int I = 0; I < c.nE; ++I) used[I] = (*keep)[I] ? 0 : 1;
  auto kept_degree = [&](int v) {
    int d = 0;
    for (int k = c.h_inc_off[v]; k < c.h_inc_off[v + 1]; ++k) d += keep ? ((*keep)[c.h_inc[k] >> 1] ? 1 : 0) : 1;
    return d;
  };
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
      const int deg = kept_degree(v0);
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

// Arcs of any graph: the maximal paths whose interior vertices have degree 2,
// from a vertex of another degree (a junction or an end) to the next one (the
// same vertex for an arc that closes on itself), then the components without
// such vertices as closed loops.  For degree <= 2 graphs, chains_of.
std::vector<Chain> arcs_of(const Curve& c) {
  if (c.chain) return chains_of(c);
  std::vector<Chain> out;
  std::vector<char> used(c.nE, 0);
  auto deg = [&](int v) { return c.h_inc_off[v + 1] - c.h_inc_off[v]; };
  auto other = [&](int I, int v) { return c.h_edges[2 * I] == v ? c.h_edges[2 * I + 1] : c.h_edges[2 * I]; };
  for (int v0 = 0; v0 < c.nV; ++v0) {
    if (deg(v0) == 2 || deg(v0) == 0) continue;
    for (int k0 = c.h_inc_off[v0]; k0 < c.h_inc_off[v0 + 1]; ++k0) {
      int I = c.h_inc[k0] >> 1;
      if (used[I]) continue;
      Chain ch;
      ch.verts.push_back(v0);
      int v = v0;
      while (true) {
        used[I] = 1;
        ch.edges.push_back(I);
        const int w = other(I, v);
        ch.verts.push_back(w);
        if (deg(w) != 2) break;
        int next = -1;
        for (int k = c.h_inc_off[w]; k < c.h_inc_off[w + 1]; ++k)
          if ((c.h_inc[k] >> 1) != I) next = c.h_inc[k] >> 1;
        v = w;
        I = next;
      }
      out.push_back(std::move(ch));
    }
  }
  std::vector<char> keep(c.nE);
  for (int I = 0; I < c.nE; ++I) keep[I] = used[I] ? 0 : 1;
  for (Chain& ch : chains_of(c, &keep)) out.push_back(std::move(ch));
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
  part_chunks = nchunk + 1;
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

rc_status Curve::set_instances(int n_inst_, const int* voff_h) {
  if (n_inst_ < 1) {
    set_error("a batch needs at least one instance");
    return RC_ERR_ARG;
  }
  h_inst_voff.assign(voff_h, voff_h + n_inst_ + 1);
  if (h_inst_voff[0] != 0 || h_inst_voff[n_inst_] != nV) {
    set_error("instance vertex offsets must start at 0 and end at the vertex count");
    return RC_ERR_ARG;
  }
  for (int i = 0; i < n_inst_; ++i)
    if (h_inst_voff[i + 1] <= h_inst_voff[i]) {
      set_error("instance vertex offsets must increase");
      return RC_ERR_ARG;
    }
  // edges must be grouped by instance, in instance order, and stay inside it
  std::vector<int> vinst(nV);
  for (int i = 0; i < n_inst_; ++i)
    for (int v = h_inst_voff[i]; v < h_inst_voff[i + 1]; ++v) vinst[v] = i;
  std::vector<int> einst(nE);
  h_inst_eoff.assign(n_inst_ + 1, 0);
  for (int I = 0; I < nE; ++I) {
    const int a = vinst[h_edges[2 * I]], b = vinst[h_edges[2 * I + 1]];
    if (a != b) {
      set_error("edge " + std::to_string(I) + " joins two instances");
      return RC_ERR_ARG;
    }
    if (I > 0 && a < einst[I - 1]) {
      set_error("edges must be grouped by instance in instance order");
      return RC_ERR_ARG;
    }
    einst[I] = a;
    h_inst_eoff[a + 1]++;
  }
  for (int i = 0; i < n_inst_; ++i) {
    if (h_inst_eoff[i + 1] == 0) {
      set_error("instance " + std::to_string(i) + " has no edges");
      return RC_ERR_ARG;
    }
    h_inst_eoff[i + 1] += h_inst_eoff[i];
  }
  n_inst = n_inst_;
  RC_TRY(dmalloc(&inst_voff, n_inst + 1));
  RC_TRY(dmalloc(&inst_eoff, n_inst + 1));
  RC_TRY(dmalloc(&inst_of_edge, nE));
  RC_TRY(dmalloc(&inst_of_vertex, nV));
  RC_TRY(dmalloc(&nch_e, nE));
  RC_TRY(dmalloc(&counter, 4));
  RC_HIP(hipMemcpy(inst_voff, h_inst_voff.data(), sizeof(int) * (n_inst + 1), hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(inst_eoff, h_inst_eoff.data(), sizeof(int) * (n_inst + 1), hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(inst_of_edge, einst.data(), sizeof(int) * nE, hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(inst_of_vertex, vinst.data(), sizeof(int) * nV, hipMemcpyHostToDevice));
  return build_items(1024, 8);
}

// Work items of the batch pair kernels for source chunks of src_chunk edges;
// blocks_per_cu_ workgroups per compute unit in the persistent launches.
rc_status Curve::build_items(int src_chunk, int blocks_per_cu_) {
  if (src_chunk < kTile || src_chunk > (1 << 20) || blocks_per_cu_ < 1 || blocks_per_cu_ > 32) {
    set_error("batch tiling out of range");
    return RC_ERR_ARG;
  }
  struct It {
    int4 w;
    long long cost;
  };
  std::vector<It> list;
  std::vector<int> nch(nE);
  int nmax = 1;
  for (int i = 0; i < n_inst; ++i) {
    const int e0 = h_inst_eoff[i], e1 = h_inst_eoff[i + 1];
    const int nc = (e1 - e0 + src_chunk - 1) / src_chunk;
    if (nc >= (1 << 15)) {
      set_error("instance too large for the batch tiling");
      return RC_ERR_ARG;
    }
    nmax = std::max(nmax, nc);
    for (int I = e0; I < e1; ++I) nch[I] = nc;
    for (int t0 = e0; t0 < e1; t0 += kTile) {
      const int tc = std::min(kTile, e1 - t0);
      for (int c = 0; c < nc; ++c) {
        const int s0 = e0 + c * src_chunk, s1 = std::min(e1, s0 + src_chunk);
        list.push_back({make_int4(t0, s0, s1, (c << 16) | tc), (long long)tc * (s1 - s0)});
      }
    }
  }
  std::stable_sort(list.begin(), list.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  std::vector<int4> h(list.size());
  for (size_t k = 0; k < list.size(); ++k) h[k] = list[k].w;
  if (items) hipFree(items);
  items = nullptr;
  n_items = (int)h.size();
  RC_TRY(dmalloc(&items, std::max<size_t>(h.size(), 1)));
  RC_HIP(hipMemcpy(items, h.data(), sizeof(int4) * h.size(), hipMemcpyHostToDevice));
  RC_HIP(hipMemcpy(nch_e, nch.data(), sizeof(int) * nE, hipMemcpyHostToDevice));
  nchunk = nmax;
  item_src = src_chunk;
  if (part_chunks < nchunk + 1) {
    hipFree(part);
    part = nullptr;
    const int slots = std::max(kTpeSlots, std::max(kSobSlots, 10));
    RC_TRY(dmalloc(&part, (size_t)(nchunk + 1) * slots * nE));
    part_chunks = nchunk + 1;
  }
  int dev = 0, ncu = 0;
  RC_HIP(hipGetDevice(&dev));
  RC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  blocks_per_cu = blocks_per_cu_;
  persist_blocks = std::max(1, ncu * blocks_per_cu);
  return RC_OK;
}

rc_status Curve::enable_vertex_pairs() {
  if (vinfo) {  // buffers kept from an earlier enable
    vp = true;
    return RC_OK;
  }
  if (!chain || n_inst > 0) {
    set_error("the vertex-pair form needs a single network of vertex degree <= 2");
    return RC_ERR_UNSUPPORTED;
  }
  std::vector<int4> hv(nV);
  for (int v = 0; v < nV; ++v) hv[v] = make_int4(-1 - v, 0, 1, 0);  // isolated vertex: a chain of its own
  std::vector<Chain> chs = chains_of(*this);
  std::vector<int> hc;  // the chains' vertices in order; a chain is named by its start in hc
  hc.reserve(nV);
  for (size_t k = 0; k < chs.size(); ++k) {
    const int m = (int)chs[k].verts.size(), start = (int)hc.size();
    for (int p = 0; p < m; ++p) {
      hv[chs[k].verts[p]] = make_int4(start, p, m, chs[k].loop ? 1 : 0);
      hc.push_back(chs[k].verts[p]);
    }
  }
  // source chunks: about 4,096 workgroups (16 per compute unit); at 16,384 vertices one source tile
  // per chunk (measured on one MI355X: 0.384 ms per energy + differential launch against 0.416 ms
  // with 2,048 workgroups and 0.453 ms with 1,024; 8,192 gave no more)
  const int tb = (nV + kTile - 1) / kTile;
  vchunk = std::max(1, std::min(tb, (4096 + tb - 1) / tb));
  vsrc_per_chunk = (nV + vchunk - 1) / vchunk;
  RC_TRY(dmalloc(&vinfo, nV));
  RC_TRY(dmalloc(&vchain, std::max<size_t>(1, hc.size())));
  for (int k = 0; k < 3; ++k) RC_TRY(dmalloc(&vg[k], nV));
  for (int k = 0; k < 3; ++k) RC_TRY(dmalloc(&vgd[k], nV));
  RC_TRY(dmalloc(&vpart, (size_t)vchunk * kVpSlots * nV));
  RC_TRY(dmalloc(&vband, (size_t)kVpSlots * nV));
  RC_TRY(dmalloc(&vout, (size_t)kVpOut * nV));
  RC_HIP(hipMemcpy(vinfo, hv.data(), sizeof(int4) * nV, hipMemcpyHostToDevice));
  if (!hc.empty()) RC_HIP(hipMemcpy(vchain, hc.data(), sizeof(int) * hc.size(), hipMemcpyHostToDevice));
  vp = true;
  return RC_OK;
}

void Curve::release() {
  void* ptrs[] = {edges, inc_off, inc, gf.a, gf.b, gf.t, gd.a, gd.b, gd.t,
                  rhs_f[0], rhs_f[1], rhs_d[0], rhs_d[1], part, edge_out, red, cinfo, chain_edge,
                  inst_voff, inst_eoff, inst_of_edge, inst_of_vertex, items, nch_e, counter,
                  vinfo, vchain, vg[0], vg[1], vg[2], vgd[0], vgd[1], vgd[2], vpart, vband, vout};
  for (void* p : ptrs)
    if (p) hipFree(p);
  spot.release();
  vp = false;
  vinfo = nullptr;
  vchain = nullptr;
  vg[0] = vg[1] = vg[2] = nullptr;
  vgd[0] = vgd[1] = vgd[2] = nullptr;
  vpart = nullptr;
  vband = nullptr;
  vout = nullptr;
  inst_voff = inst_eoff = inst_of_edge = inst_of_vertex = nch_e = counter = nullptr;
  items = nullptr;
  n_inst = n_items = 0;
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
