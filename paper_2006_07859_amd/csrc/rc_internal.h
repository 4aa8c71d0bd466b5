// Internal declarations of librcurves: device data layout, the curve record
// shared by the finest level and the multigrid levels, and the launchers
// implemented in the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rcurves.h"

namespace rc {

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error();

#define RC_HIP(call)                                                          \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::rc::set_error(std::string(#call " failed: ") + hipGetErrorString(e_)); \
      return RC_ERR_HIP;                                                      \
    }                                                                         \
  } while (0)

#define RC_TRY(expr)                     \
  do {                                   \
    rc_status s_ = (expr);               \
    if (s_ != RC_OK) return s_;          \
  } while (0)

// ---------------------------------------------------------------------------
// data layout
// ---------------------------------------------------------------------------
// Per-edge geometry in the pair kernels' precision R, structure of arrays of
// 4-vectors so that one source edge is three aligned 16/32-byte loads:
//   a[I] = (x_i1, l_I)   b[I] = (x_i2, 0)   t[I] = (T_I, 0)
// plus the endpoint indices ids[I] = (i1, i2).
template <typename R>
struct __align__(4 * sizeof(R)) V4 {
  R x, y, z, w;
};

template <typename R>
struct EdgeGeom {
  V4<R>* a = nullptr;
  V4<R>* b = nullptr;
  V4<R>* t = nullptr;
};

// Partial sums written by the pair kernels: [chunk][slot][edge] doubles.
constexpr int kTile = 256;        // threads (= target edges) per pair block
constexpr int kSub = 64;          // sources folded into FP64 accumulators at a time
constexpr int kTpeSlots = 14;     // energy + differential accumulators
constexpr int kSobSlots = 8;      // operator accumulators
constexpr int kMidSlots = 8;      // midpoint energy + differential accumulators
constexpr int kVpSlots = 17;      // vertex-pair energy + differential accumulators
constexpr int kVpOut = 12;        // per-vertex finalised values

// Exponent cases compiled as specialisations; anything else takes the
// general exp2/log2 path.
enum ExpCase : int { kGeneral = 0, kA2B4 = 1, kA2B45 = 2, kA3B6 = 3 };
ExpCase exp_case(double alpha, double beta);

// Components of a graph whose vertices have degree <= 2: loops and open paths.
struct Chain {
  std::vector<int> verts;  // v_0 .. (loop: m vertices, path: m+1 vertices)
  std::vector<int> edges;  // e_k joins verts[k] and verts[k+1 (mod m for loops)]
  bool loop = false;
};
struct Curve;
// Chains of a degree <= 2 graph; with keep, of the subgraph of the kept edges
// (whose vertices must have at most two kept edges).
std::vector<Chain> chains_of(const Curve& c, const std::vector<char>* keep = nullptr);
// Arcs between vertices of degree != 2 (and closed loops) of any graph.
std::vector<Chain> arcs_of(const Curve& c);

// Pairs of edges at most kBand apart along a chain are evaluated in FP64 by
// the near-band kernel when the pair kernels run in FP32 (see k_pairs.hip).
constexpr int kBand = 32;

// Conditions latched into a context's device status word (bitwise OR, read and
// cleared by rc_sync_status).  The kernels that detect them set their bit with
// an atomic OR; the host-side solver conditions are kept in a host word of the
// context and merged when the status is read.
enum StatusFlag : uint32_t {
  kFlagInputNonfinite = RC_FLAG_INPUT_NONFINITE,
  kFlagZeroEdge = RC_FLAG_ZERO_EDGE,
  kFlagPairOverflow = RC_FLAG_PAIR_OVERFLOW,
  kFlagResultNonfinite = RC_FLAG_RESULT_NONFINITE,
};
__device__ __forceinline__ void latch(unsigned* status, unsigned flag) {
  if (status) atomicOr(status, flag);
}

// Optional HIP-event timing of the pair kernels (enabled per context).
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> tpe, sob, lowp, asm32, sob64, basm, bh;  // start/stop pairs, in launch order
  // timing-only events: no system-scope fence (no cache writeback and invalidation between the kernels
  // they bracket); elapsed times are read after the stream has been synchronised
  void mark(std::vector<hipEvent_t>& v, hipStream_t s) {
    if (!on) return;
    hipEvent_t e;
    hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    hipEventRecord(e, s);
    v.push_back(e);
  }
  void clear() {
    for (hipEvent_t e : tpe) hipEventDestroy(e);
    for (hipEvent_t e : sob) hipEventDestroy(e);
    for (hipEvent_t e : lowp) hipEventDestroy(e);
    for (hipEvent_t e : asm32) hipEventDestroy(e);
    for (hipEvent_t e : sob64) hipEventDestroy(e);
    for (hipEvent_t e : basm) hipEventDestroy(e);
    for (hipEvent_t e : bh) hipEventDestroy(e);
    bh.clear();
    sob64.clear();
    basm.clear();
    tpe.clear();
    sob.clear();
    lowp.clear();
    asm32.clear();
  }
};

// Sphere-obstacle penalty (Sec. 7.1, surface potential with M a sphere):
// E_M = w sum_I l_I Psi(|x_I - c|), Psi the closed-form shell potential of
// exponent p = beta - alpha.
struct Obstacle {
  bool on = false;
  double c[3] = {0, 0, 0};
  double R = 0, p = 0, w = 0;
};

// Penalties of Sec. 7.1 added to the energy: w_len sum_I l_I (total length),
// w_diff sum over degree-2 vertices of (l_I - l_J)^2 (length difference) and
// w_field sum_I l_I |T_I x X|^2 for a constant unit vector X (field potential).
struct Penalties {
  bool on = false;
  double w_len = 0, w_diff = 0, w_field = 0;
  double X[3] = {0, 0, 1};
};

// Triangulated-surface potential of Sec. 7.1: weight w times sum_I l_I phi(x_I),
// phi(x) = sum_T A_T |c_T - x|^-p (p = beta - alpha; edge midpoints x_I,
// triangle centroids c_T and areas A_T), summed over a bounding-sphere tree of
// the triangles built once on the host (the surface does not move): a node
// whose sphere of radius r around its area-weighted centre c_B satisfies
// r < theta |c_B - x| contributes A_B |c_B - x|^-p; theta = 0 sums every
// triangle.
struct SurfacePotential {
  bool on = false;
  double w = 0, p = 0, theta = 0;
  int n_nodes = 0, nF = 0, depth = 0;
  void* nodes = nullptr;   // [n_nodes] tree nodes (k_surfpot.hip)
  double* tris = nullptr;  // [nF][4] centroid, area, in leaf order
  void release();
};

// A curve network on the device (the finest level, or a multigrid level).
struct Curve {
  int nV = 0, nE = 0;
  std::vector<int> h_edges;        // [nE][2]
  int2* edges = nullptr;           // device copy
  int* inc_off = nullptr;          // [nV+1] CSR: vertex -> incident (edge, endpoint)
  int* inc = nullptr;              // entries 2*edge + a (a = 0 for i1, 1 for i2)
  std::vector<int> h_inc_off, h_inc;
  bool chain = false;              // every vertex has degree <= 2
  int max_degree = 0;

  EdgeGeom<float> gf;
  EdgeGeom<double> gd;
  V4<float>* rhs_f[2] = {nullptr, nullptr};   // per-edge operator inputs (s_J, ubar_J)
  V4<double>* rhs_d[2] = {nullptr, nullptr};

  int4* cinfo = nullptr;           // per edge (chain start, position, chain length, is loop); chain graphs only
  int* chain_edge = nullptr;       // edges in chain order (cinfo.x + position -> edge)

  // Vertex-pair form of the alpha = 2 energy + differential (chain graphs,
  // FP32; enable_vertex_pairs): per vertex (chain start in vchain, position,
  // vertex count, is loop; an isolated vertex v has chain -1 - v), the chains'
  // vertices in order (vchain), the FP32 and FP64 vertex geometry (x_v,
  // Lambda_v), u_0, u_1 (sqrt(l) T of the vertex's incident edges in
  // incidence order), the FP32 chunk partial sums [vchunk][kVpSlots][nV], the
  // FP64 near-band sums [kVpSlots][nV] and the finalised per-vertex values
  // [nV][kVpOut].
  bool vp = false;
  int4* vinfo = nullptr;
  int* vchain = nullptr;
  V4<float>* vg[3] = {nullptr, nullptr, nullptr};
  V4<double>* vgd[3] = {nullptr, nullptr, nullptr};
  float* vpart = nullptr;
  double* vband = nullptr;
  double* vout = nullptr;
  int vchunk = 1, vsrc_per_chunk = 0;
  rc_status enable_vertex_pairs();

  KernelTimer* timer = nullptr;    // set on the finest level when profiling is on
  unsigned* status = nullptr;      // the context's device status word (not owned); null on coarse levels
  const struct Bvh* hbvh = nullptr; // when set (with hbct): the solver applies this level's operator as the
  struct Bct* hbct = nullptr;       // block-cluster-tree product of that tree (not owned)

  int nchunk = 1, src_per_chunk = 0;
  int part_chunks = 0;             // chunks part has room for (the near band uses chunk nchunk)
  double* part = nullptr;          // pair-kernel partials, sized for the largest slot count
  double* edge_out = nullptr;      // per-edge finalised values [nE][8]
  double* red = nullptr;           // reduction scratch
  int red_blocks = 0;

  // Batch of independent instances (n_inst > 0): the vertices and edges of
  // instance i are contiguous, and the pair kernels sum over pairs of one
  // instance only, as work items (target tile, source range) of a persistent
  // launch.  nchunk is then the largest chunk count of an instance and nch_e
  // gives every edge its instance's count.
  int n_inst = 0;
  std::vector<int> h_inst_voff, h_inst_eoff;
  int *inst_voff = nullptr, *inst_eoff = nullptr, *inst_of_edge = nullptr, *inst_of_vertex = nullptr;
  int4* items = nullptr;           // (t0, s0, s1, chunk << 16 | tcount), longest first
  int n_items = 0, item_src = 0, persist_blocks = 0, blocks_per_cu = 0;
  int* nch_e = nullptr;
  int* counter = nullptr;
  const int* inst_mask = nullptr;  // when set, work items of instances with mask 0 are skipped
  Obstacle obstacle;               // applied by launch_tpe when on
  Penalties pen;                   // applied by launch_tpe when on
  SurfacePotential spot;           // applied by launch_tpe when on

  rc_status init(int nV_, int nE_, const int* edges_h);
  rc_status set_instances(int n_inst_, const int* voff_h);
  rc_status build_items(int src_chunk, int blocks_per_cu_);
  void release();
};

// ---------------------------------------------------------------------------
// launchers (k_pairs.hip)
// ---------------------------------------------------------------------------
// Edge geometry from the FP64 state, rounded to the kernel precision.
rc_status launch_geometry(const Curve& c, const double* gamma, rc_dtype prec, hipStream_t s);
// Energy (and differential): writes energy[0] and, when dE != nullptr, dE[nV][3].
rc_status launch_tpe(const Curve& c, double alpha, double beta, rc_dtype prec, bool grad,
                     double* energy, double* dE, hipStream_t s);
// Y = Abar X (matrix-free); when diag != nullptr also writes diag(A).
rc_status launch_sobolev(const Curve& c, double alpha, double beta, rc_dtype prec,
                         const double* X, double* Y, double* diag, hipStream_t s);
// Exact edge-midpoint energy and differential.
rc_status launch_midpoint(const Curve& c, double alpha, double beta, rc_dtype prec,
                          double* energy, double* dE, hipStream_t s);
// First collision time (k_ccd.hip): per-edge FP64 endpoints and velocities,
// FP32 swept boxes and the 64-bit minimum.
struct CcdBuffers {
  V4<double>*p1 = nullptr, *p2 = nullptr, *w1 = nullptr, *w2 = nullptr;
  float4 *lo = nullptr, *hi = nullptr;
  unsigned long long* bits = nullptr;
  double* t = nullptr;
  int nE = 0;
  rc_status ensure(int nE_);
  void release();
};
// t_out (device) = the first t in (0, T] at which two edges sharing no vertex
// of gamma - t D touch, or +inf.
rc_status launch_first_collision(const Curve& c, const double* gamma, const double* D, double T, CcdBuffers& buf,
                                 double* t_out, hipStream_t s);

// Vertex-pair form (k_vpairs.hip): per-vertex FP32 geometry from the FP64
// edge geometry, and the energy (and differential) of an alpha = 2 chain graph
// in FP32 with the FP64 near band; called by launch_tpe when c.vp is set.
// The FP32 vertex-pair sums and the FP64 near band (part chunk 0), then,
// after the band's edge finalize, the vertex finalize, the edge partials and
// the gather into dE.
rc_status launch_tpe_vp_pairs(const Curve& c, double beta, bool grad, hipStream_t s);
// Adds the penalties (c.pen) to the per-edge energy / endpoint-derivative slots of edge_out.
rc_status launch_penalties(const Curve& c, bool grad, hipStream_t s);
// k_surfpot.hip: the tree of a triangulated surface (host P [nP][3], F [nF][3]) and the potential's
// per-edge energy and endpoint derivatives added to c.edge_out
rc_status build_surface_potential(SurfacePotential& sp, const double* P_h, int nP, const int* F_h, int nF);
rc_status launch_surface_potential(const Curve& c, bool grad, hipStream_t s);
rc_status launch_tpe_vp_finish(const Curve& c, double beta, bool grad, double* dE, double* energy_partial,
                               hipStream_t s);
// Shared tail of the edge-midpoint kernels: sums nparts chunks of the
// 10-slot partials, writes energy and dE.
rc_status finalize_midpoint(const Curve& c, int nparts, double* energy, double* dE, hipStream_t s);

// Device BVH over tangent-points for Barnes-Hut (k_bvh.hip).
struct Bvh {
  int nE = 0, cap = 0, n_nodes = 0, depth = 0;
  int *perm = nullptr, *scratch = nullptr, *split = nullptr, *counter = nullptr;
  float* pts = nullptr;
  int4* node = nullptr;
  float4 *na = nullptr, *nb = nullptr;
  float2* nr = nullptr;
  unsigned long long* work = nullptr;  // far-field and near-field interaction counts of the last traversal
  int* big = nullptr;                   // accumulators of the multi-workgroup split of the top levels
  int4* chunks = nullptr;               // its chunk table
  rc_status ensure(int nE_);
  void release();
};
// Block cluster tree over a BVH (k_bct.hip): per-edge and per-node sums of the
// hierarchical product and the block lists (far blocks per target node,
// near source leaves per target leaf).
struct Bct {
  int nE = 0, cap_nodes = 0, n_nodes = 0, n_far = 0, n_near = 0, n_leaves = 0, n_tasks = 0, n_red = 0, n_sub = 0;
  long long near_pairs = 0;
  double theta = 0.0;
  bool ready = false;
  double *psi = nullptr, *phi = nullptr, *ev = nullptr, *Psi = nullptr, *Phi = nullptr;
  double* part = nullptr;  // partial near sums of leaves split over several tasks
  int *far_off = nullptr, *far_src = nullptr, *near_off = nullptr, *near_src = nullptr, *leaf_node = nullptr;
  int *wseg = nullptr, *ord = nullptr;  // node-sum schedule: segments per workgroup, nodes per segment
  int2* seg = nullptr;
  int4 *task = nullptr, *red = nullptr;  // near tasks and the split leaves' partial-sum runs
  rc_status ensure(int nE_, int nodes_);
  void release();
};
// Builds the BVH (nodes of at most leaf <= 32 edges) and the block cluster
// tree of admissibility parameter theta at the curve's loaded geometry.
rc_status build_bct(const Curve& c, Bvh& bvh, Bct& bct, double theta, int leaf, hipStream_t s);
// Y = A^ X, the 0th-order hierarchical product with the kernel-matrix form of
// A = B + B0 (needs the FP64 geometry of the build loaded).
// diag (optional, [nV]): the diagonal of that approximate A, from the same row
// sums (diag_v = 1/4 sum_{I at v} (K 1)_I + sum_{I at v} (H 1)_I / l_I^2).
rc_status launch_bct_apply(const Curve& c, const Bvh& bvh, Bct& bct, double alpha, double beta, const double* X,
                           double* Y, hipStream_t s, double* diag = nullptr);

// Builds the BVH of the curve's current FP32 geometry (nodes of at most leaf
// edges; node data and the inverse permutation in bvh.scratch).
rc_status build_bvh(const Curve& c, Bvh& bvh, int leaf, hipStream_t s);
constexpr int kStepBhLeaf = 32;  // leaf size of the Barnes-Hut evaluations inside rc_step
// Barnes-Hut energy and differential in FP32 (needs the FP32 geometry).
rc_status launch_bh(const Curve& c, Bvh& bvh, double alpha, double beta, double theta, int leaf, double* energy,
                    double* dE, hipStream_t s, bool refit = false);

// Per-edge sums Wq, P0 of the operator kernel into edge_out slots 0 and 1
// (they do not depend on the vector the operator is applied to).
rc_status launch_edge_sums(const Curve& c, double alpha, double beta, rc_dtype prec, hipStream_t s);

// Dense FP64 A (row-major nV x nV); needs degree <= 2.
rc_status launch_assemble_dense(const Curve& c, double alpha, double beta, double* A,
                                hipStream_t s);

// Assembled Sobolev block (k_lowp.hip): Jacobi-scaled off-diagonal tiles in
// MFMA operand order, rounded to 16 bits (fmt 1 = BF16, 2 = FP16) and
// optionally also kept in FP32, an FP32 band along the chains and, for each
// stored version, a diagonal recomputed in FP64 from the stored rows.
constexpr int kLowpMaxBand = 64;
struct LowpOp {
  int n = 0, fmt = 0, band = 0;
  bool with32 = false;
  int nrb = 0, nkt = 0, ngroups = 0, nsplit = 1, per = 0;  // column-tile splits of the 16-bit product
  int ngroups_used = 0;  // column-tile groups of the last assembly (rows of rowpart it wrote)
  int nsplit32 = 1, per32 = 0;                               // and of the FP32 product
  void* tiles = nullptr;        // [nrb][nkt][64 lanes] 16-byte vectors of 8 16-bit values
  void* tiles32 = nullptr;      // [nrb][nkt][64 lanes] 8 floats
  double *rowpart = nullptr, *rowpart32 = nullptr, *dvec = nullptr, *sqd = nullptr;
  double *sigma = nullptr, *sigma32 = nullptr;  // diagonals balancing the tile entries (band excluded)
  double *bandpart = nullptr, *mx = nullptr, *cref = nullptr;
  float *pbuf = nullptr, *sqdf = nullptr, *part = nullptr, *band_val = nullptr;
  int4* vinfo = nullptr;        // per vertex (chain, position, vertex count, is loop)
  int* band_idx = nullptr;      // [n][2 band]
  bool ready = false;
  rc_status ensure(const Curve& c, int fmt_, int band_, bool with32_);
  void release();
  size_t tile_bytes() const { return (size_t)nrb * nkt * 1024; }
};
// Builds the blocks of the curve's current geometry (FP32 and FP64 copies
// must be loaded); diag_out (optional, [nV]) receives the diagonal of the
// 16-bit operator.
rc_status launch_assemble_lowp(const Curve& c, LowpOp& op, int fmt, int band, bool with32, double alpha,
                               double beta, double* diag_out, hipStream_t s);
// Y = A^ X with the 16-bit block (apply) or the FP32 block (apply32); X and Y
// [nV][3] FP64.  The product kernels are timed when the timer is on.
// Y = A X, or Y = base + alpha A X when base is given (Y may alias base).
// prepped: the product's operand (pbuf, cref) already holds X in its
// difference form, written by the launch that produced X.
rc_status launch_lowp_apply(const LowpOp& op, const double* X, double* Y, hipStream_t s, KernelTimer* timer,
                            const double* base = nullptr, double alpha = 1.0, bool prepped = false);
rc_status launch_lowp_apply32(const LowpOp& op, const double* X, double* Y, hipStream_t s, KernelTimer* timer);

// Learned multilevel preconditioner (k_learn.hip): the MLP and the features.
constexpr int kMlpIn = 8, kMlpWidth = 64;
constexpr int kMlpParams = kMlpIn * kMlpWidth + kMlpWidth + kMlpWidth * kMlpWidth + kMlpWidth + kMlpWidth + 1;
struct Mlp {
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *opart = nullptr;
  _Float16* w16 = nullptr;
  float *H1 = nullptr, *H2 = nullptr, *O = nullptr, *Do = nullptr, *D1 = nullptr, *D2 = nullptr;
  float *Y = nullptr, *dY = nullptr;
  int cap = 0, t = 0;
  hipStream_t stream = nullptr;
  rc_status init(const float* theta_h, hipStream_t s);
  rc_status set(const float* theta_h);
  rc_status ensure_rows(int N);
  void release();
};
rc_status mlp_forward(Mlp& M, const float* X, int N, float* Y, bool keep, hipStream_t s);
rc_status mlp_backward(Mlp& M, const float* X, int N, const float* dY, float* grad, hipStream_t s);
rc_status mlp_adam(Mlp& M, const float* grad, float lr, hipStream_t s);
// Features of one level (a loop numbered along itself) into X [n][8];
// scratch holds 9 n + 2 doubles.
rc_status launch_level_features(const Curve& cv, const double* gam, const double* diag, double* scratch, float* X,
                                hipStream_t s);
// r[v] = sum_w |A_vw| / A_vv and sc[v] = (sum_w |A_vw|)^-1/2 for a dense FP64
// n x n matrix; y = diag(sc) A diag(sc) x; x = the alternating vector;
// T = r lambda[0] (float).
rc_status launch_row_l1_ratio(const double* A, int n, double* r, double* sc, hipStream_t s);
rc_status launch_sym_scaled_mv(const double* A, const double* sc, const double* x, int n, double* y, hipStream_t s);
rc_status launch_alternating(int n, double* x, hipStream_t s);
rc_status launch_ratio_targets(const double* r, const double* lam, int n, float* T, hipStream_t s);
// diag[v] *= margin (1 + Y[v]): the learned smoother diagonal.
rc_status launch_learned_diag(const float* Y, int n, double margin, double* diag, hipStream_t s);
// One regression step of the MLP on (X, R) (see k_learn.hip); loss_dev: device double.
rc_status mlp_fit_step(Mlp& M, const float* X, const float* R, int N, float lr, double* loss_dev, float* grad_out,
                       hipStream_t s);

// ---------------------------------------------------------------------------
// dense and vector helpers (k_linalg.hip)
// ---------------------------------------------------------------------------
// All vectors are double; n counts doubles.
void vec_axpby(double a, const double* x, double b, double* y, int n, hipStream_t s);  // y = a x + b y
void vec_copy(const double* x, double* y, int n, hipStream_t s);
void vec_scale_diag_inv(const double* r, const double* d, double* z, int nV, hipStream_t s); // z = r / d (3 comps)
// result[0] = x . y (deterministic two-pass reduction), on device
void vec_dot(const double* x, const double* y, int n, double* scratch, double* result, hipStream_t s);
// In-place inverse of an m x m symmetric positive definite matrix (row major)
// by blocked Gauss-Jordan with 32 x 32 tiles (batch.hip); meta: device int[4],
// off: device long long[1], col: device double[32 m + 1024] scratch; info: device int,
// nonzero when a pivot is not positive.
void gj_invert_spd(double* M, int m, int* meta, long long* off, double* col, int* info, hipStream_t s);
// C = A B (+ beta C): small dense FP64 GEMM, row-major, all device.
void dense_gemm(const double* A, const double* B, double* C, int m, int n, int k, double beta,
                bool transA, hipStream_t s, bool transB = false);

}  // namespace rc
