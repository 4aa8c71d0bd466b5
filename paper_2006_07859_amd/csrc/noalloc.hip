// Energy and differential without any allocation: the workspace of the
// FP64 pair path (edge geometry, pair partial sums, per-edge values,
// reduction scratch) lives in one file-scope device array, so the call can
// run where hipMalloc cannot (inside HIP graph capture, tight serving loops).
//
// The arithmetic is that of rc_differential on an RC_F64 context (the same
// pair, finalize and sum kernels); only the source-chunk count (at most
// kNaMaxChunks) and the final vertex gather differ.  Each device holds its
// own copy of the array until the process ends; calls that overlap on one
// device share it and race.

#include <algorithm>
#include <array>
#include <mutex>

#include "rc_internal.h"

namespace rc {

constexpr int kNaMaxEdges = 16384;
constexpr int kNaMaxVertices = 1 << 20;
constexpr int kNaMaxChunks = 16;
constexpr int kNaRedBlocks = 256;
// doubles: geometry a, b, t (3 x 4 per edge), partials (chunks x slots per
// edge), per-edge values (8 per edge), reduction partials
constexpr size_t kNaDoubles = (size_t)kNaMaxEdges * (12 + kNaMaxChunks * kTpeSlots + 8) + kNaRedBlocks;

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::array<double*, kMaxDevices> g_scratch{};  // per device: the device address of `scratch`
std::mutex g_mu;

// Device address of this device's copy of the array (looked up once per device).
rc_status scratch_address(double** out) {
  int dev = 0;
  RC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("rc_differential_noalloc: device index out of range");
    return RC_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("rc_differential_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return RC_ERR_HIP;
    }
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return RC_OK;
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace

// Edge geometry in FP64 (as the context path's k_geometry) with the endpoint
// indices checked against nV: an invalid edge gets NaN geometry, so the
// energy becomes NaN instead of a read out of bounds.
__global__ void k_na_geometry(const double* __restrict__ gamma, const int2* __restrict__ edges, int nE, int nV,
                              V4<double>* __restrict__ A, V4<double>* __restrict__ B, V4<double>* __restrict__ T) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const int2 e = edges[I];
  if (e.x < 0 || e.x >= nV || e.y < 0 || e.y >= nV || e.x == e.y) {
    const double nan = __builtin_nan("");
    A[I] = V4<double>{nan, nan, nan, nan};
    B[I] = V4<double>{nan, nan, nan, nan};
    T[I] = V4<double>{nan, nan, nan, nan};
    return;
  }
  const double p0 = gamma[3 * e.x], p1 = gamma[3 * e.x + 1], p2 = gamma[3 * e.x + 2];
  const double q0 = gamma[3 * e.y], q1 = gamma[3 * e.y + 1], q2 = gamma[3 * e.y + 2];
  const double d0 = q0 - p0, d1 = q1 - p1, d2 = q2 - p2;
  const double l = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double il = 1.0 / l;
  A[I] = V4<double>{p0, p1, p2, l};
  B[I] = V4<double>{q0, q1, q2, 0.0};
  T[I] = V4<double>{d0 * il, d1 * il, d2 * il, 0.0};
}

__global__ void k_na_zero(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// dE_v = the sum of the endpoint partials of the edges at v.  With at most two
// edges per vertex the sum 0 + a + b does not depend on the order of the two
// atomic additions, so the result equals the context path's gather exactly.
__global__ void k_na_scatter(const double* __restrict__ edge_out, const int2* __restrict__ edges, int nE, int nV,
                             double* __restrict__ dE) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const int2 e = edges[I];
  if (e.x < 0 || e.x >= nV || e.y < 0 || e.y >= nV) return;
  const double* o = edge_out + 8 * (size_t)I;
  for (int k = 0; k < 3; ++k) {
    atomicAdd(dE + 3 * e.x + k, o[1 + k]);
    atomicAdd(dE + 3 * e.y + k, o[4 + k]);
  }
}

}  // namespace rc

using namespace rc;

extern "C" rc_status rc_differential_noalloc(const double* gamma, int32_t n_vertices, const int32_t* edges,
                                             int32_t n_edges, double alpha, double beta, double* energy, double* dE,
                                             rc_stream stream) {
  set_error("");
  if (!gamma || !edges || !dE) {
    set_error("rc_differential_noalloc: null pointer argument");
    return RC_ERR_ARG;
  }
  if (n_edges < 1 || n_edges > kNaMaxEdges || n_vertices < 2 || n_vertices > kNaMaxVertices) {
    set_error("rc_differential_noalloc: need 1 <= n_edges <= 16384 and 2 <= n_vertices <= 1048576");
    return RC_ERR_ARG;
  }
  if (!(alpha > 1.0) || !(beta >= alpha + 2.0) || !(beta < 2.0 * alpha + 1.0)) {
    set_error("rc_differential_noalloc: need alpha > 1 and alpha + 2 <= beta < 2 alpha + 1");
    return RC_ERR_PARAM_RANGE;
  }
  double* base = nullptr;
  RC_TRY(scratch_address(&base));
  hipStream_t s = (hipStream_t)stream;
  const int nE = n_edges, nV = n_vertices;
  // the workspace of a context, laid out in the array (nothing here owns memory)
  Curve c;
  c.nV = nV;
  c.nE = nE;
  c.edges = (int2*)edges;
  c.chain = false;  // FP64: no near band
  const int tblocks = cdiv(nE, kTile);
  c.nchunk = std::max(1, std::min({tblocks, cdiv(2048, tblocks), kNaMaxChunks}));
  c.src_per_chunk = cdiv(nE, c.nchunk);
  c.part_chunks = c.nchunk;
  c.red_blocks = std::max(1, std::min(kNaRedBlocks, cdiv(nE, 256)));
  double* p = base;
  c.gd.a = (V4<double>*)p;
  p += 4 * (size_t)nE;
  c.gd.b = (V4<double>*)p;
  p += 4 * (size_t)nE;
  c.gd.t = (V4<double>*)p;
  p += 4 * (size_t)nE;
  c.part = p;
  p += (size_t)c.nchunk * kTpeSlots * nE;
  c.edge_out = p;
  p += 8 * (size_t)nE;
  c.red = p;
  hipLaunchKernelGGL(k_na_geometry, dim3(cdiv(nE, 256)), dim3(256), 0, s, gamma, (const int2*)edges, nE, nV, c.gd.a,
                     c.gd.b, c.gd.t);
  RC_TRY(launch_tpe(c, alpha, beta, RC_F64, true, energy, nullptr, s));
  hipLaunchKernelGGL(k_na_zero, dim3(cdiv(3 * nV, 256)), dim3(256), 0, s, dE, 3 * nV);
  hipLaunchKernelGGL(k_na_scatter, dim3(cdiv(nE, 256)), dim3(256), 0, s, (const double*)c.edge_out,
                     (const int2*)edges, nE, nV, dE);
  RC_HIP(hipGetLastError());
  return RC_OK;
}
