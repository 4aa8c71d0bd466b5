// First collision time of a curve moving along a direction (Sec. 4.4, time
// stepping from the first collision time tau_max).
//
// The curve moves as gamma(t) = gamma - t D, every vertex on a straight line.
// Two edges that share no vertex touch at t only if their four endpoints are
// coplanar, i.e. at a root of the cubic f(t) = det[p2 - p1, q1 - p1, q2 - p1](t);
// at each root in (0, T], in increasing order, the segments touch iff their
// distance vanishes (relative tolerance kContactRtol).  When f vanishes
// identically (both segments move inside one fixed plane) the first contact is
// an endpoint reaching the other segment: a root of the quadratic
// n . ((a - p) x (b - p))(t).  The result is the minimum over all pairs.
//
// One thread per target edge I sweeps the source edges J > I of its chunk,
// staged in LDS; pairs whose boxes swept over [0, T] do not overlap cannot
// touch and are skipped after six comparisons (the common case).  The others
// are solved in FP64: the cubic's critical points split (0, T] into monotone
// pieces, each sign change is bisected to full precision, and the contact
// test follows.  The minimum goes to a 64-bit atomic min on the bits of the
// non-negative double, so the result does not depend on the order.

#include <algorithm>
#include <cfloat>

#include "rc_internal.h"

namespace rc {

constexpr double kContactRtol = 1e-9;
constexpr double kPlanarRtol = 1e-12;

static inline int ccd_cdiv(int a, int b) { return (a + b - 1) / b; }

// Per edge: endpoints and velocities in FP64, and the FP32 box (rounded
// outwards) holding the segment at every t in [0, T] (the hull of its
// endpoints at 0 and at T).
__global__ void k_ccd_prep(const double* __restrict__ gamma, const double* __restrict__ D,
                           const int2* __restrict__ edges, int nE, double T, V4<double>* __restrict__ P1,
                           V4<double>* __restrict__ P2, V4<double>* __restrict__ W1, V4<double>* __restrict__ W2,
                           float4* __restrict__ bmin, float4* __restrict__ bmax) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nE) return;
  const int2 e = edges[I];
  double p[2][3], v[2][3];
  for (int k = 0; k < 3; ++k) {
    p[0][k] = gamma[3 * e.x + k];
    p[1][k] = gamma[3 * e.y + k];
    v[0][k] = D[3 * e.x + k];
    v[1][k] = D[3 * e.y + k];
  }
  P1[I] = V4<double>{p[0][0], p[0][1], p[0][2], 0.0};
  P2[I] = V4<double>{p[1][0], p[1][1], p[1][2], 0.0};
  W1[I] = V4<double>{v[0][0], v[0][1], v[0][2], 0.0};
  W2[I] = V4<double>{v[1][0], v[1][1], v[1][2], 0.0};
  float lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    double a = fmin(fmin(p[0][k], p[1][k]), fmin(p[0][k] - T * v[0][k], p[1][k] - T * v[1][k]));
    double b = fmax(fmax(p[0][k], p[1][k]), fmax(p[0][k] - T * v[0][k], p[1][k] - T * v[1][k]));
    const double pad = 1e-6 * (fabs(a) + fabs(b)) + 1e-30;
    lo[k] = (float)(a - pad);
    hi[k] = (float)(b + pad);
  }
  bmin[I] = make_float4(lo[0], lo[1], lo[2], 0.f);
  bmax[I] = make_float4(hi[0], hi[1], hi[2], 0.f);
}

struct Vec3 {
  double x, y, z;
};
__device__ __forceinline__ Vec3 sub3(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ Vec3 axpy3(double t, Vec3 v, Vec3 a) { return {a.x - t * v.x, a.y - t * v.y, a.z - t * v.z}; }
__device__ __forceinline__ double dot3(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ Vec3 cross3(Vec3 a, Vec3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm3(Vec3 a) { return sqrt(dot3(a, a)); }

// Distance between the segments p1p2 and q1q2 (closest points, clamped).
__device__ double seg_distance(Vec3 p1, Vec3 p2, Vec3 q1, Vec3 q2) {
  const Vec3 d1 = sub3(p2, p1), d2 = sub3(q2, q1), r = sub3(p1, q1);
  const double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r), c = dot3(d1, r), b = dot3(d1, d2);
  const double den = a * e - b * b;
  double s = den > 1e-300 ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
  double u = (b * s + f) / e;
  if (u < 0.0) {
    u = 0.0;
    s = fmin(fmax(-c / a, 0.0), 1.0);
  } else if (u > 1.0) {
    u = 1.0;
    s = fmin(fmax((b - c) / a, 0.0), 1.0);
  }
  const Vec3 x = {p1.x + s * d1.x - (q1.x + u * d2.x), p1.y + s * d1.y - (q1.y + u * d2.y),
                  p1.z + s * d1.z - (q1.z + u * d2.z)};
  return norm3(x);
}

// Coefficients (c0 + c1 t + c2 t^2 + c3 t^3) of det[a0 - t a1, b0 - t b1, c0 - t c1].
__device__ void det_cubic(Vec3 a0, Vec3 a1, Vec3 b0, Vec3 b1, Vec3 c0, Vec3 c1, double (&f)[4]) {
  const Vec3 bc00 = cross3(b0, c0), bc01 = cross3(b0, c1), bc10 = cross3(b1, c0), bc11 = cross3(b1, c1);
  f[0] = dot3(a0, bc00);
  f[1] = -(dot3(a1, bc00) + dot3(a0, bc01) + dot3(a0, bc10));
  f[2] = dot3(a0, bc11) + dot3(a1, bc01) + dot3(a1, bc10);
  f[3] = -dot3(a1, bc11);
}

__device__ __forceinline__ double poly3(const double (&f)[4], double t) { return ((f[3] * t + f[2]) * t + f[1]) * t + f[0]; }

// Real roots of c0 + c1 t + c2 t^2 in (lo, hi), ascending; returns the count.
__device__ int quad_roots(double c0, double c1, double c2, double lo, double hi, double (&r)[2]) {
  int n = 0;
  if (c2 == 0.0) {
    if (c1 != 0.0) {
      const double t = -c0 / c1;
      if (t > lo && t < hi) r[n++] = t;
    }
    return n;
  }
  const double disc = c1 * c1 - 4.0 * c2 * c0;
  if (disc < 0.0) return 0;
  const double q = -0.5 * (c1 + copysign(sqrt(disc), c1));
  double t0 = q / c2, t1 = q != 0.0 ? c0 / q : t0;
  if (t0 > t1) {
    const double x = t0;
    t0 = t1;
    t1 = x;
  }
  if (t0 > lo && t0 < hi) r[n++] = t0;
  if (t1 > lo && t1 < hi && t1 != t0) r[n++] = t1;
  return n;
}

// Root of f in [lo, hi] by bisection, f(lo) f(hi) <= 0.
template <typename F>
__device__ double bisect(F f, double lo, double hi) {
  double flo = f(lo);
  if (flo == 0.0) return lo;
  for (int it = 0; it < 120 && hi - lo > 0.0; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    const double fm = f(mid);
    if ((fm < 0.0) == (flo < 0.0) && fm != 0.0) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return hi;
}

// First contact time in (0, T] of segment pq (endpoints p1, p2, velocities
// v1, v2) and rs (q1, q2, w1, w2), or +inf.
__device__ double pair_contact(Vec3 p1, Vec3 p2, Vec3 q1, Vec3 q2, Vec3 v1, Vec3 v2, Vec3 w1, Vec3 w2, double T) {
  const double speed = fmax(fmax(norm3(v1), norm3(v2)), fmax(norm3(w1), norm3(w2)));
  const double scale = fmax(fmax(norm3(sub3(p2, p1)), norm3(sub3(q2, q1))), norm3(sub3(q1, p1))) + T * speed;
  const double tol = kContactRtol * scale;
  auto touching = [&](double t) {
    return seg_distance(axpy3(t, v1, p1), axpy3(t, v2, p2), axpy3(t, w1, q1), axpy3(t, w2, q2)) <= tol;
  };
  double f[4];
  det_cubic(sub3(p2, p1), sub3(v2, v1), sub3(q1, p1), sub3(w1, v1), sub3(q2, p1), sub3(w2, v1), f);
  const double s3 = scale * scale * scale;
  bool planar = true;
  double tk = 1.0;
  for (int k = 0; k < 4; ++k) {
    planar &= fabs(f[k]) * tk <= kPlanarRtol * s3;
    tk *= T;
  }
  if (planar) {
    // an endpoint reaching the other segment, inside the common plane
    Vec3 n = cross3(sub3(p2, p1), sub3(q1, p1));
    if (norm3(n) == 0.0) n = cross3(sub3(p2, p1), sub3(q2, p1));
    const double in = 1.0 / norm3(n);
    n = {n.x * in, n.y * in, n.z * in};
    double best = INFINITY;
    const Vec3 X[4] = {p1, p2, q1, q2}, VX[4] = {v1, v2, w1, w2};
    for (int m = 0; m < 4; ++m) {
      const Vec3 x = X[m], vx = VX[m];
      const Vec3 y1 = m < 2 ? q1 : p1, vy1 = m < 2 ? w1 : v1, y2 = m < 2 ? q2 : p2, vy2 = m < 2 ? w2 : v2;
      // g(t) = n . ((y1 - x)(t) x (y2 - x)(t)), with (y - x)(t) = (y - x) - t (vy - vx)
      const Vec3 a0 = sub3(y1, x), a1 = sub3(vy1, vx), b0 = sub3(y2, x), b1 = sub3(vy2, vx);
      const double c0 = dot3(n, cross3(a0, b0));
      const double c1 = -(dot3(n, cross3(a0, b1)) + dot3(n, cross3(a1, b0)));
      const double c2 = dot3(n, cross3(a1, b1));
      double r[2];
      const int nr = quad_roots(c0, c1, c2, 0.0, T * (1.0 + 1e-15) + DBL_MIN, r);
      for (int j = 0; j < nr; ++j)
        if (r[j] <= T && touching(r[j])) {
          best = fmin(best, r[j]);
          break;
        }
    }
    return best;
  }
  // monotone pieces of the cubic on (0, T]
  double cut[4];
  int nc = 0;
  cut[nc++] = 0.0;
  double cr[2];
  const int ncr = quad_roots(f[1], 2.0 * f[2], 3.0 * f[3], 0.0, T, cr);
  for (int j = 0; j < ncr; ++j) cut[nc++] = cr[j];
  cut[nc++] = T;
  auto fval = [&](double t) { return poly3(f, t); };
  for (int j = 0; j + 1 < nc; ++j) {
    const double lo = cut[j], hi = cut[j + 1];
    const double flo = fval(lo), fhi = fval(hi);
    if (!(flo * fhi <= 0.0)) continue;
    const double t = bisect(fval, lo, hi);
    if (t > 0.0 && t <= T && touching(t)) return t;
  }
  return INFINITY;
}

__global__ void k_ccd_init(unsigned long long* out) { out[0] = __double_as_longlong(INFINITY); }

__global__ void k_ccd_out(const unsigned long long* bits, double* t) { t[0] = __longlong_as_double(bits[0]); }

__global__ __launch_bounds__(kTile) void k_ccd_pairs(const V4<double>* __restrict__ P1,
                                                     const V4<double>* __restrict__ P2,
                                                     const V4<double>* __restrict__ W1,
                                                     const V4<double>* __restrict__ W2,
                                                     const float4* __restrict__ bmin, const float4* __restrict__ bmax,
                                                     const int2* __restrict__ edges, int nE, int src_per_chunk,
                                                     double T, unsigned long long* __restrict__ out) {
  __shared__ float4 sLo[kTile], sHi[kTile];
  __shared__ int2 sE[kTile];
  __shared__ double sMin[kTile / 64];
  const int tid = threadIdx.x;
  const int I0 = blockIdx.x * kTile, I = I0 + tid;
  const int s0 = max(blockIdx.y * src_per_chunk, I0 + 1), s1 = min(nE, (int)(blockIdx.y + 1) * src_per_chunk);
  double best = INFINITY;
  if (s0 < s1) {  // uniform over the workgroup: sources J > I only
    const bool act = I < nE;
    const int Ic = act ? I : I0;
    const float4 lo = bmin[Ic], hi = bmax[Ic];
    const int2 ei = edges[Ic];
    for (int t0 = s0; t0 < s1; t0 += kTile) {
      __syncthreads();
      if (t0 + tid < s1) {
        sLo[tid] = bmin[t0 + tid];
        sHi[tid] = bmax[t0 + tid];
        sE[tid] = edges[t0 + tid];
      }
      __syncthreads();
      const int cnt = min(kTile, s1 - t0);
      for (int u = 0; u < cnt; ++u) {
        const int J = t0 + u;
        const float4 l2 = sLo[u], h2 = sHi[u];
        const bool overlap = (lo.x <= h2.x) & (l2.x <= hi.x) & (lo.y <= h2.y) & (l2.y <= hi.y) & (lo.z <= h2.z) &
                             (l2.z <= hi.z);
        if (!(act && J > I && overlap)) continue;
        const int2 ej = sE[u];
        if ((ei.x == ej.x) | (ei.x == ej.y) | (ei.y == ej.x) | (ei.y == ej.y)) continue;
        const V4<double> a1 = P1[I], a2 = P2[I], va = W1[I], vb = W2[I];
        const V4<double> b1 = P1[J], b2 = P2[J], wa = W1[J], wb = W2[J];
        const double t = pair_contact({a1.x, a1.y, a1.z}, {a2.x, a2.y, a2.z}, {b1.x, b1.y, b1.z},
                                      {b2.x, b2.y, b2.z}, {va.x, va.y, va.z}, {vb.x, vb.y, vb.z},
                                      {wa.x, wa.y, wa.z}, {wb.x, wb.y, wb.z}, T);
        best = fmin(best, t);
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) best = fmin(best, __shfl_xor(best, o));
  if ((tid & 63) == 0) sMin[tid >> 6] = best;
  __syncthreads();
  if (tid == 0) {
    double m = sMin[0];
    for (int w = 1; w < kTile / 64; ++w) m = fmin(m, sMin[w]);
    if (m < INFINITY) atomicMin(out, (unsigned long long)__double_as_longlong(m));
  }
}

rc_status CcdBuffers::ensure(int nE_) {
  if (nE == nE_ && p1) return RC_OK;
  release();
  auto al = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 16)) == hipSuccess; };
  const size_t v = sizeof(V4<double>) * (size_t)nE_, f = sizeof(float4) * (size_t)nE_;
  if (!al((void**)&p1, v) || !al((void**)&p2, v) || !al((void**)&w1, v) || !al((void**)&w2, v) ||
      !al((void**)&lo, f) || !al((void**)&hi, f) || !al((void**)&bits, 8) || !al((void**)&t, 8)) {
    release();
    set_error("allocation of the collision-time buffers failed");
    return RC_ERR_NOMEM;
  }
  nE = nE_;
  return RC_OK;
}

void CcdBuffers::release() {
  void* ps[] = {p1, p2, w1, w2, lo, hi, bits, t};
  for (void* p : ps)
    if (p) hipFree(p);
  p1 = p2 = w1 = w2 = nullptr;
  lo = hi = nullptr;
  bits = nullptr;
  t = nullptr;
  nE = 0;
}

rc_status launch_first_collision(const Curve& c, const double* gamma, const double* D, double T, CcdBuffers& buf,
                                 double* t_out, hipStream_t s) {
  const int nE = c.nE;
  hipLaunchKernelGGL(k_ccd_prep, dim3(ccd_cdiv(nE, 256)), dim3(256), 0, s, gamma, D, (const int2*)c.edges, nE, T,
                     buf.p1, buf.p2, buf.w1, buf.w2, buf.lo, buf.hi);
  hipLaunchKernelGGL(k_ccd_init, dim3(1), dim3(1), 0, s, buf.bits);
  const int tb = ccd_cdiv(nE, kTile);
  const int nchunk = std::max(1, std::min(tb, ccd_cdiv(2048, tb)));
  const int spc = ccd_cdiv(nE, nchunk);
  hipLaunchKernelGGL(k_ccd_pairs, dim3(tb, nchunk), dim3(kTile), 0, s, (const V4<double>*)buf.p1,
                     (const V4<double>*)buf.p2, (const V4<double>*)buf.w1, (const V4<double>*)buf.w2,
                     (const float4*)buf.lo, (const float4*)buf.hi, (const int2*)c.edges, nE, spc, T, buf.bits);
  hipLaunchKernelGGL(k_ccd_out, dim3(1), dim3(1), 0, s, (const unsigned long long*)buf.bits, t_out);
  RC_HIP(hipGetLastError());
  return RC_OK;
}

}  // namespace rc
