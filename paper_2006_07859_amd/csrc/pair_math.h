// Device math shared by the pair kernels and the Barnes-Hut traversal:
// transcendental helpers, exponent specialisations and the per-vertex-pair
// accumulation of the tangent-point energy and its derivatives.
#pragma once

#include <climits>
#include <type_traits>

#include "rc_internal.h"

namespace rc {

// Range (min chain, max chain, min position, max position) of the chain
// coordinates held by the valid threads of a workgroup of kTile threads: each
// wave reduces with cross-lane exchanges and writes its slot of red; after a
// barrier, range_of(red) combines the slots.
__device__ __forceinline__ void wave_range(int4 c, bool valid, int4* red) {
  int cmin = valid ? c.x : INT_MAX, cmax = valid ? c.x : INT_MIN;
  int pmin = valid ? c.y : INT_MAX, pmax = valid ? c.y : INT_MIN;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cmin = min(cmin, __shfl_xor(cmin, o));
    cmax = max(cmax, __shfl_xor(cmax, o));
    pmin = min(pmin, __shfl_xor(pmin, o));
    pmax = max(pmax, __shfl_xor(pmax, o));
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_int4(cmin, cmax, pmin, pmax);
}

__device__ __forceinline__ int4 range_of(const int4* red) {
  int4 r = red[0];
#pragma unroll
  for (int w = 1; w < kTile / 64; ++w) {
    const int4 v = red[w];
    r = make_int4(min(r.x, v.x), max(r.y, v.y), min(r.z, v.z), max(r.w, v.w));
  }
  return r;
}

// True when no target of range tr is chain-near any source of range sr: the
// chain ranges are disjoint, or both tiles lie on one chain (length m, a loop
// when loop != 0) with position intervals more than kBand apart, also around
// the loop.  Conservative: false whenever the ranges cannot decide.
__device__ __forceinline__ bool tiles_far(int4 tr, int4 sr, int m, int loop) {
  if (tr.y < sr.x || sr.y < tr.x) return true;
  if (tr.x != tr.y || sr.x != sr.y) return false;
  const int gap = max(sr.z - tr.w, tr.z - sr.w);
  if (gap <= kBand) return false;
  return !loop || m - (max(tr.w, sr.w) - min(tr.z, sr.z)) > kBand;
}

// ---------------------------------------------------------------------------
// math helpers: hardware transcendentals in FP32; in FP64 the hardware
// reciprocal square root refined by Newton-Raphson, library exp2/log2
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R f_rsq(R x);
template <> __device__ __forceinline__ float f_rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// 1/sqrt(x) for finite x > 0 (squared distances here): the hardware estimate
// and two Newton-Raphson steps for f(y) = 1/y^2 - x, y <- y + y (1 - x y^2) / 2,
// each roughly squaring the relative error.  No range handling: x = 0 or
// x = inf give NaN (the pair sums would be infinite there anyway).
template <> __device__ __forceinline__ double f_rsq<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}
template <typename R> __device__ __forceinline__ R f_sqrt(R x);
template <> __device__ __forceinline__ float f_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
// sqrt(x) = x / sqrt(x) for x > 0, and 0 for x = 0.
template <> __device__ __forceinline__ double f_sqrt<double>(double x) { return x > 0.0 ? x * f_rsq<double>(x) : 0.0; }
template <typename R> __device__ __forceinline__ R f_exp2(R x);
template <> __device__ __forceinline__ float f_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <> __device__ __forceinline__ double f_exp2<double>(double x) { return exp2(x); }
template <typename R> __device__ __forceinline__ R f_log2(R x);
template <> __device__ __forceinline__ float f_log2<float>(float x) { return __builtin_amdgcn_logf(x); }
template <> __device__ __forceinline__ double f_log2<double>(double x) { return log2(x); }

// r2^(-beta/2) from rs = 1/sqrt(r2) and ri = 1/r2.
template <int EC, typename R>
__device__ __forceinline__ R pow_beta(R r2, R rs, R ri, R half_beta) {
  if constexpr (EC == kA2B4) return ri * ri;
  else if constexpr (EC == kA2B45) return ri * ri * f_sqrt<R>(rs);
  else if constexpr (EC == kA3B6) return ri * ri * ri;
  else return f_exp2<R>(-half_beta * f_log2<R>(r2));
}

// ca = c^(alpha/2) and f = (alpha/2) c^(alpha/2 - 1) for c = |T x d|^2 >= 0.
template <int EC, typename R>
__device__ __forceinline__ void pow_alpha(R c, R half_alpha, R& ca, R& f) {
  if constexpr (EC == kA2B4 || EC == kA2B45) {
    ca = c;
    f = R(1);
  } else if constexpr (EC == kA3B6) {
    R sq = f_sqrt<R>(c);
    ca = c * sq;
    f = R(1.5) * sq;
  } else {
    if (c > R(0)) {
      ca = f_exp2<R>(half_alpha * f_log2<R>(c));
      f = half_alpha * ca / c;
    } else {
      ca = R(0);
      f = R(0);
    }
  }
}

// r2^(-(2 sigma + 1)/2): the weight exponent of B and B0 (Sec. 4.2.2-4.2.3).
template <int EC, typename R>
__device__ __forceinline__ R pow_sigma(R r2, R rs, R ri, R half_expo) {
  if constexpr (EC == kA2B4) return ri;                       // 2 sigma + 1 = 2
  else if constexpr (EC == kA2B45) return ri * f_sqrt<R>(rs);  // 2.5
  else return f_exp2<R>(-half_expo * f_log2<R>(r2));          // 7/3 for (3,6), general
}

// ri = r2^-1 and p = r2^(-(2 sigma + 1)/2) for one vertex pair.  In FP64 with
// 2 sigma + 1 = 2.5 both are powers of q = r2^(-1/4) (ri = q^4, p = q^5): q
// comes from an FP32 estimate refined by two Newton steps for q^-4 = r2,
// q <- q + q (1 - r2 q^4) / 4, each roughly squaring the relative error of
// the estimate (about 2^-22): no FP64 transcendental and no branch.
template <int EC, typename R>
__device__ __forceinline__ void sob_powers(R r2, R half_expo, R& ri, R& p) {
  if constexpr (EC == kA2B45 && std::is_same<R, double>::value) {
    double q = (double)__builtin_amdgcn_sqrtf(__builtin_amdgcn_rsqf((float)r2));
    const double mr = -0.25 * r2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double q2 = q * q;
      q = fma(q, fma(mr, q2 * q2, 0.25), q);
    }
    const double q2 = q * q;
    ri = q2 * q2;
    p = ri * q;
  } else {
    const R rs = f_rsq<R>(r2);
    ri = rs * rs;
    p = pow_sigma<EC, R>(r2, rs, ri, half_expo);
  }
}

// ri = r2^-1 and rb = r2^(-beta/2) for one vertex pair of the energy.  In
// FP64 with beta = 4.5 both are powers of q = r2^(-1/4) (ri = q^4, rb = q^9),
// with q from an FP32 estimate and two Newton steps as in sob_powers.
template <int EC, typename R>
__device__ __forceinline__ void tpe_powers(R r2, R half_beta, R& ri, R& rb) {
  if constexpr (EC == kA2B45 && std::is_same<R, double>::value) {
    double q = (double)__builtin_amdgcn_sqrtf(__builtin_amdgcn_rsqf((float)r2));
    const double mr = -0.25 * r2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double q2 = q * q;
      q = fma(q, fma(mr, q2 * q2, 0.25), q);
    }
    const double q2 = q * q;
    ri = q2 * q2;
    rb = ri * ri * q;
  } else {
    const R rs = f_rsq<R>(r2);
    ri = rs * rs;
    rb = pow_beta<EC, R>(r2, rs, ri, half_beta);
  }
}

template <typename R>
__device__ __forceinline__ R cross_norm2(R tx, R ty, R tz, R dx, R dy, R dz) {
  // |T x d|^2 from the cross product itself: accurate when d is nearly
  // parallel to T, where |d|^2 - (T.d)^2 would cancel catastrophically.
  R cx = ty * dz - tz * dy;
  R cy = tz * dx - tx * dz;
  R cz = tx * dy - ty * dx;
  return cx * cx + cy * cy + cz * cz;
}

// ---------------------------------------------------------------------------
// energy and differential, trapezoid rule over the four vertex pairs
// ---------------------------------------------------------------------------
// Accumulator slots (per target edge I; every term carries w = l_J / 4):
//  0 E    sum k(d, T_I)                                  -> energy l_I * E
//  1 S    sum k(d, T_I) + k(d, T_J)                      -> dl_I term
//  2-4 G1 sum over (i1, j_b) of grad_d[k_I + k_J] minus its T_I part
//  5-7 G2 same for i2
//  8 Gt1, 9 Gt2: coefficient of T_I in those gradients
//  10-12 Hd, 13 Ht: dk/dT_I projected on the tangent plane = -2 (Hd - Ht T_I)
// tjj = |T_J|^2: 1 for an edge; a Barnes-Hut cluster's length-weighted mean
// tangent is shorter, and d|T x d|^2/dd = 2 (|T|^2 d - (T.d) T).
template <typename R, int EC, bool GRAD>
__device__ __forceinline__ void tpe_vertex_pair(
    R px, R py, R pz, R tIx, R tIy, R tIz,                // target vertex, T_I
    R qx, R qy, R qz, R tJx, R tJy, R tJz,                // source vertex, T_J
    bool same, R w, R half_alpha, R half_beta, R beta,
    R& E, R& S, R& Gx, R& Gy, R& Gz, R& Gt, R& Hx, R& Hy, R& Hz, R& Ht, R tjj = R(1)) {
  R dx = px - qx, dy = py - qy, dz = pz - qz;
  R r2 = dx * dx + dy * dy + dz * dz;
  r2 = same ? R(1) : r2;
  R rs = f_rsq<R>(r2);
  R ri = rs * rs;
  R rbw = pow_beta<EC, R>(r2, rs, ri, half_beta) * w;
  R cI = cross_norm2<R>(tIx, tIy, tIz, dx, dy, dz);
  R caI, fI;
  pow_alpha<EC, R>(cI, half_alpha, caI, fI);
  R kI = caI * rbw;
  E += kI;
  if constexpr (GRAD) {
    R cJ = cross_norm2<R>(tJx, tJy, tJz, dx, dy, dz);
    R caJ, fJ;
    pow_alpha<EC, R>(cJ, half_alpha, caJ, fJ);
    R kJ = caJ * rbw;
    R ks = kI + kJ;
    S += ks;
    R tI = tIx * dx + tIy * dy + tIz * dz;
    R tJ = tJx * dx + tJy * dy + tJz * dz;
    R gI = R(2) * fI * rbw;
    R gJ = R(2) * fJ * rbw;
    // grad_d k = 2 f rb (d - t T) - beta k d / r2
    R c1 = gI + gJ * tjj - beta * ks * ri;
    R c2 = gJ * tJ;
    Gx += c1 * dx - c2 * tJx;
    Gy += c1 * dy - c2 * tJy;
    Gz += c1 * dz - c2 * tJz;
    Gt += gI * tI;
    // dk/dT_I on the tangent plane: -2 f rb t (d - t T_I)
    R c3 = fI * rbw * tI;
    Hx += c3 * dx;
    Hy += c3 * dy;
    Hz += c3 * dz;
    Ht += c3 * tI;
  }
}

// The same four vertex-pair terms for one ordered edge pair (I, J) of the
// all-pairs kernels, with the work the pairs share done once.  Target I has
// endpoints a (i1) and b (i2) and unit tangent T, source J endpoints c (j1)
// and e (j2) and unit tangent U; l_I and l_J are their lengths, so that
// b = a + l_I T and e = c + l_J U.  Hence, with d(p, q) = p - q and d = d(a, c):
//  * |T x d(p, q)| does not depend on p, and |U x d(p, q)| not on q, with
//    T x d(a, e) = T x d - l_J (T x U) and U x d(b, c) = U x d - l_I (T x U);
//  * T.d(a, e) = T.d - l_J (T.U), T.d(b, q) = T.d(a, q) + l_I, and likewise
//    U.d(b, c) = U.d + l_I (T.U), U.d(p, e) = U.d(p, c) - l_J;
//  * |d|^2 = |T x d|^2 + (T.d)^2 (|T| = 1), a sum of two non-negative terms;
//  * the gradient sums use d(p, e) = d(p, c) - l_J U and d(b, c) = d + l_I T,
//    whose T part joins the T coefficient Gt2; the sum H, which the caller
//    projects onto the plane normal to T, is accumulated modulo multiples of
//    T (d(b, q) = d(a, q) + l_I T).
// Every identity holds exactly for the real geometry; in rounded arithmetic
// the terms differ from the direct ones by the rounding of the coordinates.
// w = l_J / 4, and 0 for a skipped pair, whose skipv = 1 keeps |d|^2 >= 1
// (skipv = 0 otherwise; ignored when SKIP is false).  Ht is not accumulated:
// T.H replaces it after the sum.  With MASK4, only the vertex pairs whose bit
// is set in m4 are summed (bit 0: (a, c), 1: (a, e), 2: (b, c), 3: (b, e));
// every term of a vertex pair carries its factor r^-beta, so zeroing that
// factor removes the vertex pair exactly.
template <typename R, int EC, bool GRAD, bool SKIP, bool MASK4 = false>
__device__ __forceinline__ void tpe_edge_pair(
    R ax, R ay, R az, R Tx, R Ty, R Tz, R lI, R cx, R cy, R cz, R Ux, R Uy, R Uz, R lJ,
    R w, R skipv, R half_alpha, R half_beta, R beta,
    R& E, R& S, R& G1x, R& G1y, R& G1z, R& Gt1, R& G2x, R& G2y, R& G2z, R& Gt2, R& Hx, R& Hy, R& Hz,
    int m4 = 15) {
  const R dx = ax - cx, dy = ay - cy, dz = az - cz;  // d(a, c)
  const R wx = Ty * Uz - Tz * Uy, wy = Tz * Ux - Tx * Uz, wz = Tx * Uy - Ty * Ux;  // T x U
  const R tu = Tx * Ux + Ty * Uy + Tz * Uz;
  const R xIx = Ty * dz - Tz * dy, xIy = Tz * dx - Tx * dz, xIz = Tx * dy - Ty * dx;  // T x d(a, c)
  const R yIx = xIx - lJ * wx, yIy = xIy - lJ * wy, yIz = xIz - lJ * wz;                // T x d(a, e)
  R cI1 = xIx * xIx + xIy * xIy + xIz * xIz;
  R cI2 = yIx * yIx + yIy * yIy + yIz * yIz;
  if constexpr (SKIP) {
    cI1 += skipv;
    cI2 += skipv;
  }
  const R t11 = Tx * dx + Ty * dy + Tz * dz;
  const R t12 = t11 - lJ * tu;
  const R t21 = t11 + lI, t22 = t12 + lI;
  const R r11 = t11 * t11 + cI1, r12 = t12 * t12 + cI2;
  const R r21 = t21 * t21 + cI1, r22 = t22 * t22 + cI2;
  R ri11, ri12, ri21, ri22, rb11, rb12, rb21, rb22;
  tpe_powers<EC, R>(r11, half_beta, ri11, rb11);
  tpe_powers<EC, R>(r12, half_beta, ri12, rb12);
  tpe_powers<EC, R>(r21, half_beta, ri21, rb21);
  tpe_powers<EC, R>(r22, half_beta, ri22, rb22);
  rb11 *= w;
  rb12 *= w;
  rb21 *= w;
  rb22 *= w;
  if constexpr (MASK4) {
    rb11 = (m4 & 1) ? rb11 : R(0);
    rb12 = (m4 & 2) ? rb12 : R(0);
    rb21 = (m4 & 4) ? rb21 : R(0);
    rb22 = (m4 & 8) ? rb22 : R(0);
  }
  R caI1, fI1, caI2, fI2;
  pow_alpha<EC, R>(cI1, half_alpha, caI1, fI1);
  pow_alpha<EC, R>(cI2, half_alpha, caI2, fI2);
  E = fma(caI1, rb11 + rb21, E);
  E = fma(caI2, rb12 + rb22, E);
  if constexpr (GRAD) {
    const R xJx = Uy * dz - Uz * dy, xJy = Uz * dx - Ux * dz, xJz = Ux * dy - Uy * dx;  // U x d(a, c)
    const R yJx = xJx - lI * wx, yJy = xJy - lI * wy, yJz = xJz - lI * wz;                // U x d(b, c)
    const R cJ1 = xJx * xJx + xJy * xJy + xJz * xJz;
    const R cJ2 = yJx * yJx + yJy * yJy + yJz * yJz;
    R caJ1, fJ1, caJ2, fJ2;
    pow_alpha<EC, R>(cJ1, half_alpha, caJ1, fJ1);
    pow_alpha<EC, R>(cJ2, half_alpha, caJ2, fJ2);
    const R u11 = Ux * dx + Uy * dy + Uz * dz;
    const R u21 = u11 + lI * tu;
    const R u12 = u11 - lJ, u22 = u21 - lJ;
    // k(d, T) + k(d, U) per vertex pair, and its sum
    const R s11 = caI1 + caJ1, s12 = caI2 + caJ1, s21 = caI1 + caJ2, s22 = caI2 + caJ2;
    S = fma(s11, rb11, S);
    S = fma(s12, rb12, S);
    S = fma(s21, rb21, S);
    S = fma(s22, rb22, S);
    // coefficient of d in grad_d [k(d, T) + k(d, U)]: rb (2 fI + 2 fJ - beta s / |d|^2)
    const R c11 = rb11 * (R(2) * (fI1 + fJ1) - beta * s11 * ri11);
    const R c12 = rb12 * (R(2) * (fI2 + fJ1) - beta * s12 * ri12);
    const R c21 = rb21 * (R(2) * (fI1 + fJ2) - beta * s21 * ri21);
    const R c22 = rb22 * (R(2) * (fI2 + fJ2) - beta * s22 * ri22);
    // G at p: sum over q of c d(p, q) - 2 fJ rb (U.d) U, with d(p, e) = d(p, c) - l_J U;
    // at b, d(b, c) = d + l_I T, whose T part g2 l_I goes to the T coefficient
    const R g1 = c11 + c12, h1 = R(2) * fJ1 * (rb11 * u11 + rb12 * u12) + lJ * c12;
    const R g2 = c21 + c22, h2 = R(2) * fJ2 * (rb21 * u21 + rb22 * u22) + lJ * c22;
    G1x = fma(g1, dx, fma(-h1, Ux, G1x));
    G1y = fma(g1, dy, fma(-h1, Uy, G1y));
    G1z = fma(g1, dz, fma(-h1, Uz, G1z));
    G2x = fma(g2, dx, fma(-h2, Ux, G2x));
    G2y = fma(g2, dy, fma(-h2, Uy, G2y));
    G2z = fma(g2, dz, fma(-h2, Uz, G2z));
    // fI rb (T.d): half the T coefficient of the gradient, and the weight of d in H
    const R k11 = fI1 * rb11 * t11, k12 = fI2 * rb12 * t12, k21 = fI1 * rb21 * t21, k22 = fI2 * rb22 * t22;
    Gt1 = fma(R(2), k11 + k12, Gt1);
    Gt2 = fma(R(2), k21 + k22, fma(-g2, lI, Gt2));
    // H: (k11 + k21) d + (k12 + k22) (d - l_J U)
    const R m = (k11 + k21) + (k12 + k22), mu = lJ * (k12 + k22);
    Hx = fma(m, dx, fma(-mu, Ux, Hx));
    Hy = fma(m, dy, fma(-mu, Uy, Hy));
    Hz = fma(m, dz, fma(-mu, Uz, Hz));
  }
}

// Weights of the operator A = B + B0 (Sec. 4.2.2-4.2.3) for one ordered edge
// pair (I, J): rho = the sum over the four vertex pairs of |d|^-(2 sigma + 1),
// rho0 = the same terms weighted by (|T x d|^2 + |U x d|^2) / |d|^4.  The
// geometry and the shared work are those of tpe_edge_pair (two cross products
// of each kind, T.d shifted by l_I, |d|^2 = |T x d|^2 + (T.d)^2); this core
// takes the differences d(a, c), d(a, e) and d(b, c).  skipv = 1 for a
// skipped pair keeps |d|^2 >= 1 (its weight is zeroed by the caller).
template <typename R, int EC, bool SKIP>
__device__ __forceinline__ void sob_edge_pair_d(R d11x, R d11y, R d11z, R d12x, R d12y, R d12z, R d21x, R d21y,
                                                R d21z, R Tx, R Ty, R Tz, R lI, R Ux, R Uy, R Uz, R skipv,
                                                R half_expo, R& rho, R& rho0) {
  R cI1 = cross_norm2<R>(Tx, Ty, Tz, d11x, d11y, d11z);
  R cI2 = cross_norm2<R>(Tx, Ty, Tz, d12x, d12y, d12z);
  if constexpr (SKIP) {
    cI1 += skipv;
    cI2 += skipv;
  }
  const R cJ1 = cross_norm2<R>(Ux, Uy, Uz, d11x, d11y, d11z);
  const R cJ2 = cross_norm2<R>(Ux, Uy, Uz, d21x, d21y, d21z);
  const R t11 = Tx * d11x + Ty * d11y + Tz * d11z;
  const R t12 = Tx * d12x + Ty * d12y + Tz * d12z;
  const R t21 = t11 + lI, t22 = t12 + lI;
  const R r11 = t11 * t11 + cI1, r12 = t12 * t12 + cI2;
  const R r21 = t21 * t21 + cI1, r22 = t22 * t22 + cI2;
  R ri11, ri12, ri21, ri22, p11, p12, p21, p22;
  sob_powers<EC, R>(r11, half_expo, ri11, p11);
  sob_powers<EC, R>(r12, half_expo, ri12, p12);
  sob_powers<EC, R>(r21, half_expo, ri21, p21);
  sob_powers<EC, R>(r22, half_expo, ri22, p22);
  rho = (p11 + p12) + (p21 + p22);
  const R q11 = p11 * ri11 * ri11, q12 = p12 * ri12 * ri12, q21 = p21 * ri21 * ri21, q22 = p22 * ri22 * ri22;
  R z = cI1 * (q11 + q21);
  z = fma(cI2, q12 + q22, z);
  z = fma(cJ1, q11 + q12, z);
  rho0 = fma(cJ2, q21 + q22, z);
}

// The same from one endpoint of each edge: target a (tangent T, length l_I),
// source c (tangent U, length l_J); the cross products and the tangential
// component at the other endpoints are shifts by multiples of T x U and T.U
// as in tpe_edge_pair.
template <typename R, int EC, bool SKIP>
__device__ __forceinline__ void sob_edge_pair(R ax, R ay, R az, R Tx, R Ty, R Tz, R lI, R cx, R cy, R cz, R Ux,
                                              R Uy, R Uz, R lJ, R skipv, R half_expo, R& rho, R& rho0) {
  const R dx = ax - cx, dy = ay - cy, dz = az - cz;  // d(a, c)
  const R wx = Ty * Uz - Tz * Uy, wy = Tz * Ux - Tx * Uz, wz = Tx * Uy - Ty * Ux;  // T x U
  const R tu = Tx * Ux + Ty * Uy + Tz * Uz;
  const R xIx = Ty * dz - Tz * dy, xIy = Tz * dx - Tx * dz, xIz = Tx * dy - Ty * dx;  // T x d(a, c)
  const R yIx = xIx - lJ * wx, yIy = xIy - lJ * wy, yIz = xIz - lJ * wz;                // T x d(a, e)
  const R xJx = Uy * dz - Uz * dy, xJy = Uz * dx - Ux * dz, xJz = Ux * dy - Uy * dx;  // U x d(a, c)
  const R yJx = xJx - lI * wx, yJy = xJy - lI * wy, yJz = xJz - lI * wz;                // U x d(b, c)
  R cI1 = xIx * xIx + xIy * xIy + xIz * xIz;
  R cI2 = yIx * yIx + yIy * yIy + yIz * yIz;
  if constexpr (SKIP) {
    cI1 += skipv;
    cI2 += skipv;
  }
  const R cJ1 = xJx * xJx + xJy * xJy + xJz * xJz;
  const R cJ2 = yJx * yJx + yJy * yJy + yJz * yJz;
  const R t11 = Tx * dx + Ty * dy + Tz * dz;
  const R t12 = t11 - lJ * tu;
  const R t21 = t11 + lI, t22 = t12 + lI;
  const R r11 = t11 * t11 + cI1, r12 = t12 * t12 + cI2;
  const R r21 = t21 * t21 + cI1, r22 = t22 * t22 + cI2;
  R ri11, ri12, ri21, ri22, p11, p12, p21, p22;
  sob_powers<EC, R>(r11, half_expo, ri11, p11);
  sob_powers<EC, R>(r12, half_expo, ri12, p12);
  sob_powers<EC, R>(r21, half_expo, ri21, p21);
  sob_powers<EC, R>(r22, half_expo, ri22, p22);
  rho = (p11 + p12) + (p21 + p22);
  const R q11 = p11 * ri11 * ri11, q12 = p12 * ri12 * ri12, q21 = p21 * ri21 * ri21, q22 = p22 * ri22 * ri22;
  R z = cI1 * (q11 + q21);
  z = fma(cI2, q12 + q22, z);
  z = fma(cJ1, q11 + q12, z);
  rho0 = fma(cJ2, q21 + q22, z);
}

// ---------------------------------------------------------------------------
// one entry of the assembled operator A = B + B0 (Sec. 4.2.2-4.2.3)
// ---------------------------------------------------------------------------
// Entry (v, w), v != w, of the dense matrix the increment tables assemble: the
// sum over disjoint edges I at v and J at w of
//     -1/2 s_I(v) s_J(w) rho_IJ <T_I, T_J>  -  l_I l_J rho0_IJ / 16
// (rho_IJ: the sum over the four vertex pairs of |d|^-(2 sigma + 1); rho0_IJ
// the same weighted by the low-order kernel k_{2,4} with T_I and with T_J),
// plus, when v and w are the two ends of an edge K, -Wq_K / (2 l_K) + l_K P0_K / 16,
// with s(i1) = -1, s(i2) = +1 and Wq, P0 the per-edge sums of the operator
// kernel (edge_out slots 0 and 1).
// Off-diagonal entry A_vw (v != w) evaluated in precision R from the FP64
// geometry: coordinate differences are taken in FP64 and then rounded, so an
// FP32 entry carries a few ulps of error even for vertices close together
// (differences of rounded coordinates would lose bits in proportion to
// |x| / |x_v - x_w|).
template <typename R, int EC>
__device__ __forceinline__ R sobolev_entry(int v, int w, const V4<double>* __restrict__ GA,
                                        const V4<double>* __restrict__ GB, const V4<double>* __restrict__ GT,
                                        const int2* __restrict__ edges, const int* __restrict__ inc_off,
                                        const int* __restrict__ inc, const double* __restrict__ edge_out,
                                        R half_expo) {
  R acc = R(0);
  const int kw0 = inc_off[w], kw1 = inc_off[w + 1];
  for (int kv = inc_off[v]; kv < inc_off[v + 1]; ++kv) {
    const int I = inc[kv] >> 1;
    const R sv = (inc[kv] & 1) ? R(1) : R(-1);
    const int2 ei = edges[I];
    const V4<double> ia = GA[I], ib = GB[I], tid = GT[I];
    const R tix = (R)tid.x, tiy = (R)tid.y, tiz = (R)tid.z, li = (R)ia.w;
    for (int kw = kw0; kw < kw1; ++kw) {
      const int J = inc[kw] >> 1;
      if (I == J) {
        const double* o = edge_out + 8 * (size_t)I;  // (Wq, P0) in slots 0, 1
        const double l = ia.w;
        acc += (R)(-o[0] / (2.0 * l) + l * o[1] / 16.0);
        continue;
      }
      const int2 ej = edges[J];
      if (ei.x == ej.x || ei.x == ej.y || ei.y == ej.x || ei.y == ej.y) continue;
      const R sw = (inc[kw] & 1) ? R(1) : R(-1);
      const V4<double> ja = GA[J], jb = GB[J], tjd = GT[J];
      const R tjx = (R)tjd.x, tjy = (R)tjd.y, tjz = (R)tjd.z;
      R rho = R(0), rho0 = R(0);
      const V4<double>* P[2] = {&ia, &ib};
      const V4<double>* Q[2] = {&ja, &jb};
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const R dx = (R)(P[x]->x - Q[y]->x), dy = (R)(P[x]->y - Q[y]->y), dz = (R)(P[x]->z - Q[y]->z);
          const R r2 = dx * dx + dy * dy + dz * dz;
          const R rs = f_rsq<R>(r2), ri = rs * rs;
          const R p = pow_sigma<EC, R>(r2, rs, ri, half_expo);
          const R cI = cross_norm2<R>(tix, tiy, tiz, dx, dy, dz);
          const R cJ = cross_norm2<R>(tjx, tjy, tjz, dx, dy, dz);
          rho += p;
          rho0 += p * (cI + cJ) * ri * ri;
        }
      const R tt = tix * tjx + tiy * tjy + tiz * tjz;
      acc += R(-0.5) * sv * sw * rho * tt - R(0.0625) * li * (R)ja.w * rho0;
    }
  }
  return acc;
}

// The record of edge I from its pair sums s (the kTpeSlots accumulators):
// o = (E_I, dE/dg_i1 (3), dE/dg_i2 (3)).  A non-finite sum of an edge with a
// finite length means that a disjoint pair's kernel overflowed: coincident
// (or nearly coincident) vertices of disjoint edges, where the energy is
// infinite (Sec. 4.1); it is latched.
__device__ __forceinline__ void tpe_edge_record(const double (&s)[kTpeSlots], bool grad, double l, double Tx,
                                                double Ty, double Tz, double* __restrict__ o,
                                                unsigned* __restrict__ status) {
  o[0] = l * s[0];
  bool fin = isfinite(s[0]);
  if (grad)
    for (int k = 1; k < kTpeSlots; ++k) fin &= isfinite(s[k]);
  if (!fin && isfinite(l) && l > 0.0) latch(status, kFlagPairOverflow);
  if (!grad) return;
  const double S = s[1];
  const double Hx = s[10] - s[13] * Tx, Hy = s[11] - s[13] * Ty, Hz = s[12] - s[13] * Tz;
  o[1] = -Tx * S + l * (s[2] - s[8] * Tx) + 2.0 * Hx;
  o[2] = -Ty * S + l * (s[3] - s[8] * Ty) + 2.0 * Hy;
  o[3] = -Tz * S + l * (s[4] - s[8] * Tz) + 2.0 * Hz;
  o[4] = Tx * S + l * (s[5] - s[9] * Tx) - 2.0 * Hx;
  o[5] = Ty * S + l * (s[6] - s[9] * Ty) - 2.0 * Hy;
  o[6] = Tz * S + l * (s[7] - s[9] * Tz) - 2.0 * Hz;
}

}  // namespace rc
