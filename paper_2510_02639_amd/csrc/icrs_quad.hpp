// icrs_quad.hpp -- row-quadrature pieces shared by the ray and adjoint kernels (App. A).
#pragma once

#include "icrs_device.hpp"

namespace icrs {

template <typename T>
struct Num;
// Crossing solver limits: the safeguarded Newton usually stops after 3-4 steps; the cap
// only matters when steps leave the bracket and bisection takes over.
template <>
struct Num<double> {
  static constexpr double newton_tol = 1e-12;
  static constexpr int newton_iter = 16;
  static constexpr int fast_steps = 4;
};
template <>
struct Num<float> {
  static constexpr float newton_tol = 1e-6f;
  static constexpr int newton_iter = 12;
  static constexpr int fast_steps = 3;
};

// sqrt(c) for c >= 0 from the hardware reciprocal square root (one Newton step in FP64)
__device__ __forceinline__ double sqrt_fast(double c) {
  double y = __builtin_amdgcn_rsq(c);
  y = y * fma(-0.5 * c * y, y, 1.5);
  return c > 0.0 ? c * y : 0.0;
}
__device__ __forceinline__ float sqrt_fast(float c) { return __builtin_amdgcn_sqrtf(c); }

// f(delta) of App. A.2 (u1 > 0) or delta + 1/2 (uniform source, App. A.1)
template <typename T>
__device__ __forceinline__ T edge_factor(T delta, T u1, T delta_c) {
  if (u1 == T(0)) return delta + T(0.5);
  if (delta >= delta_c && delta > T(0))
    return (T(0.5) + delta) * T(2.0 / 3.0) * sqrt_fast(T(1) + T(0.5) * rcp_fast(delta));
  return T(2.0 / 3.0) * delta + T(0.5);
}

// Crossing of the cubic Lagrange interpolant through (t, d) = (-1,d0), (0,d1), (1,d2),
// (2,d3) with rho on the bracket [0,1] (d1, d2 on opposite sides of rho); linear between
// d1 and d2 when cubic is false.  Safeguarded Newton from the linear estimate: the bracket
// shrinks on every step and a step leaving it is replaced by bisection.  Quotients use the
// hardware reciprocal (refined once in FP64): they only steer the iteration.  slope (if
// given) receives the interpolant's slope L'(t) at the last iterate before t.
template <typename T>
__device__ inline T crossing_t(T d0, T d1, T d2, T d3, bool cubic, T rho, T* slope = nullptr) {
  const T den = d2 - d1;
  T t = (den == T(0)) ? T(0.5) : (rho - d1) * rcp_fast(den);
  t = fmin(fmax(t, T(0)), T(1));
  if (!cubic) {
    if (slope) *slope = den;
    return t;
  }
  const T c0 = d1 - rho;
  const T c1 = -d0 * T(1.0 / 3.0) - T(0.5) * d1 + d2 - d3 * T(1.0 / 6.0);
  const T c2 = T(0.5) * d0 - d1 + T(0.5) * d2;
  const T c3 = (d3 - d0) * T(1.0 / 6.0) + T(0.5) * (d1 - d2);
  // a few plain Newton steps from the linear estimate settle almost every crossing; a lane
  // whose iterate leaves the bracket or is still moving takes the safeguarded loop
  T tq = t;
  T last_step = T(0);
  T dg = c1;
#pragma unroll
  for (int it = 0; it < Num<T>::fast_steps; ++it) {
    const T g = ((c3 * tq + c2) * tq + c1) * tq + c0;
    dg = (T(3) * c3 * tq + T(2) * c2) * tq + c1;
    last_step = g * rcp_fast(dg);
    tq -= last_step;
  }
  if (tq >= T(0) && tq <= T(1) && fabs(last_step) <= Num<T>::newton_tol) {
    if (slope) *slope = dg;
    return tq;
  }
  const bool in0 = c0 < T(0);
  T a = T(0), b = T(1);
  for (int it = 0; it < Num<T>::newton_iter; ++it) {
    const T g = ((c3 * t + c2) * t + c1) * t + c0;
    dg = (T(3) * c3 * t + T(2) * c2) * t + c1;
    if (g == T(0)) break;
    if ((g < T(0)) == in0)
      a = t;
    else
      b = t;
    const T step = g * rcp_fast(dg);  // Newton step; its rounding does not move the root
    T tn = t - step;
    // converged: accept before the safeguard (t sits on a bracket end by now, and a
    // roundoff-sized step may land just outside it)
    if (fabs(step) <= Num<T>::newton_tol) {
      t = fmin(fmax(tn, a), b);
      break;
    }
    if (!(tn >= a && tn <= b)) tn = T(0.5) * (a + b);
    t = tn;
  }
  if (slope) *slope = dg;
  return t;
}


// e^{i x} - 1 without cancellation: (-2 sin^2(x/2), sin x)
__device__ __forceinline__ c64 expm1_i(double x) {
  double s, c;
  sincos(0.5 * x, &s, &c);
  return mk(-2.0 * s * s, 2.0 * s * c);
}

template <typename T>
__device__ __forceinline__ T brightness(T d2, T inv_rho2, T i_lin, T i_sqrt) {
  const T c = fmax(fma(-d2, inv_rho2, T(1)), T(0));
  return fma(i_sqrt, sqrt_fast(c), i_lin);  // I0 (1 - u1) + I0 u1 sqrt(1 - d^2/rho^2)
}

// Lagrange basis of the crossing interpolant at t and the interpolant's slope L'(t):
// cubic through t = -1, 0, 1, 2, or linear between t = 0 and 1.
template <typename T>
__device__ inline T crossing_basis(T d0, T d1, T d2, T d3, bool cubic, T t, T (&l)[4]) {
  if (!cubic) {
    l[0] = T(0);
    l[1] = T(1) - t;
    l[2] = t;
    l[3] = T(0);
    return d2 - d1;
  }
  const T tm1 = t + T(1), t1 = t - T(1), t2 = t - T(2);
  l[0] = -(t * t1 * t2) * T(1.0 / 6.0);
  l[1] = tm1 * t1 * t2 * T(0.5);
  l[2] = -(tm1 * t * t2) * T(0.5);
  l[3] = tm1 * t * t1 * T(1.0 / 6.0);
  const T c1 = -d0 * T(1.0 / 3.0) - T(0.5) * d1 + d2 - d3 * T(1.0 / 6.0);
  const T c2 = T(0.5) * d0 - d1 + T(0.5) * d2;
  const T c3 = (d3 - d0) * T(1.0 / 6.0) + T(0.5) * (d1 - d2);
  return (T(3) * c3 * t + T(2) * c2) * t + c1;
}

// Lower bound of d = |w(z) - w_c| over the arc z = z0 e^{i phi}, |phi| <= Phi, z0 = r e^{i theta_c}.
// w(z) = z + f(conj z) with f holomorphic, so for Delta = z - z0:
//   w(z) = w0 + Delta + K conj(Delta) + R2,  K = f'(conj z0) = sum_k eps_k / conj(z0 - a_k)^2,
//   |R2| <= sum_k eps_k / dmin_k^3 |Delta|^2   (dmin_k: lens k's distance to the arc's disc),
// and Delta = i z0 phi + e with |e| <= r phi^2 / 2, |Delta| <= r Phi.  The linear part traces
// the segment c + v phi (c = w0 - w_c, v = i z0 + K conj(i z0)); its distance to the origin
// less the two remainder bounds is the bound.  Returns 0 when a lens is within r Phi of z0.
// Quotients and roots use the refined hardware reciprocal and square root: their relative
// error (~1e-15) is far inside the 1e-3 margin the caller asks for.
template <int N>
__device__ inline double arc_distance_lower_bound(const Lens<N>& L, c64 wc, double r, double cth, double sth,
                                                  double Phi) {
  const double zx = r * cth, zy = r * sth;
  const double R = r * Phi;
  double wx = zx, wy = zy, kx = 0.0, ky = 0.0, M = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double ux = zx - L.a[k].x, uy = zy - L.a[k].y;
    const double u2 = fma(ux, ux, uy * uy);
    const double dmin = sqrt_fast(u2) - R;
    if (!(dmin > 0.0)) return 0.0;
    const double inv = rcp_fast(u2);
    const double gx = L.eps[k] * ux * inv, gy = L.eps[k] * uy * inv;  // eps / conj(u)
    wx -= gx;
    wy -= gy;
    kx += (gx * ux - gy * uy) * inv;  // eps / conj(u)^2 = (eps / conj(u)) (u / |u|^2)
    ky += (gx * uy + gy * ux) * inv;
    M += L.eps[k] * rcp_fast(dmin * dmin * dmin);
  }
  const double tx = -zy, ty = zx;  // i z0
  const double vx = tx + (kx * tx + ky * ty), vy = ty + (ky * tx - kx * ty);
  const double cx = wx - wc.x, cy = wy - wc.y;
  const double vv = fma(vx, vx, vy * vy);
  double phi = vv > 0.0 ? -(cx * vx + cy * vy) * rcp_fast(vv) : 0.0;
  phi = fmin(fmax(phi, -Phi), Phi);
  const double ex = fma(vx, phi, cx), ey = fma(vy, phi, cy);
  const double E = (1.0 + sqrt_fast(fma(kx, kx, ky * ky))) * 0.5 * r * Phi * Phi + M * R * R;
  return sqrt_fast(fma(ex, ex, ey * ey)) - E;
}

// d f / d delta on the branch that f(delta) takes
template <typename T>
__device__ __forceinline__ T edge_factor_slope(T delta, T u1, T delta_c) {
  if (u1 == T(0)) return T(1);
  if (delta >= delta_c && delta > T(0)) {
    const T B = sqrt(T(1) + T(1) / (T(2) * delta));
    return T(2.0 / 3.0) * (B - (T(0.5) + delta) / (T(4) * delta * delta * B));
  }
  return T(2.0 / 3.0);
}

}  // namespace icrs
