// icrs_device.hpp -- device-side building blocks of the gfx950 ICRS library.
//
// Complex arithmetic, the N-point-mass lens (Sec. 2.1, eq. lens_eq), the lens polynomial
// (eq. lens_eq_z), Ehrlich-Aberth root finding (Sec. 3.1), root validation against the
// lens equation, and the polar sector logic (Sec. 3.2).  Everything is written for one
// lane: the kernels decide how lanes share the work.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icrs {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxSectors = 10;  // per-epoch sector slots (cap 5(N-1) <= 10)
constexpr int kMaxRoots = 10;    // lens-polynomial roots per point, N^2 + 1 <= 10
constexpr int kBinsTheta = 64;
constexpr int kBinsR = 32;
constexpr int kMaxRunsR = 11;      // 32 bins, runs split by >= 2 empty bins
constexpr int kMaxRunsTheta = 21;  // 64 circular bins
constexpr int kMaxCand = kMaxRunsR * kMaxRunsTheta;

// status bits (values fixed by the public header)
constexpr uint32_t kStRootNonconv = 1u;
constexpr uint32_t kStImgCount = 2u;
constexpr uint32_t kStCapOverflow = 4u;
constexpr uint32_t kStClip = 8u;
constexpr uint32_t kStNan = 16u;
constexpr uint32_t kStGiven = 64u;
constexpr uint32_t kStLearned = 128u;
constexpr uint32_t kStFallback = 256u;
constexpr uint32_t kStImgRecheck = 512u;
constexpr uint32_t kStBadSectors = 1024u;
constexpr uint32_t kStPoint = 2048u;
constexpr uint32_t kStRedo = 1u << 30;  // internal: the epoch's limb solves are redone cold in FP64

// parameter vector layout: [s, q, u0, alpha, t0, tE, rho, u_ld, q3, r3, psi]
constexpr int kParams = 11;

// ---------------------------------------------------------------------------------------
template <typename T>
struct cx {
  T x, y;
};
using c64 = cx<double>;
using c32 = cx<float>;

template <typename T>
__device__ __forceinline__ cx<T> mk(T x, T y) {
  return cx<T>{x, y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) {
  return {-a.x, -a.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return {s * a.x, s * a.y};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) {
  return {a.x, -a.y};
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) {
  return a.x * a.x + a.y * a.y;
}
// Reciprocals from the hardware approximations (v_rcp_f64 is good to about 2^-24, v_rcp_f32
// to 1 ulp) refined by one Newton step in FP64: relative error about 2^-48.
__device__ __forceinline__ double rcp_fast(double x) {
  double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ __forceinline__ cx<T> recip(cx<T> b) {
  const T n = rcp_fast(norm2(b));
  return {b.x * n, -b.y * n};
}
template <typename T>
__device__ __forceinline__ cx<T> operator/(cx<T> a, cx<T> b) {
  return a * recip(b);
}
template <typename T>
__device__ __forceinline__ bool is_zero(cx<T> a) {
  return a.x == T(0) && a.y == T(0);
}
__device__ __forceinline__ c32 to32(c64 a) { return {float(a.x), float(a.y)}; }
__device__ __forceinline__ c64 to64(c32 a) { return {double(a.x), double(a.y)}; }

// ---------------------------------------------------------------------------------------
// Lens of N point masses: fractional masses eps (sum 1) at complex positions a.
template <int N>
struct Lens {
  double eps[N];
  c64 a[N];
};

// Frame of Sec. 2.1 / Fig. 3: q = m2/m1, the pair on the real axis with its barycentre at
// the origin (primary at -q s/(1+q)); the third mass q3 = m3/m1 at r3 e^{i psi} from the
// pair's midpoint.
template <int N>
__device__ inline Lens<N> make_lens(const double* p) {
  Lens<N> L;
  const double s = p[0], q = p[1];
  const double pair = 1.0 + q;
  const double q3 = (N == 3) ? p[8] : 0.0;
  const double m = pair + q3;
  L.eps[0] = 1.0 / m;
  L.eps[1] = q / m;
  L.a[0] = mk(-q * s / pair, 0.0);
  L.a[1] = mk(s / pair, 0.0);
  if constexpr (N == 3) {
    L.eps[2] = q3 / m;
    double sp, cp;
    sincos(p[10], &sp, &cp);
    const double mid = 0.5 * (L.a[0].x + L.a[1].x);
    L.a[2] = mk(mid + p[9] * cp, p[9] * sp);
  }
  return L;
}

// Source centre on the straight trajectory: tau = (t - t0)/tE, moving along e^{i alpha},
// closest approach u0 e^{i(alpha + pi/2)} at t = t0.
__device__ inline c64 source_center(const double* p, double t) {
  const double tau = (t - p[4]) / p[5];
  double sa, ca;
  sincos(p[3], &sa, &ca);
  return mk(tau * ca - p[2] * sa, tau * sa + p[2] * ca);
}

// eq. lens_eq: w = z - sum_k eps_k / conj(z - a_k)
template <int N>
__device__ __forceinline__ c64 lens_map(const Lens<N>& L, c64 z) {
  c64 w = z;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const c64 d = z - L.a[k];
    const double inv = L.eps[k] / norm2(d);
    w = w - mk(d.x * inv, d.y * inv);  // eps/conj(d) = eps d / |d|^2
  }
  return w;
}

// kappa = sum_k eps_k / conj(z - a_k)^2 (eq. detJ: det J = 1 - |kappa|^2)
template <int N>
__device__ __forceinline__ c64 lens_kappa(const Lens<N>& L, c64 z) {
  c64 k = mk(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const c64 d = conj(z - L.a[i]);
    k = k + L.eps[i] * recip(d * d);
  }
  return k;
}

// ---------------------------------------------------------------------------------------
// Lens polynomial (eq. lens_eq_z), degree N^2 + 1.  With H = prod_k (z - a_k) and
// G = conj(w) H + sum_k eps_k prod_{j != k}(z - a_j), conj(z) = G/H on an image; writing
// D_i = G - conj(a_i) H and clearing denominators of eq. lens_eq gives
//   P = (z - w) prod_i D_i - H sum_i eps_i prod_{j != i} D_j.
// Fixed-size coefficient arrays, ascending powers.
template <int A, int B>
__device__ __forceinline__ void pmul(const c64 (&a)[A], const c64 (&b)[B], c64 (&c)[A + B - 1]) {
#pragma unroll
  for (int i = 0; i < A + B - 1; ++i) c[i] = mk(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < A; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) c[i + j] = c[i + j] + a[i] * b[j];
}

template <int N>
__device__ inline void lens_polynomial(const Lens<N>& L, c64 w, c64 (&P)[N * N + 2]) {
  // monic linear factors (z - a_k)
  c64 H[N + 1];
  c64 G[N + 1];
  c64 E[N][N];  // E[k] = prod_{j != k} (z - a_j), degree N-1
  if constexpr (N == 2) {
    H[0] = L.a[0] * L.a[1];
    H[1] = -(L.a[0] + L.a[1]);
    H[2] = mk(1.0, 0.0);
    E[0][0] = -L.a[1];
    E[0][1] = mk(1.0, 0.0);
    E[1][0] = -L.a[0];
    E[1][1] = mk(1.0, 0.0);
  } else {
    const c64 a0 = L.a[0], a1 = L.a[1], a2 = L.a[2];
    H[0] = -(a0 * a1 * a2);
    H[1] = a0 * a1 + a0 * a2 + a1 * a2;
    H[2] = -(a0 + a1 + a2);
    H[3] = mk(1.0, 0.0);
    const c64 pr[3][2] = {{a1, a2}, {a0, a2}, {a0, a1}};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      E[k][0] = pr[k][0] * pr[k][1];
      E[k][1] = -(pr[k][0] + pr[k][1]);
      E[k][2] = mk(1.0, 0.0);
    }
  }
  const c64 wb = conj(w);
#pragma unroll
  for (int j = 0; j <= N; ++j) G[j] = wb * H[j];
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int j = 0; j < N; ++j) G[j] = G[j] + L.eps[k] * E[k][j];
  c64 D[N][N + 1];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j <= N; ++j) D[i][j] = G[j] - conj(L.a[i]) * H[j];

  if constexpr (N == 2) {
    c64 prodD[5];
    pmul(D[0], D[1], prodD);
    // S = eps0 D1 + eps1 D0 (degree 2)
    c64 S[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) S[j] = L.eps[0] * D[1][j] + L.eps[1] * D[0][j];
    c64 HS[5];
    pmul(H, S, HS);
    const c64 zw[2] = {-w, mk(1.0, 0.0)};
    c64 Z[6];
    pmul(zw, prodD, Z);
#pragma unroll
    for (int j = 0; j < 6; ++j) P[j] = (j < 5) ? Z[j] - HS[j] : Z[j];
  } else {
    c64 D01[7], D02[7], D12[7];
    pmul(D[0], D[1], D01);
    pmul(D[0], D[2], D02);
    pmul(D[1], D[2], D12);
    c64 prodD[10];
    pmul(D01, D[2], prodD);
    c64 S[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) S[j] = L.eps[0] * D12[j] + L.eps[1] * D02[j] + L.eps[2] * D01[j];
    c64 HS[10];
    pmul(H, S, HS);
    const c64 zw[2] = {-w, mk(1.0, 0.0)};
    c64 Z[11];
    pmul(zw, prodD, Z);
#pragma unroll
    for (int j = 0; j < 11; ++j) P[j] = (j < 10) ? Z[j] - HS[j] : Z[j];
  }
}

// ---------------------------------------------------------------------------------------
// Ehrlich-Aberth (Sec. 3.1) in precision T, all roots updated together:
//   z_k <- z_k - 1 / (P'(z_k)/P(z_k) - sum_{j != k} 1/(z_k - z_j)),
// started on the Cauchy-radius circle R = 1 + max_{j<n} |b_j/b_n| at angles
// 2 pi k/n + pi/(2n).  A root stops moving once its step is below 1e-14 max(1,|z|)
// (FP64; 1e-6 in FP32) or |P(z)| is at the rounding noise 8 n u sum_j |b_j||z|^j.
// Returns the iterations used; *conv tells whether every root stopped before max_iter.
template <typename T>
struct EAConst;
template <>
struct EAConst<double> {
  static constexpr double unit = 1.1102230246251565e-16;
  static constexpr double step_tol = 1e-14;
};
template <>
struct EAConst<float> {
  static constexpr float unit = 5.9604645e-8f;
  static constexpr float step_tol = 1e-6f;
};

__device__ __forceinline__ void sincos_t(double a, double* s, double* c) { sincos(a, s, c); }
__device__ __forceinline__ void sincos_t(float a, float* s, float* c) { sincosf(a, s, c); }

template <typename T, int D>
__device__ inline int ehrlich_aberth(const cx<T> (&b)[D + 1], cx<T> (&z)[D], int max_iter, bool* conv,
                                     bool warm = false, bool noise_stop = true) {
  T absb[D + 1];
#pragma unroll
  for (int j = 0; j <= D; ++j) absb[j] = sqrt(norm2(b[j]));
  if (!warm) {
    T R = T(0);
    const T inv_lead = T(1) / absb[D];
#pragma unroll
    for (int j = 0; j < D; ++j) R = fmax(R, absb[j] * inv_lead);
    R += T(1);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T s, c;
      const T ang = T(2) * T(kPi) * T(k) / T(D) + T(kPi) / T(2 * D);
      sincos_t(ang, &s, &c);
      z[k] = mk(R * c, R * s);
    }
  }
  uint32_t done = 0;
  constexpr uint32_t all = (1u << D) - 1u;
  int it = 0;
  for (; it < max_iter && done != all; ++it) {
    cx<T> step[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      step[k] = mk(T(0), T(0));
      if (done & (1u << k)) continue;
      // Horner for P and P'
      cx<T> p = b[D], dp = mk(T(0), T(0));
#pragma unroll
      for (int j = D - 1; j >= 0; --j) {
        dp = dp * z[k] + p;
        p = p * z[k] + b[j];
      }
      const T az = sqrt(norm2(z[k]));
      T noise = absb[D];
#pragma unroll
      for (int j = D - 1; j >= 0; --j) noise = noise * az + absb[j];
      noise *= T(8 * D) * EAConst<T>::unit;
      // P(z) exactly zero: z is a root and its correction P/P' / (1 - (P/P') S) is zero
      // (dividing by P would give NaN and spread it to every root through S)
      if (is_zero(p) || (noise_stop && norm2(p) <= noise * noise)) {
        done |= 1u << k;
        continue;
      }
      cx<T> rep = mk(T(0), T(0));
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (j == k) continue;
        const cx<T> dz = z[k] - z[j];
        if (!is_zero(dz)) rep = rep + recip(dz);
      }
      const cx<T> den = dp / p - rep;
      step[k] = is_zero(den) ? mk(T(0), T(0)) : recip(den);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (done & (1u << k)) continue;
      z[k] = z[k] - step[k];
      const T tol = EAConst<T>::step_tol * fmax(T(1), sqrt(norm2(z[k])));
      if (norm2(step[k]) <= tol * tol) done |= 1u << k;
    }
  }
  *conv = (done == all);
  return it;
}

// ---------------------------------------------------------------------------------------
// Validation (Sec. 2.1: roots are checked by substitution into eq. lens_eq).  Each candidate
// is polished by Newton steps on the lens equation itself -- the step solving
// dz + kappa conj(dz) = -F is (kappa conj(F) - F)/(1 - |kappa|^2) -- and is kept when
// |F| <= 1e-10, unless it lies within 1e-9 max(1,|z|) of an image already kept.  Steps stop
// when a step falls below 1e-14 max(1,|z|); after the first 8, a candidate goes on only while
// it is within the residual bound or its |F| at least halves per step, 24 steps at most.  The
// first rule: a spurious root of the polynomial can drift into an image's basin and stop
// inside the residual bound but outside the duplicate radius, where it would count as a
// second copy of that image.  The second: a root of a tight cluster is only as accurate as
// the cluster's conditioning allows (~1e-5 next to a planet), and Newton from there first
// crosses the critical curve between the two images; a fixed 8-step cap rejected such an
// image while its residual was still falling quadratically, which can leave a valid but
// wrong image count.
constexpr int kPolishMaxSteps = 24;
template <int N>
__device__ inline c64 polish(const Lens<N>& L, c64 w, c64 z) {
  double f_prev = __builtin_inf();
  for (int s = 0; s < kPolishMaxSteps; ++s) {
    const c64 F = lens_map(L, z) - w;
    const double f = norm2(F);
    if (s >= 8 && !(f <= 1e-20) && !(f <= 0.25 * f_prev)) break;
    f_prev = f;
    const c64 k = lens_kappa(L, z);
    const double den = 1.0 - norm2(k);
    if (den == 0.0 || !isfinite(den)) break;
    const c64 num = k * conj(F) - F;
    const c64 dz = mk(num.x / den, num.y / den);
    z = z + dz;
    const double lim = 1e-14 * fmax(1.0, sqrt(norm2(z)));
    if (norm2(dz) <= lim * lim) break;
  }
  return z;
}

template <int N>
__device__ __forceinline__ bool count_ok(int c) {
  constexpr int lo = N + 1, hi = 5 * (N - 1);
  return c >= lo && c <= hi && ((c - lo) & 1) == 0;
}

// The image list lives in registers: every access below uses a compile-time index (the
// loops are unrolled and the slot is chosen by predication), so no write depends on a
// lane-varying register index.
template <int N, int M>
__device__ inline void accept_image(const Lens<N>& L, c64 w, c64 z0, c64 (&img)[M], int& n) {
  const c64 z = polish(L, w, z0);
  const c64 F = lens_map(L, z) - w;
  if (!(norm2(F) <= 1e-20)) return;
  const double lim = 1e-9 * fmax(1.0, sqrt(norm2(z)));
  bool dup = false;
#pragma unroll
  for (int j = 0; j < M; ++j) dup = dup || (j < n && norm2(z - img[j]) <= lim * lim);
  if (dup || n >= M) return;
#pragma unroll
  for (int j = 0; j < M; ++j)
    if (j == n) img[j] = z;
  ++n;
}

// Final substitution check of the kept list: every image is put through eq. lens_eq once
// more and dropped (with kStImgRecheck) unless it still satisfies |F| <= 1e-10.  The
// acceptance test above already guarantees this; the check makes a list that breaks it
// visible in the status word instead of passing it on.
template <int N, int M>
__device__ inline uint32_t recheck_images(const Lens<N>& L, c64 w, c64 (&img)[M], int& n) {
  c64 out[M];
  int m = 0;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    out[j] = mk(0.0, 0.0);
    if (j < n && norm2(lens_map(L, img[j]) - w) <= 1e-20) {
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (k == m) out[k] = img[j];
      ++m;
    }
  }
  const uint32_t st = (m == n) ? 0u : kStImgRecheck;
#pragma unroll
  for (int j = 0; j < M; ++j) img[j] = out[j];
  n = m;
  return st;
}

// Validation of the D roots zr (Sec. 2.1): polish and keep each as described above; if the
// count is not one of N+1, N+3, .., 5(N-1), try the leading-order images next to each lens,
// z = a_k - eps_k / conj(w' - a_k) with w' shifted by the other lenses' deflection at a_k.
// Returns the status bits of the list (kStImgCount if the count stays invalid).
template <int N>
__device__ inline uint32_t validate_roots(const Lens<N>& L, c64 w, const c64 (&zr)[N * N + 1],
                                          c64 (&img)[N * N + 1], int& n_img) {
  constexpr int D = N * N + 1;
  uint32_t st = 0;
  n_img = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) accept_image<N, D>(L, w, zr[k], img, n_img);
  if (!count_ok<N>(n_img)) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      c64 wk = w;
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j != k) wk = wk + L.eps[j] * recip(conj(L.a[k] - L.a[j]));
      const c64 seed = L.a[k] - L.eps[k] * recip(conj(wk - L.a[k]));
      accept_image<N, D>(L, w, seed, img, n_img);
    }
    if (!count_ok<N>(n_img)) st |= kStImgCount;
  }
  const uint32_t rc = recheck_images<N, D>(L, w, img, n_img);
  if (rc && !count_ok<N>(n_img)) st |= kStImgCount;
  return st | rc;
}

// All validated images of the point source at w.  Cold start: EA in precision T (FP32 roots
// are then refined by FP64 EA).  With warm (the D roots of a nearby point's polynomial, e.g.
// the source centre's for a limb point) FP64 EA starts there and needs a few iterations; a
// warm start that does not converge, or two of whose roots coincide, falls back to the cold
// path.  With kCold64Retry, a cold FP32 solve whose roots validate to a forbidden image count
// is redone by FP64 EA from the Cauchy circle: inside a cluster of roots next to a low-mass
// lens, FP32 iterates can merge before the FP64 stage separates them.  (The limb kernels
// handle a warm start that validates to a forbidden count by re-running the epoch cold in
// FP64; a retry here would cost the limb kernel its register budget.)  roots_out, if given,
// receives the D polynomial roots.  Returns status bits.
constexpr int kEAWarmIter = 50;
constexpr int kEAMaxIterCold64 = 500;
constexpr int kEAContinueIter = 100;

template <int N, typename T, bool kCold64Retry = false>
__device__ inline uint32_t find_images(const Lens<N>& L, c64 w, c64 (&img)[N * N + 1], int& n_img, int max_iter,
                                       const c64* warm = nullptr, c64* roots_out = nullptr) {
  constexpr int D = N * N + 1;
  c64 P[D + 1];
  lens_polynomial<N>(L, w, P);
  c64 zr[D];
  bool conv = false, conv_warm = false;
  if (warm) {
#pragma unroll
    for (int k = 0; k < D; ++k) zr[k] = warm[k];
    conv = true;
    ehrlich_aberth<double, D>(P, zr, kEAWarmIter, &conv, true);
    // two starts that settled on one root (the repulsion normally prevents it) leave a root
    // unfound: take the cold path then
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = i + 1; j < D; ++j)
        if (norm2(zr[i] - zr[j]) <= 1e-24 * fmax(1.0, norm2(zr[i]))) conv = false;
    conv_warm = conv;
  }
  if (!conv) {
    cx<T> b[D + 1];
#pragma unroll
    for (int j = 0; j <= D; ++j) b[j] = mk(T(P[j].x), T(P[j].y));
    cx<T> z[D];
    conv = true;
    ehrlich_aberth<T, D>(b, z, max_iter, &conv);
#pragma unroll
    for (int k = 0; k < D; ++k) zr[k] = mk(double(z[k].x), double(z[k].y));
    if constexpr (sizeof(T) == 4) {
      // FP64 Ehrlich-Aberth from the FP32 roots: the repulsion keeps clustered roots next to
      // a low-mass lens apart while they converge (FP32 alone cannot resolve them)
      bool conv64 = true;
      ehrlich_aberth<double, D>(P, zr, 50, &conv64, true);
      conv = conv64;
    }
  }
  uint32_t st = validate_roots<N>(L, w, zr, img, n_img) | (conv ? 0u : kStRootNonconv);
  bool fp64_cold = sizeof(T) == 8 && !(warm && conv_warm);
  if constexpr (kCold64Retry && sizeof(T) == 4) {
    if (!warm && (st & (kStImgCount | kStRootNonconv))) {
      bool conv64 = true;
      ehrlich_aberth<double, D>(P, zr, kEAMaxIterCold64, &conv64);
      st = validate_roots<N>(L, w, zr, img, n_img) | (conv64 ? 0u : kStRootNonconv);
      fp64_cold = true;
    }
  }
  if constexpr (sizeof(T) == 8 || kCold64Retry) {
    // Two estimates that stopped on the rounding-noise test inside one root's neighbourhood
    // (a tight cluster next to a low-mass lens) leave a root, and its image, unfound.  Last
    // resort of a cold FP64 solve: continue the iteration from the current estimates with the
    // step test only (the repulsion then separates the pair), at most 100 iterations, and
    // validate again.
    if (fp64_cold && (st & kStImgCount)) {
      bool conv64 = true;
      ehrlich_aberth<double, D>(P, zr, kEAContinueIter, &conv64, true, false);
      st = validate_roots<N>(L, w, zr, img, n_img) | (st & kStRootNonconv);
    }
  }
  if (roots_out) {
#pragma unroll
    for (int k = 0; k < D; ++k) roots_out[k] = zr[k];
  }
  return st;
}

// ---------------------------------------------------------------------------------------
// Polar sectors (Sec. 3.2).  The decision logic here is kept free of fused multiply-adds so
// that bin and overlap decisions round exactly like plain IEEE double arithmetic.
struct Sector {
  double r_lo, r_hi, th_lo, th_hi;
  int periodic;
};

#pragma clang fp contract(off)

__device__ inline void normalise_theta(Sector& s) {
  // a non-finite or far-out angle (only from corrupt input) becomes a full ring, so the
  // shifting loops below always end
  const bool wild = !(fabs(s.th_lo) < 64.0 && fabs(s.th_hi) < 64.0);
  if (s.periodic || wild || s.th_hi - s.th_lo >= 2.0 * kPi) {
    s.periodic = 1;
    s.th_lo = -kPi;
    s.th_hi = kPi;
    return;
  }
  while (s.th_lo < -kPi) {
    s.th_lo += 2.0 * kPi;
    s.th_hi += 2.0 * kPi;
  }
  while (s.th_lo >= kPi) {
    s.th_lo -= 2.0 * kPi;
    s.th_hi -= 2.0 * kPi;
  }
}

// shift k in {-1,0,1} (in units of 2 pi) that makes b's theta range meet a's; 2 if none
__device__ inline int theta_shift(const Sector& a, const Sector& b) {
  if (a.periodic || b.periodic) return 0;
  for (int k = -1; k <= 1; ++k) {
    const double lo = b.th_lo + 2.0 * kPi * k, hi = b.th_hi + 2.0 * kPi * k;
    if (lo <= a.th_hi && a.th_lo <= hi) return k;
  }
  return 2;
}

__device__ inline bool sectors_overlap(const Sector& a, const Sector& b) {
  if (!(a.r_lo <= b.r_hi && b.r_lo <= a.r_hi)) return false;
  return theta_shift(a, b) != 2;
}

__device__ inline Sector sector_union(const Sector& a, const Sector& b) {
  Sector u;
  u.r_lo = fmin(a.r_lo, b.r_lo);
  u.r_hi = fmax(a.r_hi, b.r_hi);
  u.periodic = a.periodic | b.periodic;
  if (u.periodic) {
    u.th_lo = -kPi;
    u.th_hi = kPi;
    return u;
  }
  int k = theta_shift(a, b);
  if (k == 2) {  // disjoint in theta: join across the shorter way round
    double best = 1e300;
    for (int kk = -1; kk <= 1; ++kk) {
      const double lo = fmin(a.th_lo, b.th_lo + 2.0 * kPi * kk);
      const double hi = fmax(a.th_hi, b.th_hi + 2.0 * kPi * kk);
      if (hi - lo < best) {
        best = hi - lo;
        k = kk;
      }
    }
  }
  u.th_lo = fmin(a.th_lo, b.th_lo + 2.0 * kPi * k);
  u.th_hi = fmax(a.th_hi, b.th_hi + 2.0 * kPi * k);
  normalise_theta(u);
  return u;
}

__device__ inline double sector_area(const Sector& s) {
  return 0.5 * (s.r_hi * s.r_hi - s.r_lo * s.r_lo) * (s.th_hi - s.th_lo);
}

// merge overlapping pairs into their bounding box until none overlap (lowest pair first)
__device__ inline void merge_to_fixpoint(Sector* S, int& n) {
  bool changed = true;
  while (changed) {
    changed = false;
    for (int i = 0; i < n && !changed; ++i)
      for (int j = i + 1; j < n && !changed; ++j)
        if (sectors_overlap(S[i], S[j])) {
          S[i] = sector_union(S[i], S[j]);
          for (int m = j; m + 1 < n; ++m) S[m] = S[m + 1];
          --n;
          changed = true;
        }
  }
}

// stable insertion sort by (theta_lo, r_lo)
__device__ inline void sort_sectors(Sector* S, int n) {
  for (int i = 1; i < n; ++i) {
    const Sector x = S[i];
    int j = i - 1;
    while (j >= 0 && (S[j].th_lo > x.th_lo || (S[j].th_lo == x.th_lo && S[j].r_lo > x.r_lo))) {
      S[j + 1] = S[j];
      --j;
    }
    S[j + 1] = x;
  }
}

// clip bits: 1 inside rays in the first row, 2 last row, 4 first column, 8 last column.
// The touched side is widened by half the sector's extent.
__device__ inline void widen_sector(Sector& s, int clip) {
  const double er = s.r_hi - s.r_lo;
  if (clip & 1) s.r_lo = fmax(s.r_lo - 0.5 * er, 0.0);
  if (clip & 2) s.r_hi += 0.5 * er;
  if (!s.periodic) {
    const double et = s.th_hi - s.th_lo;
    if (clip & 4) s.th_lo -= 0.5 * et;
    if (clip & 8) s.th_hi += 0.5 * et;
    normalise_theta(s);
  }
}

// Candidate box (member min/max) to sector: safety margin of 0.1 x extent + a floor of
// rho/100 in r and rho/(100 r_mid) in theta on each side, r_lo >= 0, full ring when the
// theta run covers every bin or the widened extent reaches 2 pi.
__device__ inline Sector candidate_to_sector(double r_lo, double r_hi, double th_lo, double th_hi, int full,
                                             double rho) {
  Sector s;
  const double r_mid = 0.5 * (r_lo + r_hi);
  const double mr = 0.1 * (r_hi - r_lo) + rho / 100.0;
  const double mt = 0.1 * (th_hi - th_lo) + rho / (100.0 * r_mid);
  s.r_lo = fmax(r_lo - mr, 0.0);
  s.r_hi = r_hi + mr;
  s.th_lo = th_lo;
  s.th_hi = th_hi;
  s.periodic = full;
  if (!full) {
    s.th_lo -= mt;
    s.th_hi += mt;
  }
  normalise_theta(s);
  return s;
}

__device__ __forceinline__ int theta_bin(double th) {
  const double w = 2.0 * kPi / kBinsTheta;
  int b = (int)floor((th + kPi) / w);
  return min(max(b, 0), kBinsTheta - 1);
}

__device__ __forceinline__ int r_bin(double r, double rmin, double wr) {
  int b = (int)floor((r - rmin) / wr);
  return min(max(b, 0), kBinsR - 1);
}

#pragma clang fp contract(on)

// order-preserving map of doubles to unsigned 64-bit keys (for LDS atomic min/max)
__device__ __forceinline__ unsigned long long dkey(double v) {
  const unsigned long long b = __double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(b);
}

}  // namespace icrs
