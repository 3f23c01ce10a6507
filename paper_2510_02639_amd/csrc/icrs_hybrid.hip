// icrs_hybrid.hip -- the hybrid light curve (Sec. 3.4, item iii) and the point-source
// gradient (Sec. 3.5).
//
// The paper models only a preselected set of epochs with finite-source effects and uses the
// point-source magnification of eq. amp_point elsewhere; it gives no selection rule.  The
// rule here: n_check points on the circle of radius guard x rho around the source centre are
// solved like the centre (warm-started from the centre's roots); an epoch is extended when
// one of them changes the image count or carries a root flag (a caustic crosses the circle),
// when their mean point-source magnification differs from the centre's by more than
// tol x A_ps (that difference measures the Laplacian of A_ps, which leads the finite-source
// correction), or when one of them differs by more than vary_max x A_ps.  Extended epochs go
// through the plain path; every other epoch takes A_ps.
//
// hybrid_select_kernel: groups of P lanes per epoch (P a power of two covering n_check), a
// lane per circle point, butterfly reductions inside the group (fixed order).
// point_jacobian_kernel: one lane per epoch.  Images z of the centre satisfy
// F = z - sum_k eps_k / conj(z - a_k) - w = 0; a parameter change moves them by
//   dz + kappa conj(dz) = R,  R = dw + sum_k deps_k / conj(z - a_k) + sum_k eps_k conj(da_k) / conj(z - a_k)^2,
//   dz = (R - kappa conj(R)) / (1 - |kappa|^2),
// and each image's magnification 1/|det J|, det J = 1 - |kappa|^2 (eq. detJ), changes by
// 2 s_j Re(conj(kappa) dkappa) / det J^2 with s_j = sign det J and
//   dkappa = sum_k deps_k / conj(z - a_k)^2 - 2 eps_k (conj(dz) - conj(da_k)) / conj(z - a_k)^3.
// This is the implicit derivative of the roots (Sec. 3.5) taken on the lens equation, whose
// solutions are the validated polynomial roots.
#include "icrs_device.hpp"
#include "icrs_launch.hpp"

namespace icrs {
namespace {

constexpr int kEAMaxIterFP64 = 500;
constexpr int kEAMaxIterFP32 = 200;

template <int N>
__device__ inline double point_mag(const Lens<N>& L, const c64 (&img)[N * N + 1], int n) {
  double A = 0.0;
#pragma unroll
  for (int j = 0; j < N * N + 1; ++j)
    if (j < n) A += 1.0 / fabs(1.0 - norm2(lens_kappa(L, img[j])));
  return A;
}

template <int N, typename T>
__global__ __launch_bounds__(256) void hybrid_select_kernel(Batch b, int n_check, int P, double guard, double tol,
                                                            double vary_max, const int32_t* __restrict__ cn,
                                                            const double* __restrict__ a_c,
                                                            const double* __restrict__ roots, double* __restrict__ mag,
                                                            uint32_t* __restrict__ status, int32_t* __restrict__ nsec,
                                                            int32_t* __restrict__ ext_list,
                                                            int32_t* __restrict__ ext_count) {
  constexpr int MI = N * N + 1;
  const int G = blockDim.x / P;
  const int g = threadIdx.x / P, k = threadIdx.x % P;
  const int64_t e = (int64_t)blockIdx.x * G + g;
  const bool valid = e < b.n_epochs;
  const int64_t ee = valid ? e : 0;  // lanes past the end compute on epoch 0 and write nothing
  const double* p = b.params + (int64_t)b.epoch_event[ee] * kParams;
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = source_center(p, b.t[ee]);
  const int nc = cn[ee];
  const double Ac = a_c[ee];
  int bad = 0;
  double A = 0.0, dev = 0.0;
  if (k < n_check) {
    double sp, cp;
    sincospi(2.0 * k / n_check, &sp, &cp);
    const double rad = guard * p[6];
    const c64 w = mk(wc.x + rad * cp, wc.y + rad * sp);
    c64 img[MI], warm[MI];
#pragma unroll
    for (int j = 0; j < MI; ++j) warm[j] = mk(roots[(ee * kMaxRoots + j) * 2], roots[(ee * kMaxRoots + j) * 2 + 1]);
    int n = 0;
    const uint32_t st = find_images<N, T>(L, w, img, n, sizeof(T) == 8 ? kEAMaxIterFP64 : kEAMaxIterFP32, warm);
    bad = (st != 0u || n != nc) ? 1 : 0;
    A = point_mag<N>(L, img, n);
    dev = fabs(A - Ac);
  }
  // group reductions (butterflies inside the P lanes: the same order on every run)
  for (int off = P >> 1; off >= 1; off >>= 1) {
    A += __shfl_xor(A, off, P);
    dev = fmax(dev, __shfl_xor(dev, off, P));
    bad |= __shfl_xor(bad, off, P);
  }
  if (!valid || k != 0) return;
  const bool extended = (status[e] & (kStRootNonconv | kStImgCount | kStImgRecheck)) != 0u || bad != 0 ||
                        !(fabs(A / n_check - Ac) <= tol * Ac) || !(dev <= vary_max * Ac);
  nsec[e] = 0;
  if (extended) {
    ext_list[atomicAdd(ext_count, 1)] = (int32_t)e;
  } else {
    mag[e] = Ac;
    status[e] = kStPoint;
  }
}

// d(source centre)/d(u0, alpha, t0, tE) and d(eps_k, a_k)/d(s, q, q3, r3, psi) as in the
// adjoint's chain rule; A_ps and its 11 derivatives of epoch e.
template <int N, typename T>
__device__ inline void point_jacobian_epoch(const Batch& b, int64_t e, double* A_out, double* jac, uint32_t* st_out) {
  constexpr int MI = N * N + 1;
  constexpr int NP = kParams;
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = source_center(p, b.t[e]);
  c64 img[MI];
  int n = 0;
  *st_out = find_images<N, T, true>(L, wc, img, n, sizeof(T) == 8 ? kEAMaxIterFP64 : kEAMaxIterFP32);
  // parameter tangents of the frame and of the source centre
  const double s = p[0], q = p[1];
  const double q3 = (N == 3) ? p[8] : 0.0;
  const double pair = 1.0 + q, m = pair + q3;
  double deps[N][NP] = {};
  c64 da[N][NP];
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int c = 0; c < NP; ++c) da[k][c] = mk(0.0, 0.0);
  // eps_0 = 1/m, eps_1 = q/m, eps_2 = q3/m
  deps[0][1] = -1.0 / (m * m);
  deps[1][1] = (1.0 + q3) / (m * m);
  if constexpr (N == 3) {
    deps[2][1] = -q3 / (m * m);
    deps[0][8] = -1.0 / (m * m);
    deps[1][8] = -q / (m * m);
    deps[2][8] = pair / (m * m);
  }
  // a_0 = -q s/(1+q), a_1 = s/(1+q); a_2 = midpoint + r3 e^{i psi}
  da[0][0] = mk(-q / pair, 0.0);
  da[1][0] = mk(1.0 / pair, 0.0);
  da[0][1] = mk(-s / (pair * pair), 0.0);
  da[1][1] = mk(-s / (pair * pair), 0.0);
  if constexpr (N == 3) {
    double sp3, cp3;
    sincos(p[10], &sp3, &cp3);
    da[2][0] = mk((1.0 - q) / (2.0 * pair), 0.0);
    da[2][1] = mk(-s / (pair * pair), 0.0);
    da[2][9] = mk(cp3, sp3);
    da[2][10] = mk(-p[9] * sp3, p[9] * cp3);
  }
  double sa, ca;
  sincos(p[3], &sa, &ca);
  const double tau = (b.t[e] - p[4]) / p[5];
  c64 dw[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) dw[c] = mk(0.0, 0.0);
  dw[2] = mk(-sa, ca);                                // u0
  dw[3] = mk(-wc.y, wc.x);                            // alpha
  dw[4] = mk(-ca / p[5], -sa / p[5]);                 // t0
  dw[5] = mk(-ca * tau / p[5], -sa * tau / p[5]);     // tE
  double A = 0.0;
  double dA[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) dA[c] = 0.0;
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    if (j >= n) continue;
    const c64 z = img[j];
    c64 u1[N], u2[N], u3[N];  // 1/conj(z - a_k)^{1,2,3}
    c64 kap = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const c64 d = conj(z - L.a[k]);
      u1[k] = recip(d);
      u2[k] = u1[k] * u1[k];
      u3[k] = u2[k] * u1[k];
      kap = kap + L.eps[k] * u2[k];
    }
    const double det = 1.0 - norm2(kap);
    const double sgn = det > 0.0 ? 1.0 : -1.0;
    A += sgn / det;
    const double kn = 1.0 / det;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      c64 R = dw[c];
#pragma unroll
      for (int k = 0; k < N; ++k) R = R + deps[k][c] * u1[k] + L.eps[k] * (conj(da[k][c]) * u2[k]);
      const c64 dz = kn * (R - kap * conj(R));
      c64 dk = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < N; ++k) dk = dk + deps[k][c] * u2[k] - (2.0 * L.eps[k]) * ((conj(dz) - conj(da[k][c])) * u3[k]);
      const double re = kap.x * dk.x + kap.y * dk.y;  // Re(conj(kappa) dkappa)
      dA[c] += 2.0 * sgn * re * kn * kn;
    }
  }
  *A_out = A;
#pragma unroll
  for (int c = 0; c < NP; ++c) jac[c] = dA[c];
}

// one lane per epoch; with only_status, epochs whose status lacks it are skipped
template <int N, typename T>
__global__ __launch_bounds__(64) void point_jacobian_kernel(Batch b, double* __restrict__ a_ps, double* __restrict__ jac,
                                                            uint32_t* __restrict__ status_out,
                                                            const uint32_t* __restrict__ status_in,
                                                            uint32_t only_status) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.n_epochs) return;
  if (only_status && !(status_in[e] & only_status)) return;
  double A, J[kParams];
  uint32_t st;
  point_jacobian_epoch<N, T>(b, e, &A, J, &st);
  if (a_ps) a_ps[e] = A;
  for (int c = 0; c < kParams; ++c) jac[e * kParams + c] = J[c];
  if (status_out) status_out[e] = st;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Grid-free reference (Sec. 2.2): the finite-source magnification is the brightness-weighted
// mean of the point-source magnification (eq. amp_point) over the source disk.  Radius
// nodes: Gauss-Legendre in x on [0, pi/2] with r = sin x, which turns the limb-darkening
// factor sqrt(1 - r^2) into cos x; angle nodes: midpoints of n_phi equal arcs.  The mean is
// only a quadrature of a smooth integrand while no caustic crosses the disk: changes[e]
// counts the nodes whose image count differs from the centre's or whose solve carries a
// status bit, plus one when the centre's own solve does (0: trustworthy).  One workgroup per epoch, nodes spread over its threads, each
// node solved in FP64 from the centre's roots; sums reduced in a fixed order.
constexpr int kDiskMaxX = 64;
constexpr int kDiskThreads = 256;

template <int N>
__global__ __launch_bounds__(kDiskThreads) void disk_mag_kernel(Batch b, int n_x, int n_phi,
                                                                int32_t* __restrict__ cn_changes,
                                                                const uint32_t* __restrict__ centre_status,
                                                                const double* __restrict__ roots,
                                                                double* __restrict__ mag) {
  constexpr int MI = N * N + 1;
  __shared__ double gl_x[kDiskMaxX], gl_w[kDiskMaxX];
  __shared__ double part_num[kDiskThreads / 64], part_den[kDiskThreads / 64];
  __shared__ int part_ch[kDiskThreads / 64];
  const int64_t e = blockIdx.x;
  if ((int)threadIdx.x < n_x) {
    // i-th Gauss-Legendre node on [-1, 1]: Newton on P_n from the usual cosine estimate;
    // P_n and P_{n-1} by the three-term recurrence, P_n' = n (x P_n - P_{n-1}) / (x^2 - 1)
    const int i = threadIdx.x;
    double x = cos(kPi * (i + 0.75) / (n_x + 0.5)), d = 1.0;
    for (int it = 0; it < 64; ++it) {
      double pm = 1.0, pc = x;
      for (int k = 2; k <= n_x; ++k) {
        const double pn = ((2 * k - 1) * x * pc - (k - 1) * pm) / k;
        pm = pc;
        pc = pn;
      }
      if (n_x == 1) {
        pc = x;
        pm = 1.0;
      }
      d = n_x * (x * pc - pm) / (x * x - 1.0);
      const double step = pc / d;
      x -= step;
      if (fabs(step) <= 1e-16) break;
    }
    gl_x[i] = x;
    gl_w[i] = 2.0 / ((1.0 - x * x) * d * d);
  }
  __syncthreads();
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = source_center(p, b.t[e]);
  const double rho = p[6], u1 = p[7];
  const int nc = cn_changes[e];
  c64 warm[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) warm[j] = mk(roots[(e * kMaxRoots + j) * 2], roots[(e * kMaxRoots + j) * 2 + 1]);
  double num = 0.0, den = 0.0;
  int ch = 0;
  for (int q = threadIdx.x; q < n_x * n_phi; q += kDiskThreads) {
    const int i = q / n_phi, j = q - (q / n_phi) * n_phi;
    const double xx = 0.25 * kPi * (gl_x[i] + 1.0);
    double sx, cx;
    sincos(xx, &sx, &cx);
    // weight: dx Jacobian pi/4, area element r dr = sin x cos x dx, linear limb darkening
    const double wr = gl_w[i] * 0.25 * kPi * sx * cx * ((1.0 - u1) + u1 * cx);
    double sp, cp;
    sincospi((2.0 * j + 1.0) / n_phi, &sp, &cp);
    const c64 w = mk(wc.x + rho * sx * cp, wc.y + rho * sx * sp);
    c64 img[MI];
    int n = 0;
    const uint32_t st = find_images<N, double>(L, w, img, n, kEAMaxIterFP64, warm);
    if (st != 0u || n != nc) ++ch;
    num += wr * point_mag<N>(L, img, n);
    den += wr;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    num += __shfl_xor(num, off);
    den += __shfl_xor(den, off);
    ch += __shfl_xor(ch, off);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    part_num[wave] = num;
    part_den[wave] = den;
    part_ch[wave] = ch;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tn = 0.0, td = 0.0;
    int tc = 0;
    for (int k = 0; k < kDiskThreads / 64; ++k) {
      tn += part_num[k];
      td += part_den[k];
      tc += part_ch[k];
    }
    mag[e] = tn / td;
    cn_changes[e] = tc + (centre_status[e] != 0u ? 1 : 0);
  }
}

}  // namespace

hipError_t launch_hybrid_select(int n_lens, int root_fp32, int n_check, double guard, double tol, double vary_max,
                                const Batch& b, const int32_t* cn, const double* a_c, const double* roots,
                                double* mag, uint32_t* status, int32_t* nsec, int32_t* ext_list, int32_t* ext_count,
                                hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  int P = 16;
  while (P < n_check) P <<= 1;
  if (P > 64) return hipErrorInvalidValue;
  const int bs = 256, G = bs / P;
  const dim3 g((unsigned)((b.n_epochs + G - 1) / G)), blk(bs);
#define ICRS_HYB(NN, TT)                                                                                          \
  hipLaunchKernelGGL((hybrid_select_kernel<NN, TT>), g, blk, 0, s, b, n_check, P, guard, tol, vary_max, cn, a_c, \
                     roots, mag, status, nsec, ext_list, ext_count)
  if (n_lens == 2) {
    if (root_fp32)
      ICRS_HYB(2, float);
    else
      ICRS_HYB(2, double);
  } else {
    if (root_fp32)
      ICRS_HYB(3, float);
    else
      ICRS_HYB(3, double);
  }
#undef ICRS_HYB
  return hipGetLastError();
}

hipError_t launch_point_jacobian(int n_lens, int root_fp32, const Batch& b, double* a_ps, double* jac,
                                 uint32_t* status_out, const uint32_t* status_in, uint32_t only_status,
                                 hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  const dim3 g(blocks_for(b.n_epochs, 64)), blk(64);
#define ICRS_PJ(NN, TT)                                                                                     \
  hipLaunchKernelGGL((point_jacobian_kernel<NN, TT>), g, blk, 0, s, b, a_ps, jac, status_out, status_in, \
                     only_status)
  if (n_lens == 2) {
    if (root_fp32)
      ICRS_PJ(2, float);
    else
      ICRS_PJ(2, double);
  } else {
    if (root_fp32)
      ICRS_PJ(3, float);
    else
      ICRS_PJ(3, double);
  }
#undef ICRS_PJ
  return hipGetLastError();
}

hipError_t launch_disk_mag(int n_lens, int n_x, int n_phi, const Batch& b, int32_t* cn_changes,
                           const uint32_t* centre_status, const double* roots, double* mag, hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  if (n_x < 1 || n_x > kDiskMaxX || n_phi < 1 || b.n_epochs > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)b.n_epochs), blk(kDiskThreads);
  if (n_lens == 2)
    hipLaunchKernelGGL((disk_mag_kernel<2>), g, blk, 0, s, b, n_x, n_phi, cn_changes, centre_status, roots, mag);
  else
    hipLaunchKernelGGL((disk_mag_kernel<3>), g, blk, 0, s, b, n_x, n_phi, cn_changes, centre_status, roots, mag);
  return hipGetLastError();
}

}  // namespace icrs
