// icrs_likelihood.hip -- marginalised light-curve likelihood (App. B, eq. NLL).
//
// Each event j is one data set: fluxes F_i = (A_i - 1) F_S + F_base with noise sigma_i, the
// design matrix M = [A - 1, 1] (n x 2), linear parameters beta = (F_S, F_base) with prior
// N(mu, Lambda), Lambda = diag(sigma_S^2, sigma_B^2).  With x_i = A_i - 1, w_i = 1/sigma_i^2
// and r_i = F_i - mu_S x_i - mu_B (the residual about the prior mean) the appendix's
// Woodbury forms reduce to sums over the event's epochs:
//   K = Lambda^{-1} + M^T C^{-1} M = [[1/sigma_S^2 + S_xx, S_x], [S_x, 1/sigma_B^2 + S_1]],
//   u = M^T C^{-1} r = (S_xr, S_1r),   r^T (C + M Lambda M^T)^{-1} r = S_rr - u^T K^{-1} u,
//   ln |C + M Lambda M^T| = sum_i ln sigma_i^2 + ln sigma_S^2 + ln sigma_B^2 + ln det K,
// with S_xx = sum w x^2, S_x = sum w x, S_1 = sum w, S_xr = sum w x r, S_1r = sum w r,
// S_rr = sum w r^2, and NLL = (S_rr - u^T K^{-1} u + ln |...|) / 2.  The posterior of beta
// is N(a, K^{-1}) with a = K^{-1} (Lambda^{-1} mu + M^T C^{-1} F) = mu + K^{-1} u.
// Differentiating in x_i (v = K^{-1} u; only S_xx, S_x, S_xr, S_1r, S_rr depend on x_i):
//   dNLL/dA_i = w_i [ -mu_S r_i - v_0 (r_i - mu_S x_i) + mu_S v_1 + v_0^2 x_i + v_0 v_1
//                     + (K^{-1})_00 x_i + (K^{-1})_01 ].
//
// nll_kernel: one workgroup per event; each thread sums a stride of the event's epochs, the
// six sums are reduced in a fixed order (wave butterflies, then waves in order), thread 0
// solves the 2 x 2 system, and every thread writes dNLL/dA of its epochs.
#include "icrs_launch.hpp"

namespace icrs {
namespace {

constexpr int kNllThreads = 256;
constexpr int kNllWaves = kNllThreads / 64;
constexpr int kSums = 7;  // S_xx, S_x, S_1, S_xr, S_1r, S_rr, sum ln sigma^2

__global__ __launch_bounds__(kNllThreads) void nll_kernel(const int64_t* __restrict__ offsets,
                                                          const double* __restrict__ mag,
                                                          const double* __restrict__ flux,
                                                          const double* __restrict__ sigma,
                                                          const double* __restrict__ prior, double* __restrict__ nll,
                                                          double* __restrict__ beta, double* __restrict__ dnll) {
  __shared__ double part[kNllWaves][kSums];
  __shared__ double sol[6];  // v0, v1, Kinv00, Kinv01, Kinv11, (unused)
  const int64_t ev = blockIdx.x;
  const int64_t e0 = offsets[ev], e1 = offsets[ev + 1];
  const double muS = prior[ev * 4 + 0], muB = prior[ev * 4 + 1];
  const double sS = prior[ev * 4 + 2], sB = prior[ev * 4 + 3];
  double acc[kSums];
#pragma unroll
  for (int k = 0; k < kSums; ++k) acc[k] = 0.0;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kNllThreads) {
    const double x = mag[i] - 1.0;
    const double s2 = sigma[i] * sigma[i];
    const double w = 1.0 / s2;
    const double r = flux[i] - muS * x - muB;
    acc[0] += w * x * x;
    acc[1] += w * x;
    acc[2] += w;
    acc[3] += w * x * r;
    acc[4] += w * r;
    acc[5] += w * r * r;
    acc[6] += log(s2);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kSums; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) part[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S[kSums];
    for (int k = 0; k < kSums; ++k) {
      S[k] = 0.0;
      for (int q = 0; q < kNllWaves; ++q) S[k] += part[q][k];
    }
    const double lS = sS * sS, lB = sB * sB;
    const double k00 = 1.0 / lS + S[0], k01 = S[1], k11 = 1.0 / lB + S[2];
    const double det = k00 * k11 - k01 * k01;
    const double i00 = k11 / det, i01 = -k01 / det, i11 = k00 / det;
    const double u0 = S[3], u1 = S[4];
    const double v0 = i00 * u0 + i01 * u1, v1 = i01 * u0 + i11 * u1;
    const double quad = S[5] - (u0 * v0 + u1 * v1);
    const double logdet = S[6] + log(lS) + log(lB) + log(det);
    nll[ev] = 0.5 * (quad + logdet);
    if (beta) {
      beta[ev * 5 + 0] = muS + v0;
      beta[ev * 5 + 1] = muB + v1;
      beta[ev * 5 + 2] = i00;
      beta[ev * 5 + 3] = i01;
      beta[ev * 5 + 4] = i11;
    }
    sol[0] = v0;
    sol[1] = v1;
    sol[2] = i00;
    sol[3] = i01;
    sol[4] = i11;
  }
  __syncthreads();
  if (!dnll) return;
  const double v0 = sol[0], v1 = sol[1], i00 = sol[2], i01 = sol[3];
  for (int64_t i = e0 + threadIdx.x; i < e1; i += kNllThreads) {
    const double x = mag[i] - 1.0;
    const double w = 1.0 / (sigma[i] * sigma[i]);
    const double r = flux[i] - muS * x - muB;
    dnll[i] = w * (-muS * r - v0 * (r - muS * x) + muS * v1 + v0 * v0 * x + v0 * v1 + i00 * x + i01);
  }
}

}  // namespace

hipError_t launch_nll(int64_t n_events, const int64_t* offsets, const double* mag, const double* flux,
                      const double* sigma, const double* prior, double* nll, double* beta, double* dnll,
                      hipStream_t s) {
  if (n_events == 0) return hipSuccess;
  if (n_events > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nll_kernel, dim3((unsigned)n_events), dim3(kNllThreads), 0, s, offsets, mag, flux, sigma, prior,
                     nll, beta, dnll);
  return hipGetLastError();
}

}  // namespace icrs
