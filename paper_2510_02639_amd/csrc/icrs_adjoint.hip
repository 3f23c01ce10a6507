// icrs_adjoint.hip -- derivatives of the ICRS magnification on a frozen structure.
//
// The sector boxes, the inside/outside pattern chi, every crossing's stencil and every
// edge factor's branch are those of the primal evaluation (the rays are recomputed here with
// the same arithmetic, so the decisions repeat exactly); with them fixed the magnification
// A = (1/rho^2) sum_sectors dr dtheta sum_rows r_i sum_l chi_l I(d_l) W_l  (App. A) is a
// smooth function of the event parameters.  Per node the kernel forms the partials of d^2
// over the generalised coordinates (eps_k, a_k, w_c); a crossing's position t solves
// L(t) = rho on its stencil, so dt = (drho - sum_j l_j(t) dd_j) / L'(t).  The per-epoch
// partials are chained to (s, q, u0, alpha, t0, tE, rho, u_ld, q3, r3, psi) and contracted
// with the cotangent per event.
//
// One persistent workgroup (4 wave64s) per epoch at a time; lane l owns columns l + 64 j;
// column cos/sin in LDS, one row buffer of d^2 per wave.  FP64 throughout.
#include "icrs_device.hpp"
#include "icrs_launch.hpp"
#include "icrs_quad.hpp"

namespace icrs {

namespace {

constexpr int kAW = 4;
constexpr int kAdjMaxTheta = 1024;

// d^2 = |w(z) - w_c|^2 at the node (x, y) and its partials over g = (eps_0..eps_{N-1},
// a_0.x..a_{N-1}.x, a_0.y..a_{N-1}.y, w_c.x, w_c.y).  With v_k = 1/conj(z - a_k):
// dD/deps_k = -v_k, dD/da_k.x = -eps_k v_k^2, dD/da_k.y = i eps_k v_k^2, dD/dw_c = -1, -i,
// and d(d^2) = 2 Re(conj(D) dD) for D = w - w_c.
template <int N>
__device__ inline double node_d2_grad(const Lens<N>& L, c64 wc, double x, double y, double (&g)[3 * N + 2]) {
  double Dx = x - wc.x, Dy = y - wc.y;
  double vx[N], vy[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double dx = x - L.a[k].x, dy = y - L.a[k].y;
    const double inv = rcp_fast(fma(dx, dx, dy * dy));
    vx[k] = dx * inv;
    vy[k] = dy * inv;
    Dx = fma(-L.eps[k], vx[k], Dx);
    Dy = fma(-L.eps[k], vy[k], Dy);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double sqx = vx[k] * vx[k] - vy[k] * vy[k], sqy = 2.0 * vx[k] * vy[k];
    g[k] = -2.0 * fma(Dx, vx[k], Dy * vy[k]);
    g[N + k] = -2.0 * L.eps[k] * fma(Dx, sqx, Dy * sqy);
    g[2 * N + k] = 2.0 * L.eps[k] * fma(-Dx, sqy, Dy * sqx);
  }
  g[3 * N] = -2.0 * Dx;
  g[3 * N + 1] = -2.0 * Dy;
  return fma(Dx, Dx, Dy * Dy);
}

// Brightness I(d^2) and its partials in d^2, rho (at fixed d) and u1.
struct Bright {
  double I, dI_dd2, dI_drho, dI_du1;
};
// The epoch's constants of I: I0 = 3 / (pi (3 - u1)), 1/rho^2, 2/rho^3 and dI0/du1 = I0 / (3 - u1),
// so that no node divides.
struct BrightConst {
  double u1, I0, inv_rho2, two_inv_rho3, dI0_du1;
  __device__ inline BrightConst(double rho, double u1_) : u1(u1_) {
    I0 = 3.0 / (kPi * (3.0 - u1));
    inv_rho2 = 1.0 / (rho * rho);
    two_inv_rho3 = 2.0 * inv_rho2 / rho;
    dI0_du1 = I0 / (3.0 - u1);
  }
};
__device__ inline Bright bright_grad(double d2, const BrightConst& k) {
  const double c = fmax(1.0 - d2 * k.inv_rho2, 0.0);
  const double s = sqrt_fast(c);
  Bright b;
  b.I = k.I0 * (1.0 - k.u1 + k.u1 * s);
  const double ds_dc = (s > 0.0) ? 0.5 * rcp_fast(s) : 0.0;  // refined reciprocal, ~1e-15 relative
  b.dI_dd2 = k.I0 * k.u1 * ds_dc * (-k.inv_rho2);
  b.dI_drho = k.I0 * k.u1 * ds_dc * (d2 * k.two_inv_rho3);
  b.dI_du1 = k.dI0_du1 * (1.0 - k.u1 + k.u1 * s) + k.I0 * (s - 1.0);
  return b;
}

// Three waves per SIMD: the compiler's own choice, 256 VGPRs and one or two waves, runs the
// VJP 1.6x slower despite the spills this costs; four waves spill too much.
template <int N, int JMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void adjoint_kernel(
    Batch b, SectorBuf sec, int n_r, int n_theta, double delta_c, double* __restrict__ jac, double* __restrict__ mag_out,
    unsigned long long* __restrict__ queue) {
  constexpr int NG = 3 * N + 2;
  constexpr int NA = NG + 3;  // g partials, flux, rho, u1
  __shared__ double colc[JMAX * 64], cols[JMAX * 64];  // the launch picks JMAX with n_theta <= 64 JMAX
  __shared__ double rowbuf[kAW][JMAX * 64];
  __shared__ double red[kAW][NA];
  __shared__ unsigned long long next_sh;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (as in the ray kernel)
  const int J = (n_theta + 63) >> 6;
  const int last = n_theta - 1;
  double* buf = rowbuf[wave];

  for (;;) {
    if (threadIdx.x == 0) next_sh = atomicAdd(queue, 1ull);
    __syncthreads();
    const unsigned long long idx = next_sh;
    __syncthreads();
    if (idx >= (unsigned long long)b.n_epochs) break;
    const int64_t e = (int64_t)idx;
    const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
    const Lens<N> L = make_lens<N>(p);
    const c64 wc = source_center(p, b.t[e]);
    const double rho = p[6], u1 = p[7];
    const double rho2 = rho * rho;
    const double f_edge = edge_factor<double>(0.5, u1, delta_c) - 1.0;
    const BrightConst bk(rho, u1);
    double tot[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) tot[a] = 0.0;

    // a sector count outside 0..kMaxSectors (only from a caller's given list) is not used:
    // the epoch's derivatives and magnification become NaN
    const int ns_in = sec.nsec[e];
    const bool bad_ns = ns_in < 0 || ns_in > kMaxSectors;
    const int ns = bad_ns ? 0 : ns_in;
    for (int slot = 0; slot < ns; ++slot) {
      const double* sp = sec.sectors + (e * kMaxSectors + slot) * 4;
      const bool per = sec.periodic[e * kMaxSectors + slot] != 0;
      const double r_lo = sp[0], r_hi = sp[1], th_lo = sp[2];
      const double dr = (r_hi - r_lo) / n_r, dth = (sp[3] - th_lo) / n_theta;
      for (int l = threadIdx.x; l < n_theta; l += blockDim.x) sincos(th_lo + (l + 0.5) * dth, &cols[l], &colc[l]);
      __syncthreads();

      double acc[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) acc[a] = 0.0;
      for (int i = wave; i < n_r; i += kAW) {
        const double r = r_lo + (i + 0.5) * dr;
        // chunk culling as in the forward kernel: lane j tests chunk j's arc, widened by two
        // columns on each side; one that provably maps farther than rho (1 + 1e-3) from the
        // source centre has no inside node and no stencil node of a crossing (changes no bit)
        bool sk = false;
        if (lane < J) {
          double cs, sn;
          sincos(th_lo + (64.0 * lane + 32.0) * dth, &sn, &cs);
          sk = arc_distance_lower_bound<N>(L, wc, r, cs, sn, 34.0 * dth) > rho * 1.001;
        }
        const uint64_t rowskip = __ballot(sk);
        if (rowskip == (1ull << J) - 1ull) continue;  // the whole row misses the image
        uint64_t m[JMAX];
        uint64_t any = 0;
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
          m[j] = 0;
          if (j >= J || ((rowskip >> j) & 1ull)) continue;
          const int l = lane + 64 * j;
          const bool valid = l < n_theta;
          const int lc = valid ? l : last;
          double gg[NG];
          const double d2 = node_d2_grad<N>(L, wc, r * colc[lc], r * cols[lc], gg);
          const bool in = valid && d2 < rho2;
          m[j] = __ballot(in);
          any |= m[j];
          if (valid) buf[l] = d2;
          if (in) {
            const Bright br = bright_grad(d2, bk);
#pragma unroll
            for (int g = 0; g < NG; ++g) acc[g] = fma(r * br.dI_dd2, gg[g], acc[g]);
            acc[NG] = fma(r, br.I, acc[NG]);
            acc[NG + 1] = fma(r, br.dI_drho, acc[NG + 1]);
            acc[NG + 2] = fma(r, br.dI_du1, acc[NG + 2]);
          }
        }
        if (any == 0) continue;
        uint64_t m_last = 0;
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
          if (j == (last >> 6)) m_last = m[j];
        const uint64_t in_last = (m_last >> (last & 63)) & 1ull;
        // boundary words (as in the forward kernel), items = (node, side)
        int n_left = 0, n_all = 0;
        uint64_t wl[JMAX], wr[JMAX];
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
          wl[j] = wr[j] = 0;
          if (j >= J) continue;
          const uint64_t carry = (j > 0) ? (m[j > 0 ? j - 1 : 0] >> 63) : (per ? in_last : 0ull);
          wl[j] = m[j] & ~((m[j] << 1) | carry);
          uint64_t right = (m[j] >> 1) | ((j + 1 < J) ? (m[j + 1 < JMAX ? j + 1 : j] << 63) : 0ull);
          if (j == (last >> 6) && per) right |= (m[0] & 1ull) << (last & 63);
          wr[j] = m[j] & ~right;
          n_left += __popcll(wl[j]);
          n_all += __popcll(wr[j]);
        }
        n_all += n_left;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int base = 0; base < n_all; base += 64) {
          const int k = base + lane;
          if (k >= n_all) continue;
          const int side = k >= n_left ? 1 : 0;
          int rem = side ? k - n_left : k;
          int l = 0;
#pragma unroll
          for (int j = 0; j < JMAX; ++j) {
            if (j >= J) continue;
            uint64_t w = side ? wr[j] : wl[j];
            const int pc = __popcll(w);
            if (rem >= 0 && rem < pc) {
              for (int q = 0; q < rem && q < 64; ++q) w &= w - 1ull;
              l = 64 * j + __ffsll((unsigned long long)w) - 1;
            }
            rem -= pc;
          }
          double gl[NG];
          const double d2l = node_d2_grad<N>(L, wc, r * colc[l], r * cols[l], gl);
          const Bright br = bright_grad(d2l, bk);
          double corr;
          const bool edge = (side == 0 && l == 0 && !per) || (side == 1 && l == last && !per);
          if (edge) {
            corr = f_edge;
          } else {
            const int pp = side ? l : (l == 0 ? last : l - 1);
            const bool cubic = per || (pp - 1 >= 0 && pp + 2 <= last);
            int ix[4];
            ix[0] = per ? (pp - 1 + n_theta) % n_theta : max(pp - 1, 0);
            ix[1] = pp;
            ix[2] = (pp + 1) % n_theta;
            ix[3] = per ? (pp + 2) % n_theta : min(pp + 2, last);
            double dv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) dv[q] = sqrt(buf[ix[q]]);
            const double t = crossing_t<double>(dv[0], dv[1], dv[2], dv[3], cubic, rho);
            const double delta = side ? t : 1.0 - t;
            corr = edge_factor<double>(delta, u1, delta_c) - 1.0;
            double lb[4];
            const double Lp = crossing_basis<double>(dv[0], dv[1], dv[2], dv[3], cubic, t, lb);
            // d(I_l (f(delta) - 1)) through delta = +-t
            const double K = r * br.I * edge_factor_slope<double>(delta, u1, delta_c) * (side ? 1.0 : -1.0) / Lp;
            acc[NG + 1] += K;  // dt/drho = 1/L'
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (lb[q] == 0.0) continue;
              double gq[NG];
              node_d2_grad<N>(L, wc, r * colc[ix[q]], r * cols[ix[q]], gq);
              const double c = -K * lb[q] / (2.0 * dv[q]);  // dd_q = d(d_q^2) / (2 d_q)
#pragma unroll
              for (int g = 0; g < NG; ++g) acc[g] = fma(c, gq[g], acc[g]);
            }
          }
#pragma unroll
          for (int g = 0; g < NG; ++g) acc[g] = fma(r * br.dI_dd2 * corr, gl[g], acc[g]);
          acc[NG] = fma(r * corr, br.I, acc[NG]);
          acc[NG + 1] = fma(r * corr, br.dI_drho, acc[NG + 1]);
          acc[NG + 2] = fma(r * corr, br.dI_du1, acc[NG + 2]);
        }
        __builtin_amdgcn_wave_barrier();
      }
      // deterministic reduction of the sector's sums
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        double v = acc[a];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][a] = v;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const double S = dr * dth;
        for (int a = 0; a < NA; ++a) {
          double v = 0.0;
          for (int q = 0; q < kAW; ++q) v += red[q][a];
          tot[a] += S * v;
        }
      }
      __syncthreads();
    }

    if (threadIdx.x == 0) {
      // A = F / rho^2; chain the generalised coordinates to the event parameters
      const double inv_rho2 = 1.0 / rho2;
      const double A = tot[NG] * inv_rho2;
      double dg[NG];
      for (int g = 0; g < NG; ++g) dg[g] = tot[g] * inv_rho2;
      const double s = p[0], q = p[1];
      const double q3 = (N == 3) ? p[8] : 0.0;
      const double pair = 1.0 + q, m = pair + q3;
      double out[kParams];
      for (int k = 0; k < kParams; ++k) out[k] = 0.0;
      // eps_0 = 1/m, eps_1 = q/m, eps_2 = q3/m
      const double de_dq[3] = {-1.0 / (m * m), (1.0 + q3) / (m * m), -q3 / (m * m)};
      const double de_dq3[3] = {-1.0 / (m * m), -q / (m * m), pair / (m * m)};
      // a_0.x = -q s/(1+q), a_1.x = s/(1+q), a_2.x = s(1-q)/(2(1+q)) + r3 cos psi
      const double dax_ds[3] = {-q / pair, 1.0 / pair, (1.0 - q) / (2.0 * pair)};
      const double dax_dq[3] = {-s / (pair * pair), -s / (pair * pair), -s / (pair * pair)};
      for (int k = 0; k < N; ++k) {
        out[0] += dg[N + k] * dax_ds[k];
        out[1] += dg[k] * de_dq[k] + dg[N + k] * dax_dq[k];
        if (N == 3) out[8] += dg[k] * de_dq3[k];
      }
      if constexpr (N == 3) {
        double sp3, cp3;
        sincos(p[10], &sp3, &cp3);
        out[9] = dg[N + 2] * cp3 + dg[2 * N + 2] * sp3;
        out[10] = p[9] * (-dg[N + 2] * sp3 + dg[2 * N + 2] * cp3);
      }
      double sa, ca;
      sincos(p[3], &sa, &ca);
      const double gx = dg[3 * N], gy = dg[3 * N + 1];
      const double tau = (b.t[e] - p[4]) / p[5];
      out[2] = -gx * sa + gy * ca;                 // u0
      out[3] = -gx * wc.y + gy * wc.x;             // alpha
      out[4] = -(gx * ca + gy * sa) / p[5];        // t0
      out[5] = -(gx * ca + gy * sa) * tau / p[5];  // tE
      out[6] = tot[NG + 1] * inv_rho2 - 2.0 * A / rho;
      out[7] = tot[NG + 2] * inv_rho2;
      const double nan = __builtin_nan("");
      for (int k = 0; k < kParams; ++k) jac[e * kParams + k] = bad_ns ? nan : out[k];
      if (mag_out) mag_out[e] = bad_ns ? nan : A;
    }
    __syncthreads();
  }
}

// grad[ev][k] = sum over the event's epochs of cot[e] jac[e][k] (fixed order)
__global__ void contract_kernel(Batch b, const double* __restrict__ jac, const double* __restrict__ cot,
                                double* __restrict__ grad) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= b.n_events * kParams) return;
  const int64_t ev = idx / kParams;
  const int k = (int)(idx % kParams);
  double s = 0.0;
  for (int64_t e = b.offsets[ev]; e < b.offsets[ev + 1]; ++e) s = fma(cot[e], jac[e * kParams + k], s);
  grad[idx] = s;
}

template <int N, int JMAX>
hipError_t launch_adjoint_j(const Batch& b, const SectorBuf& sec, int n_r, int n_theta, double delta_c, double* jac,
                            double* mag, unsigned long long* queue, hipStream_t s) {
  auto kern = adjoint_kernel<N, JMAX>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kAW * 64, 0);
  if (e != hipSuccess) return e;
  int64_t grid = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  if (b.n_epochs < grid) grid = b.n_epochs;
  e = launch_fill_i32((int32_t*)queue, 2, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kAW * 64), 0, s, b, sec, n_r, n_theta, delta_c, jac, mag, queue);
  return hipGetLastError();
}

template <int N>
hipError_t launch_adjoint_n(const Batch& b, const SectorBuf& sec, int n_r, int n_theta, double delta_c, double* jac,
                            double* mag, unsigned long long* queue, hipStream_t s) {
  const int J = (n_theta + 63) / 64;
  if (J <= 4) return launch_adjoint_j<N, 4>(b, sec, n_r, n_theta, delta_c, jac, mag, queue, s);
  if (J <= 8) return launch_adjoint_j<N, 8>(b, sec, n_r, n_theta, delta_c, jac, mag, queue, s);
  return launch_adjoint_j<N, 16>(b, sec, n_r, n_theta, delta_c, jac, mag, queue, s);
}

}  // namespace

hipError_t launch_adjoint(int n_lens, const Batch& b, const SectorBuf& sec, int n_r, int n_theta, double delta_c,
                          const double* cot, double* jac, double* grad, double* mag, unsigned long long* queue,
                          hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  if (n_theta > kAdjMaxTheta) return hipErrorInvalidValue;
  hipError_t e = (n_lens == 2) ? launch_adjoint_n<2>(b, sec, n_r, n_theta, delta_c, jac, mag, queue, s)
                               : launch_adjoint_n<3>(b, sec, n_r, n_theta, delta_c, jac, mag, queue, s);
  if (e != hipSuccess || !cot || !grad) return e;
  return launch_contract(b, jac, cot, grad, s);
}

hipError_t launch_contract(const Batch& b, const double* jac, const double* cot, double* grad, hipStream_t s) {
  const int64_t n = b.n_events * kParams;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(contract_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, jac, cot, grad);
  return hipGetLastError();
}

}  // namespace icrs
