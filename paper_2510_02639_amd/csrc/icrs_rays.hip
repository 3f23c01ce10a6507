// icrs_rays.hip -- inverse ray shooting and row quadrature (Sec. 3.3, App. A).
//
// One workgroup (4 wave64s) per (epoch, sector).  The sector's N_r x N_theta polar grid is
// never stored: each wave owns every 4th row; lane l owns the columns l, l+64, l+128, ...
// whose cos/sin stay in registers for the whole sector.  For one row a lane maps its nodes
// through the lens equation, the wave takes ballots of chi = [d < rho] (one 64-bit mask per
// 64 columns), and only lanes holding a boundary node read their neighbours' distances back
// from a per-wave LDS row buffer to place the crossing on the cubic interpolant.  Row sums
// stay in registers; each workgroup writes one partial flux per (epoch, sector).
#include "icrs_device.hpp"
#include "icrs_launch.hpp"

namespace icrs {

namespace {

constexpr int kWaves = 4;

template <typename T>
struct Num;
template <>
struct Num<double> {
  static constexpr double newton_tol = 1e-15;
};
template <>
struct Num<float> {
  static constexpr float newton_tol = 1e-7f;
};

// f(delta) of App. A.2 (u1 > 0) or delta + 1/2 (uniform source, App. A.1)
template <typename T>
__device__ __forceinline__ T edge_factor(T delta, T u1, T delta_c) {
  if (u1 == T(0)) return delta + T(0.5);
  if (delta >= delta_c && delta > T(0)) return (T(0.5) + delta) * T(2.0 / 3.0) * sqrt(T(1) + T(1) / (T(2) * delta));
  return T(2.0 / 3.0) * delta + T(0.5);
}

// Crossing of the cubic Lagrange interpolant through (t, d) = (-1,d0), (0,d1), (1,d2),
// (2,d3) with rho on the bracket [0,1] (d1, d2 on opposite sides of rho); linear between
// d1 and d2 when cubic is false.  Safeguarded Newton from the linear estimate: the bracket
// shrinks on every step and a step leaving it is replaced by bisection.
template <typename T>
__device__ inline T crossing_t(T d0, T d1, T d2, T d3, bool cubic, T rho) {
  const T den = d2 - d1;
  T t = (den == T(0)) ? T(0.5) : (rho - d1) / den;
  t = fmin(fmax(t, T(0)), T(1));
  if (!cubic) return t;
  const T c0 = d1;
  const T c1 = -d0 * T(1.0 / 3.0) - T(0.5) * d1 + d2 - d3 * T(1.0 / 6.0);
  const T c2 = T(0.5) * d0 - d1 + T(0.5) * d2;
  const T c3 = (d3 - d0) * T(1.0 / 6.0) + T(0.5) * (d1 - d2);
  const bool in0 = (d1 - rho) < T(0);
  T a = T(0), b = T(1);
  for (int it = 0; it < 16; ++it) {
    const T g = ((c3 * t + c2) * t + c1) * t + c0 - rho;
    if (g == T(0)) break;
    if ((g < T(0)) == in0)
      a = t;
    else
      b = t;
    const T dg = (T(3) * c3 * t + T(2) * c2) * t + c1;
    T tn = t - g / dg;
    if (!(tn > a && tn < b)) tn = T(0.5) * (a + b);
    const bool done = fabs(tn - t) <= Num<T>::newton_tol;
    t = tn;
    if (done) break;
  }
  return t;
}

__device__ __forceinline__ int bit_of(uint64_t m, int b) { return (int)((m >> b) & 1ull); }

// Node maps.  MapF64 evaluates eq. lens_eq directly in FP64.  MapF32 works relative to an
// FP64 anchor z_a = r_i e^{i theta_a} on each row: with dz = z - z_a = r_i e^{i theta_a}
// (e^{i dtheta_l} - 1), u_k = z - a_k and h_k = eps_k / (z_a - a_k),
//   w - w_c = (w(z_a) - w_c) + dz + sum_k conj(dz h_k / u_k),
// an identity with no cancellation, so FP32 rounding scales with |dz| instead of |z|.
template <int N, int JMAX>
struct MapF64 {
  using T = double;
  double cs[JMAX], sn[JMAX];
  Lens<N> L;
  c64 wc;
  double r;
  __device__ void init_sector(const Lens<N>& lens, c64 w_c, double th_lo, double dth, double th_a, int lane) {
    L = lens;
    wc = w_c;
    (void)th_a;
#pragma unroll
    for (int j = 0; j < JMAX; ++j) sincos(th_lo + (lane + 64 * j + 0.5) * dth, &sn[j], &cs[j]);
  }
  __device__ void init_row(double r_i) { r = r_i; }
  __device__ __forceinline__ double d2(int j) const {
    const double x = r * cs[j], y = r * sn[j];
    double wx = x - wc.x, wy = y - wc.y;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double dx = x - L.a[k].x, dy = y - L.a[k].y;
      const double inv = L.eps[k] / (dx * dx + dy * dy);
      wx -= inv * dx;
      wy -= inv * dy;
    }
    return wx * wx + wy * wy;
  }
};

template <int N, int JMAX>
struct MapF32 {
  using T = float;
  float gx[JMAX], gy[JMAX];  // e^{i theta_a} (e^{i dtheta_l} - 1) per owned column
  Lens<N> L;
  c64 wc;
  double ca, sa;             // e^{i theta_a}
  float r, bx, by;           // row: r_i, w(z_a) - w_c
  float ax[N], ay[N], hx[N], hy[N];
  __device__ void init_sector(const Lens<N>& lens, c64 w_c, double th_lo, double dth, double th_a, int lane) {
    L = lens;
    wc = w_c;
    sincos(th_a, &sa, &ca);
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const double dt = th_lo + (lane + 64 * j + 0.5) * dth - th_a;
      double sd, cd;
      sincos(dt, &sd, &cd);
      const double sh = sin(0.5 * dt);
      const double ex = -2.0 * sh * sh, ey = sd;  // e^{i dt} - 1 without cancellation
      gx[j] = (float)(ca * ex - sa * ey);
      gy[j] = (float)(ca * ey + sa * ex);
    }
  }
  __device__ void init_row(double r_i) {
    const c64 za = mk(r_i * ca, r_i * sa);
    c64 w = za;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const c64 d = za - L.a[k];
      const double n = norm2(d);
      w = w - mk(L.eps[k] * d.x / n, L.eps[k] * d.y / n);
      ax[k] = (float)d.x;
      ay[k] = (float)d.y;
      const double s = L.eps[k] / n;  // eps/d = eps conj(d)/|d|^2
      hx[k] = (float)(s * d.x);
      hy[k] = (float)(-s * d.y);
    }
    r = (float)r_i;
    bx = (float)(w.x - wc.x);
    by = (float)(w.y - wc.y);
  }
  __device__ __forceinline__ float d2(int j) const {
    const float dzx = r * gx[j], dzy = r * gy[j];
    float Dx = bx + dzx, Dy = by + dzy;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const float ux = ax[k] + dzx, uy = ay[k] + dzy;
      const float inv = __builtin_amdgcn_rcpf(ux * ux + uy * uy);
      const float px = dzx * hx[k] - dzy * hy[k];
      const float py = dzx * hy[k] + dzy * hx[k];
      const float qx = px * ux + py * uy;  // p conj(u)
      const float qy = py * ux - px * uy;
      Dx += qx * inv;
      Dy -= qy * inv;
    }
    return Dx * Dx + Dy * Dy;
  }
};

template <int N, int JMAX, typename MAP>
__global__ __launch_bounds__(256) void rays_kernel(Batch b, SectorBuf sec, RayWork w, int n_r, int n_theta,
                                                   double delta_c_d, double* __restrict__ partial,
                                                   uint8_t* __restrict__ clip_out) {
  using T = typename MAP::T;
  __shared__ T rowbuf[kWaves][JMAX * 64];
  __shared__ double wsum[kWaves];
  __shared__ int wclip[kWaves];

  const int slot = blockIdx.x % kMaxSectors;
  const int64_t widx = blockIdx.x / kMaxSectors;
  const int64_t e = w.list ? (int64_t)w.list[widx] : widx;
  if (slot >= sec.nsec[e]) return;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const double* sp = sec.sectors + (e * kMaxSectors + slot) * 4;
  const double r_lo = sp[0], r_hi = sp[1], th_lo = sp[2], th_hi = sp[3];
  const bool per = sec.periodic[e * kMaxSectors + slot] != 0;
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const double rho_d = p[6], u1_d = p[7];
  const T rho = (T)rho_d, u1 = (T)u1_d, delta_c = (T)delta_c_d;
  const T rho2 = (T)(rho_d * rho_d), inv_rho2 = (T)(1.0 / (rho_d * rho_d));
  const T I0 = (T)(3.0 / (kPi * (3.0 - u1_d)));
  const int J = (n_theta + 63) >> 6;
  const double dr = (r_hi - r_lo) / n_r;
  const double dth = (th_hi - th_lo) / n_theta;
  const T f_edge = edge_factor<T>(T(0.5), u1, delta_c) - T(1);  // neighbour beyond a sector edge
  const int last = n_theta - 1;

  MAP map;
  map.init_sector(make_lens<N>(p), source_center(p, b.t[e]), th_lo, dth, 0.5 * (th_lo + th_hi), lane);

  double acc = 0.0;
  int clip = 0;
  T* buf = rowbuf[wave];

  for (int i = wave; i < n_r; i += kWaves) {
    const double r = r_lo + (i + 0.5) * dr;
    map.init_row(r);
    T d2[JMAX];
    uint64_t m[JMAX];
    uint64_t any = 0;
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      m[j] = 0;
      d2[j] = T(0);
      if (j < J) {
        const int l = lane + 64 * j;
        d2[j] = (l < n_theta) ? map.d2(j) : T(__builtin_inf());
        m[j] = __ballot(d2[j] < rho2);
        any |= m[j];
      }
    }
    if (any == 0) continue;  // wave-uniform
    if (i == 0 && r_lo > 0.0) clip |= 1;
    if (i == n_r - 1) clip |= 2;
    uint64_t m_last = 0;
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
      if (j == (last >> 6)) m_last = m[j];
    const int in_last = bit_of(m_last, last & 63);
    if (!per) {
      if (m[0] & 1ull) clip |= 4;
      if (in_last) clip |= 8;
    }
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      const int l = lane + 64 * j;
      if (j < J && l < n_theta) buf[l] = d2[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    T row = T(0);
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      if (j >= J) continue;
      const int l = lane + 64 * j;
      if (!bit_of(m[j], lane)) continue;
      // neighbour flags: -1 beyond a non-periodic edge, else inside (1) / outside (0)
      int lin, rin;
      if (l >= 1)
        lin = lane ? bit_of(m[j], lane - 1) : bit_of(m[j > 0 ? j - 1 : 0], 63);
      else
        lin = per ? in_last : -1;
      if (l + 1 < n_theta)
        rin = (lane < 63) ? bit_of(m[j], lane + 1) : (int)(m[j + 1 < JMAX ? j + 1 : j] & 1ull);
      else
        rin = per ? (int)(m[0] & 1ull) : -1;
      T W = T(1);
      if (lin < 0) {
        W += f_edge;
      } else if (lin == 0) {  // crossing in (theta_{l-1}, theta_l): bracket p = l-1
        const int pp = l - 1 < 0 ? last : l - 1;
        const bool cubic = per || (l - 2 >= 0 && l + 1 <= last);
        const int im1 = per ? (pp - 1 + n_theta) % n_theta : max(pp - 1, 0);
        const int ip2 = per ? (pp + 2) % n_theta : min(pp + 2, last);
        const int ip1 = (pp + 1) % n_theta;
        const T t = crossing_t<T>(sqrt(buf[im1]), sqrt(buf[pp]), sqrt(buf[ip1]), sqrt(buf[ip2]), cubic, rho);
        W += edge_factor<T>(T(1) - t, u1, delta_c) - T(1);
      }
      if (rin < 0) {
        W += f_edge;
      } else if (rin == 0) {  // crossing in (theta_l, theta_{l+1}): bracket p = l
        const int pp = l;
        const bool cubic = per || (l - 1 >= 0 && l + 2 <= last);
        const int im1 = per ? (pp - 1 + n_theta) % n_theta : max(pp - 1, 0);
        const int ip2 = per ? (pp + 2) % n_theta : min(pp + 2, last);
        const int ip1 = (pp + 1) % n_theta;
        const T t = crossing_t<T>(sqrt(buf[im1]), sqrt(buf[pp]), sqrt(buf[ip1]), sqrt(buf[ip2]), cubic, rho);
        W += edge_factor<T>(t, u1, delta_c) - T(1);
      }
      const T c = fmax(T(1) - d2[j] * inv_rho2, T(0));
      const T I = I0 * (T(1) - u1 * (T(1) - sqrt(c)));
      row += I * W;
    }
    acc += r * (double)row;
    __builtin_amdgcn_wave_barrier();
  }

  // deterministic reductions: butterfly inside the wave, then waves in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    wsum[wave] = acc;
    wclip[wave] = clip;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    int c = 0;
    for (int q = 0; q < kWaves; ++q) {
      tot += wsum[q];
      c |= wclip[q];
    }
    partial[e * kMaxSectors + slot] = tot * dr * dth;
    clip_out[e * kMaxSectors + slot] = (uint8_t)c;
  }
}

__global__ void finalize_kernel(Batch b, SectorBuf sec, RayWork w, const double* __restrict__ partial,
                                const uint8_t* __restrict__ clip, int attempt, int max_retries,
                                int32_t* __restrict__ next_list, int32_t* __restrict__ next_count,
                                double* __restrict__ mag, uint32_t* __restrict__ status, uint32_t extra_status) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= w.n) return;
  const int64_t e = w.list ? (int64_t)w.list[idx] : idx;
  const int ns = sec.nsec[e];
  double flux = 0.0;
  int clips[kMaxSectors];
  int any = 0;
  for (int s = 0; s < ns; ++s) {
    flux += partial[e * kMaxSectors + s];
    clips[s] = clip[e * kMaxSectors + s];
    any |= clips[s];
  }
  if (any && attempt < max_retries) {
    // widen the touched sides, merge, sort, and queue the epoch for another pass
    Sector S[kMaxSectors];
    int n = ns;
    for (int s = 0; s < ns; ++s) {
      const double* g = sec.sectors + (e * kMaxSectors + s) * 4;
      S[s] = Sector{g[0], g[1], g[2], g[3], (int)sec.periodic[e * kMaxSectors + s]};
      if (clips[s]) widen_sector(S[s], clips[s]);
    }
    merge_to_fixpoint(S, n);
    sort_sectors(S, n);
    for (int s = 0; s < n; ++s) {
      double* g = sec.sectors + (e * kMaxSectors + s) * 4;
      g[0] = S[s].r_lo;
      g[1] = S[s].r_hi;
      g[2] = S[s].th_lo;
      g[3] = S[s].th_hi;
      sec.periodic[e * kMaxSectors + s] = (uint8_t)S[s].periodic;
    }
    sec.nsec[e] = n;
    const int pos = atomicAdd(next_count, 1);
    next_list[pos] = (int32_t)e;
    return;
  }
  const double rho = b.params[(int64_t)b.epoch_event[e] * kParams + 6];
  uint32_t st = status[e] | extra_status;
  if (any) st |= kStClip;
  const double m = flux / (rho * rho);
  if (!isfinite(m)) st |= kStNan;
  mag[e] = m;
  status[e] = st;
}

template <int N, template <int, int> class MAP>
hipError_t launch_rays_n(const Batch& b, const SectorBuf& sec, const RayWork& w, int n_r, int n_theta,
                         double delta_c, double* partial, uint8_t* clip, hipStream_t s) {
  const dim3 g((unsigned)(w.n * kMaxSectors)), blk(kWaves * 64);
  const int J = (n_theta + 63) / 64;
  if (J <= 4)
    hipLaunchKernelGGL((rays_kernel<N, 4, MAP<N, 4>>), g, blk, 0, s, b, sec, w, n_r, n_theta, delta_c, partial, clip);
  else if (J <= 8)
    hipLaunchKernelGGL((rays_kernel<N, 8, MAP<N, 8>>), g, blk, 0, s, b, sec, w, n_r, n_theta, delta_c, partial, clip);
  else if (J <= 16)
    hipLaunchKernelGGL((rays_kernel<N, 16, MAP<N, 16>>), g, blk, 0, s, b, sec, w, n_r, n_theta, delta_c, partial,
                       clip);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rays(int n_lens, int ray_fp32, const Batch& b, const SectorBuf& sec, const RayWork& w, int n_r,
                       int n_theta, double delta_c, double* partial, uint8_t* clip, hipStream_t s) {
  if (w.n == 0) return hipSuccess;
  if (n_lens == 2)
    return ray_fp32 ? launch_rays_n<2, MapF32>(b, sec, w, n_r, n_theta, delta_c, partial, clip, s)
                    : launch_rays_n<2, MapF64>(b, sec, w, n_r, n_theta, delta_c, partial, clip, s);
  return ray_fp32 ? launch_rays_n<3, MapF32>(b, sec, w, n_r, n_theta, delta_c, partial, clip, s)
                  : launch_rays_n<3, MapF64>(b, sec, w, n_r, n_theta, delta_c, partial, clip, s);
}

hipError_t launch_finalize(const Batch& b, const SectorBuf& sec, const RayWork& w, const double* partial,
                           const uint8_t* clip, int attempt, int max_retries, int32_t* next_list,
                           int32_t* next_count, double* mag, uint32_t* status, uint32_t extra_status,
                           hipStream_t s) {
  if (w.n == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((w.n + 255) / 256)), dim3(256), 0, s, b, sec, w, partial, clip,
                     attempt, max_retries, next_list, next_count, mag, status, extra_status);
  return hipGetLastError();
}

}  // namespace icrs
