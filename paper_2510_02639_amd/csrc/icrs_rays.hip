// icrs_rays.hip -- inverse ray shooting and row quadrature (Sec. 3.3, App. A).
//
// Persistent kernel: a grid sized to the chip; each workgroup (4 wave64s) takes the next task
// (all sectors of one epoch, or one (epoch, sector) item) from a device counter.  The
// N_r x N_theta polar grid is never stored: each wave owns every 4th row, lane l owns the
// columns l, l+64, l+128, ...  For one row a lane maps its nodes through the lens equation,
// adds the brightness of its inside nodes, and the wave takes ballots of chi = [d < rho].
// Inside nodes with an outside (or missing) neighbour are found with bit operations on the
// ballot masks and handed out one per lane; each queues its stencil (squared neighbour
// distances read back from a per-wave LDS row buffer) in a per-wave LDS queue, and one
// out-of-line pass solves 64 queued crossings at a time, rows mixed.
#include "icrs_device.hpp"
#include "icrs_launch.hpp"
#include "icrs_quad.hpp"

namespace icrs {

namespace {

constexpr int kWaves = 4;

// Node maps.  Column phases come from one sincos per lane and a rotation recurrence
// across the lane's columns (64 apart).
//
// MapF64 evaluates eq. lens_eq directly in FP64.
//
// MapF32 works relative to the sector's FP64 anchor z_s = r_s e^{i theta_s} (box centre):
// with dz = z - z_s = r e^{i theta_s}(e^{i dtheta} - 1) + (r - r_s) e^{i theta_s},
// u_k = z - a_k and h_k = eps_k/(z_s - a_k),
//   w - w_c = (w(z_s) - w_c) + dz + conj(dz sum_k h_k / u_k),
// an identity with no cancellation (each lens term eps_k/conj(u_k) minus its anchor value
// is -conj(dz h_k / u_k)), so FP32 rounding scales with |dz| (the sector's size) instead of
// |z|.
template <int N, int JMAX>
struct MapF64 {
  using T = double;
  static constexpr bool kRefine = false;
  // up to 512 columns: three waves per SIMD (168 VGPRs, a few spills) beat two and four
  static constexpr int kMinWaves = JMAX <= 8 ? 3 : 1;
  static constexpr bool kPhaseTable = false;
  static constexpr int kPhaseEntries = 1;
  double cs[JMAX], sn[JMAX];
  Lens<N> L;
  c64 wc;
  double r;
  __device__ void init_sector(const Lens<N>& lens, c64 w_c, const double* sp, int n_r, int n_theta, int lane,
                              const float2* phases) {
    (void)phases;
    L = lens;
    wc = w_c;
    (void)n_r;
    const double dth = (sp[3] - sp[2]) / n_theta;
    double s0, c0;
    sincos(sp[2] + (lane + 0.5) * dth, &s0, &c0);
    const c64 rot = expm1_i(64.0 * dth);  // e^{i 64 dtheta} - 1
    c64 e = mk(c0, s0);
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      cs[j] = e.x;
      sn[j] = e.y;
      e = e + e * rot;
    }
  }
  __device__ void init_row(double r_i, double dr_i) {
    (void)dr_i;
    r = r_i;
  }
  __device__ __forceinline__ double d2(int j) const {
    const double x = r * cs[j], y = r * sn[j];
    double wx = x - wc.x, wy = y - wc.y;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double dx = x - L.a[k].x, dy = y - L.a[k].y;
      const double inv = L.eps[k] * rcp_fast(fma(dx, dx, dy * dy));
      wx = fma(-inv, dx, wx);
      wy = fma(-inv, dy, wy);
    }
    return fma(wx, wx, wy * wy);
  }
};

template <int N, int JMAX>
struct MapF32 {
  using T = float;
  static constexpr bool kRefine = true;  // chi of nodes near the edge decided in FP64
  // an occupancy floor: the binary lens at four waves per SIMD (128 VGPRs, 160-270 B of
  // spills per lane) runs ~10% faster than at three and ~40% faster than at two; five or six
  // waves spill more than they gain; the triple lens is best at three
  static constexpr int kMinWaves = N == 2 ? 4 : 3;
  // the column phases g_l = e^{i theta_s} (e^{i dtheta_l} - 1): from 12 chunks per lane up
  // they live in a per-workgroup LDS table (JMAX x 64 entries) -- in registers they took
  // 2 JMAX of the 128 VGPRs and were spilled and reloaded in every row; below, registers
  // are faster (the table's read latency cost 4% at 8 chunks)
  static constexpr bool kPhaseTable = JMAX >= 12;
  static constexpr int kPhaseEntries = kPhaseTable ? JMAX * 64 : 1;
  static constexpr int kPhaseRegs = kPhaseTable ? 1 : JMAX;
  const float2* ph;          // this lane's column phases in the table, stride 64
  float gx[kPhaseRegs], gy[kPhaseRegs];  // or in registers
  float ux0, uy0;            // e^{i theta_s}
  float bx, by;              // w(z_s) - w_c
  float ax[N], ay[N], hx[N], hy[N];
  float r, ex, ey;           // row: r_i, (r_i - r_s) e^{i theta_s}
  // g_l for l = 0 .. 64 JMAX - 1, filled by the whole workgroup (threads t, t + 256, ...)
  __device__ static void fill_phases(float2* tab, const double* sp, int n_theta) {
    const double th_s = 0.5 * (sp[2] + sp[3]);
    const double dth = (sp[3] - sp[2]) / n_theta;
    double sa, ca;
    sincos(th_s, &sa, &ca);
    for (int l = (int)threadIdx.x; l < kPhaseEntries; l += (int)blockDim.x) {
      // e^{i dt_l} - 1 with dt_l = (l + 1/2 - N_theta/2) dtheta
      const c64 e = expm1_i((l + 0.5 - 0.5 * n_theta) * dth);
      tab[l] = make_float2((float)(ca * e.x - sa * e.y), (float)(ca * e.y + sa * e.x));
    }
  }
  __device__ void init_sector(const Lens<N>& L, c64 wc, const double* sp, int n_r, int n_theta, int lane,
                              const float2* phases) {
    (void)n_r;
    ph = phases + lane;
    const double r_s = 0.5 * (sp[0] + sp[1]);
    const double th_s = 0.5 * (sp[2] + sp[3]);
    const double dth = (sp[3] - sp[2]) / n_theta;
    double sa, ca;
    sincos(th_s, &sa, &ca);
    const double zx = r_s * ca, zy = r_s * sa;
    double wx = zx - wc.x, wy = zy - wc.y;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double dx = zx - L.a[k].x, dy = zy - L.a[k].y;
      const double s = L.eps[k] * rcp_fast(fma(dx, dx, dy * dy));  // eps/d = eps conj(d)/|d|^2
      wx = fma(-s, dx, wx);
      wy = fma(-s, dy, wy);
      ax[k] = (float)dx;
      ay[k] = (float)dy;
      hx[k] = (float)(s * dx);
      hy[k] = (float)(-s * dy);
    }
    bx = (float)wx;
    by = (float)wy;
    ux0 = (float)ca;
    uy0 = (float)sa;
    if constexpr (!kPhaseTable) {
      // E_j = e^{i dt_j} - 1 with dt_j = (l + 1/2 - N_theta/2) dtheta, l = lane + 64 j, by
      // the recurrence E_{j+1} = E_j + F + E_j F, F = e^{i 64 dtheta} - 1 (FP64)
      const c64 f = expm1_i(64.0 * dth);
      c64 e = expm1_i((lane + 0.5 - 0.5 * n_theta) * dth);
#pragma unroll
      for (int j = 0; j < kPhaseRegs; ++j) {
        gx[j] = (float)(ca * e.x - sa * e.y);
        gy[j] = (float)(ca * e.y + sa * e.x);
        e = e + f + e * f;
      }
    } else {
      (void)dth;
    }
  }
  __device__ void init_row(double r_i, double dr_i) {
    r = (float)r_i;
    ex = (float)dr_i * ux0;
    ey = (float)dr_i * uy0;
  }
  // w - w_c = B + dz + conj(dz G), G = sum_k h_k / u_k (dz factored out of the lens sum)
  __device__ __forceinline__ float d2(int j) const {
    float2 g;
    if constexpr (kPhaseTable) {
      g = ph[64 * j];
    } else {
      g = make_float2(gx[j], gy[j]);
    }
    const float dzx = fmaf(r, g.x, ex), dzy = fmaf(r, g.y, ey);
    float Gx = 0.0f, Gy = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const float ux = ax[k] + dzx, uy = ay[k] + dzy;
      const float inv = __builtin_amdgcn_rcpf(fmaf(ux, ux, uy * uy));
      const float px = fmaf(hx[k], ux, hy[k] * uy);  // h conj(u)
      const float py = fmaf(hy[k], ux, -hx[k] * uy);
      Gx = fmaf(px, inv, Gx);
      Gy = fmaf(py, inv, Gy);
    }
    const float Dx = (bx + dzx) + fmaf(dzx, Gx, -dzy * Gy);
    const float Dy = (by + dzy) - fmaf(dzx, Gy, dzy * Gx);
    return fmaf(Dx, Dx, Dy * Dy);
  }
};

// Rounding bound of the FP32 map on one sector, relative to rho: |dz| is at most the chord
// of the half angular width plus half the radial extent, and each lens term is at most
// eps_k |dz| / dist_k^2 with dist_k a lower bound of the lens' distance to the sector box.
// The map rounds quantities of that size a handful of times; four units in the last place
// (2^-22) per unit of |dz| amp / rho keep the figure above the error of an FP32 emulation of
// the map on sampled workload sectors, which reaches 2.3 units.
template <int N>
__device__ inline double fp32_error_bound(const Lens<N>& L, const double* sp, bool per, double rho) {
  const double r_lo = sp[0], r_hi = sp[1], th_lo = sp[2], th_hi = sp[3];
  const double half = per ? kPi : 0.5 * (th_hi - th_lo);
  const double dz = 2.0 * r_hi * sin(0.5 * fmin(half, kPi)) + 0.5 * (r_hi - r_lo);
  double amp = 1.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double rk = sqrt(norm2(L.a[k]));
    const double tk = atan2(L.a[k].y, L.a[k].x);
    const double dr = fmax(fmax(r_lo - rk, rk - r_hi), 0.0);
    double dth = 0.0;
    if (!per) {  // circular distance from tk to [th_lo, th_hi]
      const double off = remainder(tk - 0.5 * (th_lo + th_hi), 2.0 * kPi);
      dth = fmax(fabs(off) - half, 0.0);
    }
    const double dist = fmax(dr, rk * (dth >= 0.5 * kPi ? 1.0 : sin(dth)));
    amp += (dist > 0.0) ? L.eps[k] / (dist * dist) : 1e300;
  }
  return 0x1p-22 * (1.0 + dz * amp / rho);
}
constexpr double kFp32Budget = 3e-5;  // per-node distance error (relative to rho) allowed in FP32

// Nodes whose FP32 squared distance lies within 2 e_s + 2^-21 (relative to rho^2) of rho^2,
// e_s the sector's rounding bound, have chi decided by the FP64 map: under the limb-darkened
// edge rule a flipped node moves the sector's flux by a sizeable part of a node's weight, which
// in a poorly resolved image exceeds the FP32 tolerance.  The FP64 evaluation stays out of
// line: inlined into the row loop it costs the hot path registers.
//
// |w(z) - w_c|^2 at z = r e^{i theta} in FP64 (eq. lens_eq).
template <int N>
__device__ __attribute__((noinline)) double node_d2_f64(const Lens<N> L, c64 wc, double r, double theta) {
  double s, c;
  sincos(theta, &s, &c);
  const double x = r * c, y = r * s;
  double wx = x - wc.x, wy = y - wc.y;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double dx = x - L.a[k].x, dy = y - L.a[k].y;
    const double inv = L.eps[k] / fma(dx, dx, dy * dy);
    wx = fma(-inv, dx, wx);
    wy = fma(-inv, dy, wy);
  }
  return fma(wx, wx, wy * wy);
}

// The limb-darkened edge rule jumps at delta = delta_c (by 0.41 of the node's brightness at
// delta_c = 0.1), so which side of delta_c a crossing falls on is a decision, like chi.  An
// FP32 crossing whose delta lies within rounding of delta_c is retaken here: FP64 distances
// of the stencil nodes p-1 .. p+2 of column p (eq. lens_eq), the same interpolant and edge
// rule (App. A); returns the item's I (f(delta) - 1), the brightness at the boundary node (p
// for a right-side item, p + 1 for a left-side one) in FP64 too.
template <int N>
__device__ __attribute__((noinline)) double crossing_term_f64(const Lens<N> L, c64 wc, double r, double th0,
                                                              double dth, int p, int flags, double rho, double u1,
                                                              double delta_c, double i_lin, double i_sqrt) {
  const bool cubic = (flags & 2) != 0;
  double d2[4] = {0.0, 0.0, 0.0, 0.0}, d[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < 4; ++k) {
    if (cubic || k == 1 || k == 2) {
      d2[k] = node_d2_f64<N>(L, wc, r, th0 + (p + k - 0.5) * dth);
      d[k] = sqrt(d2[k]);
    }
  }
  const double t = crossing_t<double>(d[0], d[1], d[2], d[3], cubic, rho);
  const double b = brightness<double>((flags & 1) ? d2[1] : d2[2], 1.0 / (rho * rho), i_lin, i_sqrt);
  return b * (edge_factor<double>((flags & 1) ? t : 1.0 - t, u1, delta_c) - 1.0);
}


// Wave-uniform boundary words of chunk j: inside nodes whose left (side 0) or right
// (side 1) neighbour is outside or beyond a non-periodic edge.
template <int JMAX>
__device__ __forceinline__ uint64_t boundary_word(const uint64_t (&m)[JMAX], int j, int J, int side, bool per,
                                                  uint64_t in_last, int jl, int bl) {
  if (side == 0) {
    const uint64_t carry = (j > 0) ? (m[j > 0 ? j - 1 : 0] >> 63) : (per ? in_last : 0ull);
    return m[j] & ~((m[j] << 1) | carry);
  }
  uint64_t right = (m[j] >> 1) | ((j + 1 < J) ? (m[j + 1 < JMAX ? j + 1 : j] << 63) : 0ull);
  if (j == jl && per) right |= (m[0] & 1ull) << bl;
  return m[j] & ~right;
}

// Per-wave queue of boundary nodes waiting for their crossing correction.  Rows append
// their (node, side) items with the stencil already read from the row buffer; one pass of
// 64 lanes then solves 64 crossings at once instead of a handful per row.  An item's row
// radius is its weight r_i.
constexpr int kQueue = 128;

template <typename T>
struct CrossQueue {
  T d[4][kQueue];    // squared stencil distances d_{p-1}^2 .. d_{p+2}^2 (an edge item keeps its node's in d[1])
  double r[kQueue];  // its row radius
  int f[kQueue];     // bit 0: side (1 = right), bit 1: cubic stencil, bit 2: neighbour beyond an edge,
                     // bits 3-12: the bracket's left column p, bits 13+: the row
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// clip bit of a sector whose retake list was full (the FP64 pass redoes it)
constexpr int kClipRetakeOverflow = 256;

// Per-wave staging of the crossings to retake (their queue flags): the row loop writes LDS
// only, and the wave copies the list to the global one once per sector, so no global
// pointer is live in the loop.  A wave with more than kRetake in one sector overflows.
// Kept small: at 64 columns per lane the kernel's LDS stays under the 40 KB that leaves room
// for four workgroups per CU.
constexpr int kRetake = 16;

struct RetakeList {
  int f[kRetake];
};

// sum over the n queued items of r_i I (f(delta) - 1), lane k taking items k, k + 64, ...;
// square roots and brightness are taken here, where every lane has an item.  Inlined: as an
// out-of-line call its register saves and restores cost 4-5% of the kernel.
//
// FP32 only, for the edge rule's jump at delta_c (crossing_term_f64): t_err is 2.5 times
// the bound (e_s + 2^-21) rho on a stencil distance's error; the cubic's Lebesgue constant
// on [0, 1] is 1.25, so the FP32 crossing lies within t_err / 2 / abs(L'(t)) of the exact
// one, plus the solver's 1e-6 step tolerance.  An item with delta that close to delta_c
// adds nothing here and is staged in rl, rl_n counting all of them (wave-uniform).
template <typename T>
__device__ __forceinline__ double flush_crossings(const CrossQueue<T>* q, int n, T rho, T u1, T delta_c,
                                                  T f_edge, T inv_rho2, T i_lin, T i_sqrt, T t_err,
                                                  RetakeList* rl, int& rl_n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int base = 0; base < n; base += 64) {
    const int k = base + lane;
    bool take = false;
    int f = 0;
    if (k < n) {
      f = q->f[k];
      // the boundary node is p (right side, or an edge item) or p + 1 (left side)
      const T b = brightness<T>((f & 5) ? q->d[1][k] : q->d[2][k], inv_rho2, i_lin, i_sqrt);
      T corr;
      if (f & 4) {
        corr = f_edge;
      } else {
        // side 0: crossing in (theta_{l-1}, theta_l), delta = 1 - t; side 1: in (theta_l, theta_{l+1}), delta = t
        const bool cubic = (f & 2) != 0;
        T slope;
        const T t = crossing_t<T>(sqrt_fast(q->d[0][k]), sqrt_fast(q->d[1][k]), sqrt_fast(q->d[2][k]),
                                  sqrt_fast(q->d[3][k]), cubic, rho, &slope);
        const T delta = (f & 1) ? t : T(1) - t;
        corr = edge_factor<T>(delta, u1, delta_c) - T(1);
        if constexpr (sizeof(T) == 4) {
          slope = fabs(slope);
          take = u1 != T(0) && fabs(delta - delta_c) * slope <= t_err + T(4e-6) * slope;
        }
      }
      if (!take) s += q->r[k] * (double)(b * corr);
    }
    if constexpr (sizeof(T) == 4) {
      const uint64_t tm = __ballot(take);
      if (tm) {
        const int pos = rl_n + (int)__popcll(tm & ((1ull << lane) - 1ull));
        if (take && pos < kRetake) rl->f[pos] = f;
        rl_n += (int)__popcll(tm);
      }
    }
  }
  return s;
}

// One (epoch, sector) grid shot by the whole workgroup; the flux and clip bits end up in
// thread 0, with kClipRetakeOverflow set when an FP32 wave listed more crossings near delta_c
// than it can retake (the flux is then incomplete).  EXACT: n_theta == 64 * JMAX (no partial
// column chunk).
template <int N, int JMAX, bool EXACT, typename MAP>
__device__ inline void shoot_sector(const double* sp, bool per, const Lens<N>& L, c64 wc, double rho_d, double u1_d,
                                    double delta_c_d, int n_r, int n_theta, typename MAP::T* rowbuf_all,
                                    uint64_t* bwords, CrossQueue<typename MAP::T>* queues, double* wsum,
                                    int* wclip, double ebound, float2* phase_sh, RetakeList* retakes,
                                    const RayWork& w, int code, double* flux_out, int* clip_out_bits) {
  using T = typename MAP::T;
  const int lane = threadIdx.x & 63;
  // wave-uniform, which the compiler cannot tell from threadIdx.x >> 6: without it the row
  // loop counter is taken as divergent and the loop carries its conditions in vector registers
  // (2-9% on the binary lens; the triple lens's register allocation does 4% worse with it)
  const int wave = N == 2 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const double r_lo = sp[0], r_hi = sp[1];
  const T rho = (T)rho_d, u1 = (T)u1_d, delta_c = (T)delta_c_d;
  const T rho2 = (T)(rho_d * rho_d), inv_rho2 = (T)(1.0 / (rho_d * rho_d));
  const T chi_band = (T)((2.0 * ebound + 0x1p-21) * rho_d * rho_d);
  const double I0d = 3.0 / (kPi * (3.0 - u1_d));
  const T i_lin = (T)(I0d * (1.0 - u1_d)), i_sqrt = (T)(I0d * u1_d);
  const int J = EXACT ? JMAX : (n_theta + 63) >> 6;
  const double dr = (r_hi - r_lo) / n_r;
  const double dth = (sp[3] - sp[2]) / n_theta;
  const T f_edge = edge_factor<T>(T(0.5), u1, delta_c) - T(1);  // neighbour beyond a sector edge
  const T t_err = (T)(2.5 * (ebound + 0x1p-21) * rho_d);
  const int last = (EXACT ? 64 * JMAX : n_theta) - 1;  // a compile-time constant for exact grids
  const int jl = last >> 6, bl = last & 63;

  if constexpr (MAP::kPhaseTable) {
    MAP::fill_phases(phase_sh, sp, n_theta);
    __syncthreads();
  }
  MAP map;
  map.init_sector(L, wc, sp, n_r, n_theta, lane, phase_sh);

  double acc = 0.0;
  int clip = 0;
  T* buf = rowbuf_all + wave * (JMAX * 64);
  uint64_t* bwl = bwords + wave * (2 * JMAX);
  CrossQueue<T>* cq = queues + wave;
  int qn = 0;
  RetakeList* rl = retakes + (sizeof(T) == 4 ? wave : 0);  // FP64 maps have one unused list
  int rl_n = 0;

  // Chunk culling: a 64-column chunk of a row is skipped when the arc through it, widened
  // by two columns on each side, provably maps farther than rho (1 + 1e-3) from the source
  // centre -- beyond the FP32 map's rounding budget, so every node there would be outside,
  // and no crossing stencil (at most two columns from an inside node) reaches into it.
  // One test pass per wave covers G = 64 / J of its rows: lane (st, jt) tests chunk jt of
  // the st-th next row.  Skipping changes no result bit.
  const int G = 64 / J;
  const int jt = lane % J, st = lane / J;
  double tcs, tsn;
  sincos(sp[2] + (64.0 * jt + 32.0) * dth, &tsn, &tcs);
  const double Phi = 34.0 * dth;
  uint64_t skipmask = 0;
  int it = 0;
  for (int i = wave; i < n_r; i += kWaves, ++it) {
    const int s = it % G;
    if (s == 0) {
      bool sk = false;
      const int is = i + kWaves * st;
      if (st < G && is < n_r)
        sk = arc_distance_lower_bound<N>(L, wc, r_lo + (is + 0.5) * dr, tcs, tsn, Phi) > rho_d * 1.001;
      skipmask = __ballot(sk);
    }
    const uint32_t rowskip = (uint32_t)(skipmask >> (s * J)) & ((1u << J) - 1u);
    if (rowskip == (1u << J) - 1u) continue;  // the whole row misses the image
    const double r = r_lo + (i + 0.5) * dr;
    map.init_row(r, (i + 0.5 - 0.5 * n_r) * dr);
    uint64_t m[JMAX];
    uint64_t any = 0;
    // the row's inside nodes: count, first and last column (for the one-run test below)
    int n_in = 0, first = 0, lastc = 0;
    T row = T(0);
    T mind = T(__builtin_inf());  // closest |d^2 - rho^2| among the lane's nodes of the row
#pragma unroll
    for (int j = 0; j < JMAX; ++j) {
      m[j] = 0;
      if ((EXACT || j < J) && !((rowskip >> j) & 1u)) {
        T d2 = map.d2(j);
        if (!EXACT) d2 = (lane + 64 * j < n_theta) ? d2 : T(__builtin_inf());
        if constexpr (MAP::kRefine) mind = fmin(mind, fabs(d2 - rho2));
        const bool in = d2 < rho2;
        m[j] = __ballot(in);
        any |= m[j];
        if (EXACT || lane + 64 * j < n_theta) buf[lane + 64 * j] = d2;
        if (m[j]) {
          // an empty inline asm keeps this wave-uniform branch a branch: without it the
          // compiler computes the brightness for every chunk and selects
          __asm__ volatile("");
          row += in ? brightness<T>(d2, inv_rho2, i_lin, i_sqrt) : T(0);
          if (n_in == 0) first = 64 * j + (int)__builtin_ctzll(m[j]);
          n_in += __popcll(m[j]);
          lastc = 64 * j + 63 - (int)__builtin_clzll(m[j]);
        }
      }
    }
    if constexpr (MAP::kRefine) {
      if (__ballot(mind <= chi_band)) {
        // chi of the nodes in the band decided in FP64; the stored FP32 value keeps the
        // decision (d2 < rho2 iff inside) and the row sum swaps the node's brightness
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < JMAX; ++j)
          if ((EXACT || j < J) && !((rowskip >> j) & 1u) && (EXACT || lane + 64 * j < n_theta))
            mine |= (fabs(buf[lane + 64 * j] - rho2) <= chi_band ? 1u : 0u) << j;
        while (mine) {
          const int j = __ffs(mine) - 1;
          mine &= mine - 1u;
          const int l = lane + 64 * j;
          const T old = buf[l];
          const double e = node_d2_f64<N>(L, wc, r, sp[2] + (l + 0.5) * dth);
          const bool in = e < rho_d * rho_d;
          const T d2 = in ? fmin((T)e, nextafterf(rho2, T(0))) : fmax((T)e, rho2);
          buf[l] = d2;
          row += (in ? brightness<T>(d2, inv_rho2, i_lin, i_sqrt) : T(0)) -
                 (old < rho2 ? brightness<T>(old, inv_rho2, i_lin, i_sqrt) : T(0));
        }
        any = 0;
        n_in = 0;
#pragma unroll
        for (int j = 0; j < JMAX; ++j) {
          if ((EXACT || j < J) && !((rowskip >> j) & 1u))
            m[j] = __ballot((EXACT || lane + 64 * j < n_theta) && buf[lane + 64 * j] < rho2);
          any |= m[j];
          if (m[j]) {
            if (n_in == 0) first = 64 * j + (int)__builtin_ctzll(m[j]);
            n_in += __popcll(m[j]);
            lastc = 64 * j + 63 - (int)__builtin_clzll(m[j]);
          }
        }
      }
    }
    if (any == 0) continue;  // wave-uniform: the row misses the image
    if (i == 0 && r_lo > 0.0) clip |= 1;
    if (i == n_r - 1) clip |= 2;
    uint64_t m_last = 0;
#pragma unroll
    for (int j = 0; j < JMAX; ++j)
      if (j == jl) m_last = m[j];
    const uint64_t in_last = (m_last >> bl) & 1ull;
    if (!per) {
      if (m[0] & 1ull) clip |= 4;
      if (in_last) clip |= 8;
    }
    // Boundary items: inside nodes whose left (side 0) or right (side 1) neighbour is outside
    // or beyond a non-periodic edge.  A row whose inside nodes form one run -- an image
    // crossed once, most rows -- has exactly one per side, its first and last inside column,
    // known from the masks' population count and bit scans taken while the row was mapped
    // (all scalar), and queued from lanes 0 and 1.  A run that touches both ends of a periodic ring may wrap around and
    // takes the general path with the other rows.
    const bool one_run = n_in == lastc - first + 1 && !(per && (first == 0 || lastc == last));
    // the row buffer's stencil values are read across lanes below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // one item: its stencil (squared distances from the row buffer), row radius and flags
    auto enqueue = [&](int side, int l, int slot) {
      int fl = side;
      if ((side == 0 && l == 0 && !per) || (side == 1 && l == last && !per)) {
        fl |= 4;
        cq->d[1][slot] = buf[l];
      } else {
        // side 0: crossing in (theta_{l-1}, theta_l), bracket p = l-1; side 1: in (theta_l, theta_{l+1}), p = l
        const int pp = side ? l : (l == 0 ? last : l - 1);
        const bool cubic = per || (pp - 1 >= 0 && pp + 2 <= last);
        // neighbours of pp in [0, n_theta): wrap by one subtraction (periodic) or clamp
        const int im1 = per ? (pp == 0 ? last : pp - 1) : max(pp - 1, 0);
        const int ip1 = pp == last ? 0 : pp + 1;
        const int ip2 = per ? (pp + 2 > last ? pp + 1 - last : pp + 2) : min(pp + 2, last);
        cq->d[0][slot] = buf[im1];
        cq->d[1][slot] = buf[pp];
        cq->d[2][slot] = buf[ip1];
        cq->d[3][slot] = buf[ip2];
        if (cubic) fl |= 2;
        fl |= (pp << 3) | (i << 13);
      }
      cq->r[slot] = r;
      cq->f[slot] = fl;
    };
    if (one_run) {
      if (qn + 2 > kQueue) {
        wave_lds_sync();
        acc += flush_crossings<T>(cq, qn, rho, u1, delta_c, f_edge, inv_rho2, i_lin, i_sqrt, t_err, rl, rl_n);
        wave_lds_sync();
        qn = 0;
      }
      if (lane < 2) enqueue(lane, lane ? lastc : first, qn + lane);
      qn += 2;
    } else {
      // general rows: boundary words per chunk (their popcounts scalar, the words in LDS);
      // lane k finds the k-th item by comparing counts and reading one word
      int n_left = 0, n_all = 0;
      int pc0[JMAX], pc1[JMAX];
#pragma unroll
      for (int j = 0; j < JMAX; ++j) {
        pc0[j] = pc1[j] = 0;
        if ((EXACT || j < J) && m[j]) {  // an empty chunk has no boundary nodes
          const uint64_t w0 = boundary_word<JMAX>(m, j, J, 0, per, in_last, jl, bl);
          const uint64_t w1 = boundary_word<JMAX>(m, j, J, 1, per, in_last, jl, bl);
          pc0[j] = __popcll(w0);
          pc1[j] = __popcll(w1);
          n_left += pc0[j];
          n_all += pc1[j];
          if (lane == 0) {
            bwl[j] = w0;
            bwl[JMAX + j] = w1;
          }
        }
      }
      n_all += n_left;
      wave_lds_sync();
      // 64 items per step, flushing when the queue would overflow
      for (int base = 0; base < n_all; base += 64) {
        if (qn + 64 > kQueue) {
          wave_lds_sync();
          acc += flush_crossings<T>(cq, qn, rho, u1, delta_c, f_edge, inv_rho2, i_lin, i_sqrt, t_err, rl, rl_n);
          wave_lds_sync();
          qn = 0;
        }
        const int k = base + lane;
        if (k < n_all) {
          const int side = k >= n_left ? 1 : 0;
          int rem = side ? k - n_left : k;
          int jw = 0;
#pragma unroll
          for (int j = 0; j < JMAX; ++j) {
            if (EXACT || j < J) {
              const int pc = side ? pc1[j] : pc0[j];
              if (rem >= 0 && rem < pc) jw = j;
              if (rem >= 0) rem -= (rem < pc) ? (1 << 30) : pc;
            }
          }
          uint64_t word = bwl[side * JMAX + jw];
          rem += 1 << 30;  // rank of the node inside its word (< 64 whenever k < n_all)
          for (int q = 0; q < rem && q < 64; ++q) word &= word - 1ull;
          enqueue(side, 64 * jw + __ffsll((unsigned long long)word) - 1, qn + lane);
        }
        qn += min(64, n_all - base);
      }
    }
    acc += r * (double)row;
    __builtin_amdgcn_wave_barrier();
  }

  if (qn > 0) {
    wave_lds_sync();
    acc += flush_crossings<T>(cq, qn, rho, u1, delta_c, f_edge, inv_rho2, i_lin, i_sqrt, t_err, rl, rl_n);
  }
  if constexpr (sizeof(T) == 4) {
    // the staged crossings to the global list, one reservation per wave.  Every reserved slot
    // below the capacity is written (the retake kernel reads all of them); an overflowed
    // sector's retakes are harmless, as the FP64 pass overwrites its flux.
    if (rl_n > 0) {
      const int nw = min(rl_n, kRetake);
      unsigned long long at = 0;
      if (lane == 0) at = atomicAdd(w.n_retake, (unsigned long long)nw);
      at = __shfl(at, 0);
      if (rl_n > kRetake || at + nw > (unsigned long long)w.retake_cap) clip |= kClipRetakeOverflow;
      wave_lds_sync();
      if (lane < nw && at + lane < (unsigned long long)w.retake_cap) {
        w.retake[2 * (at + lane)] = code;
        w.retake[2 * (at + lane) + 1] = rl->f[lane];
      }
    }
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
    *flux_out = tot * dr * dth;
    *clip_out_bits = c;
  }
  __syncthreads();
}

// Persistent ray kernel.  Tasks come from a device counter: with w.items set, task k is the
// single sector w.items[k] = 16 e + slot (k < *w.n_items); otherwise task k is every sector
// of epoch w.list[k] (or k).  An FP32 pass sends sectors whose rounding bound exceeds the
// budget, and those with more crossings near delta_c than the waves retake, to w.fallback
// for the FP64 pass (an FP32 pass always has the list).  Every workgroup leaves once the
// counter has passed the end.
template <int N, int JMAX, bool EXACT, typename MAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MAP::kMinWaves))) void rays_kernel(
    Batch b, SectorBuf sec, RayWork w, int n_r, int n_theta, double delta_c, double* __restrict__ partial,
    uint8_t* __restrict__ clip_out, unsigned long long* __restrict__ queue) {
  using T = typename MAP::T;
  __shared__ T rowbuf[kWaves * JMAX * 64];
  __shared__ uint64_t bwords[kWaves * 2 * JMAX];
  __shared__ CrossQueue<T> queues[kWaves];
  __shared__ double wsum[kWaves];
  __shared__ int wclip[kWaves];
  __shared__ unsigned long long next_sh;
  __shared__ double ebound_sh[kMaxSectors];
  __shared__ float2 phase_sh[MAP::kPhaseEntries];
  __shared__ RetakeList retakes[sizeof(T) == 4 ? kWaves : 1];

  const unsigned long long total = w.items   ? (unsigned long long)(*w.n_items)
                                   : w.n_dev ? (unsigned long long)(*w.n_dev)
                                             : (unsigned long long)w.n;
  // thread 0 takes the next task's ticket when it starts a task, so the atomic's round trip
  // overlaps the task's work
  if (threadIdx.x == 0) next_sh = atomicAdd(queue, 1ull);
  __syncthreads();
  unsigned long long idx = next_sh;
  __syncthreads();
  while (idx < total) {
    unsigned long long ticket = 0;
    if (threadIdx.x == 0) ticket = atomicAdd(queue, 1ull);
    int64_t e;
    int s0, s1;
    if (w.items) {
      const int32_t it = w.items[idx];
      e = it >> 4;
      s0 = it & 15;
      s1 = s0 + 1;
    } else {
      e = w.list ? (int64_t)w.list[idx] : (int64_t)idx;
      s0 = 0;
      s1 = sec.nsec[e];
      if (s1 < 0 || s1 > kMaxSectors) s1 = 0;  // out of range: no rays (finalize flags the epoch)
    }
    const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
    const Lens<N> L = make_lens<N>(p);
    const c64 wc = source_center(p, b.t[e]);
    if constexpr (sizeof(T) == 4) {
      // the task's sectors get their rounding bounds in parallel, one lane each; sectors
      // over the budget are listed for the FP64 pass
      const int slot = s0 + (int)threadIdx.x;
      if (slot < s1) {
        const double* sp = sec.sectors + (e * kMaxSectors + slot) * 4;
        const double eb = fp32_error_bound<N>(L, sp, sec.periodic[e * kMaxSectors + slot] != 0, p[6]);
        ebound_sh[threadIdx.x] = eb;
        if (w.fallback && eb > kFp32Budget) w.fallback[atomicAdd(w.n_fallback, 1)] = (int32_t)(e * 16 + slot);
      }
      __syncthreads();
    }
    for (int slot = s0; slot < s1; ++slot) {
      const double* sp = sec.sectors + (e * kMaxSectors + slot) * 4;
      const bool per = sec.periodic[e * kMaxSectors + slot] != 0;
      double ebound = 0.0;
      if constexpr (sizeof(T) == 4) {
        ebound = ebound_sh[slot - s0];
        if (w.fallback && ebound > kFp32Budget) continue;  // uniform: one LDS value for the workgroup
      }
      double flux = 0.0;
      int c = 0;
      shoot_sector<N, JMAX, EXACT, MAP>(sp, per, L, wc, p[6], p[7], delta_c, n_r, n_theta, rowbuf, bwords, queues, wsum,
                                        wclip, ebound, phase_sh, retakes, w, (int)(e * 16 + slot), &flux, &c);
      if (threadIdx.x == 0) {
        partial[e * kMaxSectors + slot] = flux;
        clip_out[e * kMaxSectors + slot] = (uint8_t)c;
        if constexpr (sizeof(T) == 4) {
          // the retake kernel adds into the sector's sum from zero; the FP64 pass overwrites
          // partial and clip of an overflowed sector
          w.retake_fx[e * kMaxSectors + slot] = 0ull;
          if (c & kClipRetakeOverflow) w.fallback[atomicAdd(w.n_fallback, 1)] = (int32_t)(e * 16 + slot);
        }
      }
    }
    if (threadIdx.x == 0) next_sh = ticket;
    __syncthreads();
    idx = next_sh;
    __syncthreads();
  }
}

// FP64 retake of the crossings an FP32 pass listed (one per thread): its term r I (f(delta) - 1)
// goes into the sector's sum as an integer multiple of 2^-40, so the sum is the same whatever
// order the atomic additions take (a term's magnitude is below r_max I0 < 2^22).
template <int N>
__global__ __launch_bounds__(256) void retake_kernel(Batch b, SectorBuf sec, RayWork w, int n_r, int n_theta,
                                                     double delta_c) {
  const int64_t n = (int64_t)min(*w.n_retake, (unsigned long long)w.retake_cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int code = w.retake[2 * k], f = w.retake[2 * k + 1];
    const int64_t e = code >> 4;
    const int slot = code & 15;
    const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
    const Lens<N> L = make_lens<N>(p);
    const c64 wc = source_center(p, b.t[e]);
    const double* sp = sec.sectors + (e * kMaxSectors + slot) * 4;
    // the same row radius and column width as the ray kernel
    const double dr = (sp[1] - sp[0]) / n_r, dth = (sp[3] - sp[2]) / n_theta;
    const double r = sp[0] + ((f >> 13) + 0.5) * dr;
    const double rho = p[6], u1 = p[7];
    const double I0 = 3.0 / (kPi * (3.0 - u1));
    const double term =
        r * crossing_term_f64<N>(L, wc, r, sp[2], dth, (f >> 3) & 1023, f, rho, u1, delta_c, I0 * (1.0 - u1), I0 * u1);
    atomicAdd(&w.retake_fx[e * kMaxSectors + slot], (unsigned long long)llrint(ldexp(term, 40)));
  }
}

// Adds each listed sector's retake sum to its flux once: the first thread to exchange the sum
// for zero holds all of it.
__global__ __launch_bounds__(256) void retake_fold_kernel(SectorBuf sec, RayWork w, int n_r, int n_theta,
                                                          double* __restrict__ partial) {
  const int64_t n = (int64_t)min(*w.n_retake, (unsigned long long)w.retake_cap);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int code = w.retake[2 * k];
    const int64_t at = (code >> 4) * kMaxSectors + (code & 15);
    const unsigned long long v = atomicExch(&w.retake_fx[at], 0ull);
    if (v != 0ull) {
      const double* sp = sec.sectors + at * 4;
      const double dr = (sp[1] - sp[0]) / n_r, dth = (sp[3] - sp[2]) / n_theta;
      partial[at] += ldexp((double)(long long)v, -40) * dr * dth;
    }
  }
}

__global__ void finalize_kernel(Batch b, SectorBuf sec, RayWork w, const double* __restrict__ partial,
                                const uint8_t* __restrict__ clip, int attempt, int max_retries,
                                int32_t* __restrict__ next_list, int32_t* __restrict__ next_count,
                                double* __restrict__ mag, uint32_t* __restrict__ status, uint32_t extra_status,
                                unsigned long long* __restrict__ passes, const double* __restrict__ add_mag) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (w.n_dev ? (int64_t)(*w.n_dev) : w.n)) return;
  const int64_t e = w.list ? (int64_t)w.list[idx] : idx;
  // a sector count outside 0..kMaxSectors (only from a caller's given list) is not used
  const int ns_in = sec.nsec[e];
  const bool bad_ns = ns_in < 0 || ns_in > kMaxSectors;
  const int ns = bad_ns ? 0 : ns_in;
  if (passes && ns) atomicAdd(passes, (unsigned long long)ns);
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
  const double m = bad_ns ? __builtin_nan("") : flux / (rho * rho) + (add_mag ? add_mag[e] : 0.0);
  if (bad_ns) st |= kStBadSectors;
  if (!isfinite(m)) st |= kStNan;
  mag[e] = m;
  status[e] = st;
}

template <int N, int JMAX, bool EXACT, template <int, int> class MAP>
hipError_t launch_rays_j(const Batch& b, const SectorBuf& sec, const RayWork& w, int n_r, int n_theta,
                         double delta_c, double* partial, uint8_t* clip, unsigned long long* queue, hipStream_t s) {
  auto kern = rays_kernel<N, JMAX, EXACT, MAP<N, JMAX>>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWaves * 64, 0);
  if (e != hipSuccess) return e;
  int64_t grid = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  if (!w.items && w.n < grid) grid = w.n;
  if (grid < 1) grid = 1;
  e = launch_fill_i32((int32_t*)queue, 2, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kWaves * 64), 0, s, b, sec, w, n_r, n_theta, delta_c, partial,
                     clip, queue);
  return hipGetLastError();
}

template <int N, template <int, int> class MAP>
hipError_t launch_rays_n(const Batch& b, const SectorBuf& sec, const RayWork& w, int n_r, int n_theta,
                         double delta_c, double* partial, uint8_t* clip, unsigned long long* queue, hipStream_t s) {
  const int J = (n_theta + 63) / 64;
  const bool exact = (n_theta % 64) == 0;
#define ICRS_RAYS_J(JJ)                                                                                   \
  if (J <= JJ) {                                                                                          \
    if (exact && J == JJ)                                                                                 \
      return launch_rays_j<N, JJ, true, MAP>(b, sec, w, n_r, n_theta, delta_c, partial, clip, queue, s);  \
    return launch_rays_j<N, JJ, false, MAP>(b, sec, w, n_r, n_theta, delta_c, partial, clip, queue, s);   \
  }
  ICRS_RAYS_J(2)
  ICRS_RAYS_J(4)
  ICRS_RAYS_J(8)
  ICRS_RAYS_J(12)
  ICRS_RAYS_J(16)
#undef ICRS_RAYS_J
  return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_rays_lens(int ray_fp32, int stage, const Batch& b, const SectorBuf& sec, const RayWork& w,
                            int n_r, int n_theta, double delta_c, double* partial, uint8_t* clip,
                            unsigned long long* queue, int32_t* fallback, int32_t* n_fallback, const RetakeBuf& rb,
                            hipStream_t s) {
  if (!ray_fp32)
    return stage == 0 ? launch_rays_n<N, MapF64>(b, sec, w, n_r, n_theta, delta_c, partial, clip, queue, s)
                      : hipSuccess;
  if (stage == 0) {
    // FP32 pass; sectors over the rounding budget are listed for the FP64 pass, crossings
    // next to delta_c for the retake, which follows at once
    if (!rb.items || !rb.n || !rb.fx || rb.cap < 0) return hipErrorInvalidValue;
    hipError_t e = launch_fill_i32(n_fallback, 1, 0, s);
    if (e == hipSuccess) e = launch_fill_i32((int32_t*)rb.n, 2, 0, s);
    if (e != hipSuccess) return e;
    RayWork w32 = w;
    w32.fallback = fallback;
    w32.n_fallback = n_fallback;
    w32.retake = rb.items;
    w32.n_retake = rb.n;
    w32.retake_cap = rb.cap;
    w32.retake_fx = rb.fx;
    e = launch_rays_n<N, MapF32>(b, sec, w32, n_r, n_theta, delta_c, partial, clip, queue, s);
    if (e != hipSuccess) return e;
    // grid-stride over the device-side count: 1024 x 256 threads cover a typical list in a
    // few strides
    hipLaunchKernelGGL(retake_kernel<N>, dim3(1024), dim3(256), 0, s, b, sec, w32, n_r, n_theta, delta_c);
    hipLaunchKernelGGL(retake_fold_kernel, dim3(1024), dim3(256), 0, s, sec, w32, n_r, n_theta, partial);
    return hipGetLastError();
  }
  RayWork w64{};
  w64.items = fallback;
  w64.n_items = n_fallback;
  w64.n = 1;
  return launch_rays_n<N, MapF64>(b, sec, w64, n_r, n_theta, delta_c, partial, clip, queue, s);
}

}  // namespace

hipError_t launch_rays(int n_lens, int ray_fp32, int stage, const Batch& b, const SectorBuf& sec, const RayWork& w,
                       int n_r, int n_theta, double delta_c, double* partial, uint8_t* clip,
                       unsigned long long* queue, int32_t* fallback, int32_t* n_fallback, const RetakeBuf& rb,
                       hipStream_t s) {
  if (w.n == 0) return hipSuccess;
  if (n_lens == 2)
    return launch_rays_lens<2>(ray_fp32, stage, b, sec, w, n_r, n_theta, delta_c, partial, clip, queue, fallback,
                               n_fallback, rb, s);
  return launch_rays_lens<3>(ray_fp32, stage, b, sec, w, n_r, n_theta, delta_c, partial, clip, queue, fallback,
                             n_fallback, rb, s);
}

hipError_t launch_finalize(const Batch& b, const SectorBuf& sec, const RayWork& w, const double* partial,
                           const uint8_t* clip, int attempt, int max_retries, int32_t* next_list,
                           int32_t* next_count, double* mag, uint32_t* status, uint32_t extra_status,
                           unsigned long long* passes, hipStream_t s, const double* add_mag) {
  if (w.n == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((w.n + 255) / 256)), dim3(256), 0, s, b, sec, w, partial, clip,
                     attempt, max_retries, next_list, next_count, mag, status, extra_status, passes, add_mag);
  return hipGetLastError();
}

}  // namespace icrs
