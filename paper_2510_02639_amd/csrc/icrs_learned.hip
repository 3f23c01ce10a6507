// icrs_learned.hip -- per-image polar boxes for the learned-bounds path.
//
// The plain sector step (Sec. 3.2) solves the lens polynomial at n_limb points of the
// source limb and bins every limb image.  The learned path instead
//   1. solves a few limb points (n_check) to confirm that the image count over the disk
//      equals the count at its centre (no caustic crosses the disk there) and to sample
//      each image's extent,
//   2. predicts each point-source image's box with the network (offsets in units of the
//      image's linearised size sigma = rho / |1 - |kappa||),
//   3. gives every image its own box: network box joined with the sampled extent, a
//      safety margin (margin_frac of the extent plus the plain floors), merged where boxes
//      overlap; images whose point-source
//      magnification is below prune_ratio of the epoch's total get no grid and add their
//      point-source magnification instead,
// and the rays and clip retries run as in the plain path.  Epochs that fail a check fall
// back to the plain path; a drift gate against a second-order (source-size) estimate of
// the magnification sends suspicious results back too.
//
// image_extents_kernel also produces the training targets: run with n_check = n_limb it
// returns, for every centre image, the extent of its limb images as the plain step sees
// them.
#include "icrs_device.hpp"
#include "icrs_launch.hpp"

namespace icrs {
namespace {

constexpr int kEAMaxIterFP64 = 500;
constexpr int kEAMaxIterFP32 = 200;

// flags of an epoch (learned path)
constexpr uint32_t kLfCount = 1u;     // a limb point's image count differs from the centre's
constexpr uint32_t kLfEmpty = 2u;     // a centre image received no limb image
constexpr uint32_t kLfWide = 4u;      // an image spans half a turn or more
constexpr uint32_t kLfRoots = 8u;     // a root solve did not converge
constexpr uint32_t kLfVary = 16u;     // magnification varies strongly across the disk
constexpr uint32_t kLfGate = 32u;     // the drift gate rejected the learned result
constexpr uint32_t kLfClip = 64u;     // inside rays still touch a box edge after the retries

__device__ inline double wrap_pi(double a) {
  while (a > kPi) a -= 2.0 * kPi;
  while (a <= -kPi) a += 2.0 * kPi;
  return a;
}

// features of centre image z: log10 s, log10 q, w_c, log10 rho, z, parity, log10 mu,
// log10(sigma / rho) with sigma = rho / |1 - |kappa||
template <int N>
__device__ inline void image_features(const double* p, const Lens<N>& L, c64 wc, c64 z, float* f, double* sigma,
                                      double* mu) {
  const double k = sqrt(norm2(lens_kappa(L, z)));
  const double det = 1.0 - k * k;
  const double g = fmax(fabs(1.0 - k), 1e-12);
  *mu = 1.0 / fmax(fabs(det), 1e-300);
  *sigma = p[6] / g;
  f[0] = (float)log10(p[0]);
  f[1] = (float)log10(p[1]);
  f[2] = (float)wc.x;
  f[3] = (float)wc.y;
  f[4] = (float)log10(p[6]);
  f[5] = (float)z.x;
  f[6] = (float)z.y;
  f[7] = det > 0.0 ? 1.0f : -1.0f;
  f[8] = (float)log10(*mu);
  f[9] = (float)(-log10(g));
}

// Groups of P lanes (P a power of two >= max(n_pts, 16); G = blockDim / P groups per
// workgroup, one epoch per group): images of n_pts limb points assigned to the nearest
// centre image; per centre image the min/max of r and of theta relative to the image
// (ext [E][MI][4]); features [E][MI][10]; with tgt, the training targets
// ln(offset / sigma) of the four extents (offsets floored at 1e-3 sigma);
// a_ring[e] = mean point-source magnification over the limb points; flags[e].
constexpr int kMaxGroups = 4;

template <int N, typename T>
__global__ __launch_bounds__(256) void image_extents_kernel(Batch b, int n_pts, int P, const double* __restrict__ cimg,
                                                            const int32_t* __restrict__ cn, double* __restrict__ ext,
                                                            float* __restrict__ feat, float* __restrict__ tgt,
                                                            double* __restrict__ a_ring, uint32_t* __restrict__ flags,
                                                            const double* __restrict__ roots) {
  constexpr int MI = N * N + 1;
  __shared__ c64 cz[kMaxGroups][MI];
  __shared__ unsigned long long key[kMaxGroups][MI][4];
  __shared__ int cnt[kMaxGroups][MI];
  __shared__ uint32_t flag_sh[kMaxGroups];
  __shared__ double asum[kMaxGroups];
  const int G = blockDim.x / P;
  const int g = threadIdx.x / P, k = threadIdx.x % P;
  const int64_t e = (int64_t)blockIdx.x * G + g;
  const bool valid = e < b.n_epochs;
  const int nc = valid ? cn[e] : 0;
  const double* p = b.params + (valid ? (int64_t)b.epoch_event[e] * kParams : 0);
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = valid ? source_center(p, b.t[e]) : mk(0.0, 0.0);
  if (valid && k < MI) {
    cz[g][k] = mk(cimg[(e * kMaxSectors + k) * 2], cimg[(e * kMaxSectors + k) * 2 + 1]);
    key[g][k][0] = key[g][k][2] = ~0ull;
    key[g][k][1] = key[g][k][3] = 0ull;
    cnt[g][k] = 0;
  }
  if (valid && k == 0) {
    flag_sh[g] = (nc < 1) ? kLfEmpty : 0u;
    asum[g] = 0.0;
  }
  __syncthreads();
  if (valid && k < n_pts && nc >= 1) {
    double sp, cp;
    sincospi(2.0 * k / n_pts, &sp, &cp);
    const double rho = p[6];
    const c64 w = mk(wc.x + rho * cp, wc.y + rho * sp);
    c64 img[MI], warm[MI];
    if (roots)
      for (int j = 0; j < MI; ++j) warm[j] = mk(roots[(e * kMaxRoots + j) * 2], roots[(e * kMaxRoots + j) * 2 + 1]);
    int n = 0;
    const uint32_t st = find_images<N, T>(L, w, img, n, sizeof(T) == 8 ? kEAMaxIterFP64 : kEAMaxIterFP32,
                                          roots ? warm : nullptr);
    uint32_t f = st ? kLfRoots : 0u;
    if (n != nc) f |= kLfCount;
    double A = 0.0;
    for (int j = 0; j < n; ++j) {
      A += 1.0 / fabs(1.0 - norm2(lens_kappa(L, img[j])));
      int best = 0;
      double bd = 1e300;
      for (int i = 0; i < nc; ++i) {
        const double d = norm2(img[j] - cz[g][i]);
        if (d < bd) {
          bd = d;
          best = i;
        }
      }
      const double r = sqrt(norm2(img[j]));
      const double dth = wrap_pi(atan2(img[j].y, img[j].x) - atan2(cz[g][best].y, cz[g][best].x));
      atomicMin(&key[g][best][0], dkey(r));
      atomicMax(&key[g][best][1], dkey(r));
      atomicMin(&key[g][best][2], dkey(dth));
      atomicMax(&key[g][best][3], dkey(dth));
      atomicAdd(&cnt[g][best], 1);
    }
    if (f) atomicOr(&flag_sh[g], f);
    atomicAdd(&asum[g], A);
  }
  __syncthreads();
  if (valid && k < MI) {
    const int j = k;
    float fv[10];
    double o[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t f = 0u;
    if (j < nc) {
      double sigma, mu;
      image_features<N>(p, L, wc, cz[g][j], fv, &sigma, &mu);
      if (cnt[g][j] == 0) {
        f |= kLfEmpty;
      } else {
        o[0] = dkey_inv(key[g][j][0]);
        o[1] = dkey_inv(key[g][j][1]);
        o[2] = dkey_inv(key[g][j][2]);
        o[3] = dkey_inv(key[g][j][3]);
        if (o[3] - o[2] >= kPi) f |= kLfWide;
      }
      if (tgt) {
        const double rz = sqrt(norm2(cz[g][j]));
        const double off[4] = {rz - o[0], o[1] - rz, -rz * o[2], rz * o[3]};
        for (int q = 0; q < 4; ++q) tgt[(e * MI + j) * 4 + q] = (float)log(fmax(off[q], 1e-3 * sigma) / sigma);
      }
    } else {
      for (int q = 0; q < 10; ++q) fv[q] = 0.0f;
      if (tgt)
        for (int q = 0; q < 4; ++q) tgt[(e * MI + j) * 4 + q] = 0.0f;
    }
    for (int q = 0; q < 10; ++q) feat[(e * MI + j) * 10 + q] = fv[q];
    for (int q = 0; q < 4; ++q) ext[(e * MI + j) * 4 + q] = o[q];
    if (f) atomicOr(&flag_sh[g], f);
  }
  __syncthreads();
  if (valid && k == 0) {
    flags[e] = flag_sh[g];
    if (a_ring) a_ring[e] = asum[g] / n_pts;
  }
}

// Per epoch: learned boxes -> sectors.  y: network outputs [E][MI][4] (ln offset / sigma);
// epochs with flags or strongly varying magnification get no sectors and go to the
// fallback list; the others to the learned list.
template <int N>
__global__ void learned_sectors_kernel(Batch b, const double* __restrict__ cimg, const int32_t* __restrict__ cn,
                                       const double* __restrict__ a_c, const double* __restrict__ a_ring,
                                       const double* __restrict__ ext, const float* __restrict__ y, double log_safety,
                                       double margin_frac, double prune_ratio, double vary_max,
                                       uint32_t* __restrict__ flags,
                                       SectorBuf sec, double* __restrict__ add_mag, int32_t* __restrict__ lists,
                                       int32_t* __restrict__ counts, int32_t* __restrict__ n_pruned) {
  constexpr int MI = N * N + 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.n_epochs) return;
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const double rho = p[6];
  uint32_t f = flags[e];
  if (!f && fabs(a_ring[e] - a_c[e]) > vary_max * a_c[e]) f |= kLfVary;
  sec.nsec[e] = 0;
  add_mag[e] = 0.0;
  if (f) {
    flags[e] = f;
    lists[b.n_epochs + atomicAdd(&counts[1], 1)] = (int32_t)e;
    return;
  }
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = source_center(p, b.t[e]);
  const int nc = cn[e];
  Sector S[kMaxSectors];
  int ns = 0;
  double pruned = 0.0;
  int np = 0;
  for (int j = 0; j < nc; ++j) {
    const c64 z = mk(cimg[(e * kMaxSectors + j) * 2], cimg[(e * kMaxSectors + j) * 2 + 1]);
    float fv[10];
    double sigma, mu;
    image_features<N>(p, L, wc, z, fv, &sigma, &mu);
    if (mu < prune_ratio * a_c[e]) {
      pruned += mu;
      ++np;
      continue;
    }
    const double rz = sqrt(norm2(z)), thz = atan2(z.y, z.x);
    const float* yy = y + (e * MI + j) * 4;
    const double o0 = sigma * exp((double)yy[0] + log_safety), o1 = sigma * exp((double)yy[1] + log_safety);
    const double o2 = sigma * exp((double)yy[2] + log_safety), o3 = sigma * exp((double)yy[3] + log_safety);
    const double* x = ext + (e * MI + j) * 4;
    double r_lo = fmin(rz - o0, x[0]), r_hi = fmax(rz + o1, x[1]);
    double t_lo = fmin(-o2 / rz, x[2]), t_hi = fmax(o3 / rz, x[3]);
    r_lo = fmax(r_lo, 0.0);
    if (!(t_hi - t_lo < kPi) || !(r_hi > r_lo)) {
      f |= kLfWide;
      break;
    }
    // safety margin margin_frac x extent plus the plain floors (rho/100 in r, rho/(100 r_mid) in theta)
    const double mr = margin_frac * (r_hi - r_lo) + rho / 100.0;
    const double mt = margin_frac * (t_hi - t_lo) + rho / (50.0 * (r_lo + r_hi));
    Sector sc{fmax(r_lo - mr, 0.0), r_hi + mr, thz + t_lo - mt, thz + t_hi + mt, 0};
    normalise_theta(sc);
    S[ns++] = sc;
  }
  if (f) {
    flags[e] = f;
    lists[b.n_epochs + atomicAdd(&counts[1], 1)] = (int32_t)e;
    return;
  }
  merge_to_fixpoint(S, ns);
  sort_sectors(S, ns);
  for (int s = 0; s < ns; ++s) {
    double* g = sec.sectors + (e * kMaxSectors + s) * 4;
    g[0] = S[s].r_lo;
    g[1] = S[s].r_hi;
    g[2] = S[s].th_lo;
    g[3] = S[s].th_hi;
    sec.periodic[e * kMaxSectors + s] = (uint8_t)S[s].periodic;
  }
  sec.nsec[e] = ns;
  add_mag[e] = pruned;
  if (np) atomicAdd(n_pruned, np);
  lists[atomicAdd(&counts[0], 1)] = (int32_t)e;
}

// Drift gate over the learned list: compare with A_c + w2 (A_ring - A_c), the source-size
// estimate from the centre and the limb ring (w2 = <r~^2> of the limb-darkened profile,
// (15 - 7u)/(10 (3 - u))), within gate_rel A_c plus gate_slack |A_ring - A_c| (the estimate's
// own error grows with that difference; 0 holds every epoch to gate_rel); reject clipped
// results too.  Rejected epochs are appended to
// the fallback list.
__global__ void learned_gate_kernel(Batch b, const int32_t* __restrict__ learned, const int32_t* __restrict__ n_learned,
                                    const double* __restrict__ a_c, const double* __restrict__ a_ring,
                                    const double* __restrict__ mag, uint32_t* __restrict__ status, double gate_rel,
                                    double gate_slack,
                                    uint32_t* __restrict__ flags, int32_t* __restrict__ lists,
                                    int32_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_learned) return;
  const int64_t e = learned[i];
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const double u = p[7];
  const double w2 = (15.0 - 7.0 * u) / (10.0 * (3.0 - u));
  const double dA = a_ring[e] - a_c[e];
  const double est = a_c[e] + w2 * dA;
  uint32_t f = 0u;
  if (status[e] & kStClip) f |= kLfClip;
  if (!(fabs(mag[e] - est) <= gate_rel * a_c[e] + gate_slack * fabs(dA))) f |= kLfGate;
  if (f) {
    flags[e] |= f;
    status[e] &= ~(kStClip | kStNan | kStLearned);
    lists[b.n_epochs + atomicAdd(&counts[1], 1)] = (int32_t)e;
    atomicAdd(&counts[3], 1);
  }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_image_extents(int n_lens, int root_fp32, int n_pts, const Batch& b, const double* cimg,
                                const int32_t* cn, double* ext, float* feat, float* tgt, double* a_ring,
                                uint32_t* flags, hipStream_t s, const double* roots) {
  if (b.n_epochs == 0) return hipSuccess;
  // group width: a power of two covering the points and the images (>= 16); small point
  // counts share a wave between several epochs
  int P = 16;
  while (P < n_pts) P <<= 1;
  const int bs = P >= 64 ? P : 64;
  const int G = bs / P;
  if (G > kMaxGroups || P > 256) return hipErrorInvalidValue;
  const dim3 g((unsigned)((b.n_epochs + G - 1) / G)), blk(bs);
  if (n_lens == 2) {
    if (root_fp32)
      hipLaunchKernelGGL((image_extents_kernel<2, float>), g, blk, 0, s, b, n_pts, P, cimg, cn, ext, feat, tgt,
                         a_ring, flags, roots);
    else
      hipLaunchKernelGGL((image_extents_kernel<2, double>), g, blk, 0, s, b, n_pts, P, cimg, cn, ext, feat, tgt,
                         a_ring, flags, roots);
  } else {
    if (root_fp32)
      hipLaunchKernelGGL((image_extents_kernel<3, float>), g, blk, 0, s, b, n_pts, P, cimg, cn, ext, feat, tgt,
                         a_ring, flags, roots);
    else
      hipLaunchKernelGGL((image_extents_kernel<3, double>), g, blk, 0, s, b, n_pts, P, cimg, cn, ext, feat, tgt,
                         a_ring, flags, roots);
  }
  return hipGetLastError();
}

hipError_t launch_learned_sectors(int n_lens, const Batch& b, const double* cimg, const int32_t* cn,
                                  const double* a_c, const double* a_ring, const double* ext, const float* y,
                                  double log_safety, double margin_frac, double prune_ratio, double vary_max,
                                  uint32_t* flags, const SectorBuf& sec, double* add_mag, int32_t* lists,
                                  int32_t* counts, int32_t* n_pruned, hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  const dim3 g(blocks_for(b.n_epochs, 64)), blk(64);
  if (n_lens == 2)
    hipLaunchKernelGGL((learned_sectors_kernel<2>), g, blk, 0, s, b, cimg, cn, a_c, a_ring, ext, y, log_safety,
                       margin_frac, prune_ratio, vary_max, flags, sec, add_mag, lists, counts, n_pruned);
  else
    hipLaunchKernelGGL((learned_sectors_kernel<3>), g, blk, 0, s, b, cimg, cn, a_c, a_ring, ext, y, log_safety,
                       margin_frac, prune_ratio, vary_max, flags, sec, add_mag, lists, counts, n_pruned);
  return hipGetLastError();
}

hipError_t launch_learned_gate(const Batch& b, const int32_t* learned, const int32_t* n_learned, int64_t n_max,
                               const double* a_c, const double* a_ring, const double* mag, uint32_t* status,
                               double gate_rel, double gate_slack, uint32_t* flags, int32_t* lists,
                               int32_t* counts, hipStream_t s) {
  if (n_max == 0) return hipSuccess;
  hipLaunchKernelGGL(learned_gate_kernel, dim3(blocks_for(n_max, 256)), dim3(256), 0, s, b, learned, n_learned, a_c,
                     a_ring, mag, status, gate_rel, gate_slack, flags, lists, counts);
  return hipGetLastError();
}

}  // namespace icrs
