// icrs_prep.hip -- image finding and sector construction (Secs. 2.1, 3.1, 3.2).
//
// limb_sectors_kernel: one workgroup per epoch, one lane per source-limb point.  Each lane
// builds the lens polynomial of its limb point, finds its roots by Ehrlich-Aberth (FP64, or
// FP32 followed by an FP64 polish on the lens equation), validates them, and stages the
// image-limb points (r, theta) in LDS.  The workgroup then bins them in r and theta with
// LDS histograms, forms the candidate (r-run x theta-run) boxes with LDS atomic min/max,
// and lane 0 applies margins, merges, caps and sorts the few resulting sectors.
//
// centre_images_kernel: one lane per epoch, images of the source centre and the
// point-source magnification of eq. amp_point.
#include <algorithm>

#include "icrs_device.hpp"
#include "icrs_launch.hpp"

namespace icrs {

namespace {

constexpr int kEAMaxIterFP64 = 500;
constexpr int kEAMaxIterFP32 = 200;

__global__ void epoch_event_kernel(const int64_t* __restrict__ off, int64_t n_events, int64_t n_epochs,
                                   int32_t* __restrict__ ev) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_epochs) return;
  // largest i with off[i] <= e (offsets validated on the host: sorted, off[0] = 0)
  int64_t lo = 0, hi = n_events - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  ev[e] = (int32_t)lo;
}

template <int N, typename T>
__global__ __launch_bounds__(256) void centre_images_kernel(Batch b, double* __restrict__ images,
                                                            int32_t* __restrict__ n_images, double* __restrict__ a_ps,
                                                            uint32_t* __restrict__ status, double* __restrict__ roots) {
  constexpr int MI = N * N + 1;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.n_epochs) return;
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const Lens<N> L = make_lens<N>(p);
  const c64 wc = source_center(p, b.t[e]);
  c64 img[MI], zr[MI];
  int n = 0;
  const uint32_t st =
      find_images<N, T, true>(L, wc, img, n, sizeof(T) == 8 ? kEAMaxIterFP64 : kEAMaxIterFP32, nullptr, zr);
  if (roots)
    for (int j = 0; j < MI; ++j) {
      roots[(e * kMaxRoots + j) * 2 + 0] = zr[j].x;
      roots[(e * kMaxRoots + j) * 2 + 1] = zr[j].y;
    }
  double A = 0.0;
  for (int j = 0; j < n; ++j) A += 1.0 / fabs(1.0 - norm2(lens_kappa(L, img[j])));
  if (a_ps) a_ps[e] = A;
  if (n_images) n_images[e] = n;
  if (images)
    for (int j = 0; j < 10; ++j) {
      images[(e * 10 + j) * 2 + 0] = (j < n) ? img[j].x : 0.0;
      images[(e * 10 + j) * 2 + 1] = (j < n) ? img[j].y : 0.0;
    }
  if (status) status[e] = st;
}

// four waves per SIMD for the binary lens (128 VGPRs): 23% faster than the three the
// registers alone allow; the triple lens keeps its registers
template <int N, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N == 2 ? 4 : 1))) void limb_sectors_kernel(
    Batch b, int n_limb, SectorBuf out, uint32_t* __restrict__ status, const int32_t* __restrict__ list,
    int64_t n_list, const int32_t* __restrict__ n_list_dev, const double* __restrict__ roots,
    int32_t* __restrict__ redo_list, int32_t* __restrict__ redo_count) {
  constexpr int MI = N * N + 1;  // images per source point at most
  constexpr int cap = 5 * (N - 1);
  extern __shared__ double pts[];  // [blockDim.x * MI] r, then [blockDim.x * MI] theta
  double* pr = pts;
  double* pth = pts + blockDim.x * MI;
  Sector* S = reinterpret_cast<Sector*>(pts);  // step 5's candidates reuse the point buffer
  __shared__ unsigned long long rmin_k, rmax_k;
  __shared__ int occ_t[kBinsTheta], occ_r[kBinsR];
  __shared__ int trun_of[kBinsTheta], rrun_of[kBinsR], trun_first[kMaxRunsTheta];
  __shared__ int n_tr, n_rr, full_ring;
  __shared__ unsigned long long ck[kMaxCand][4];
  __shared__ int ccount[kMaxCand];
  __shared__ uint32_t st_sh;

  const int tid = threadIdx.x;
  // one workgroup per list entry; with a device-side list length the grid covers its upper
  // bound and the workgroups past the end leave at once
  const int64_t li = blockIdx.x;
  if (li >= (n_list_dev ? (int64_t)(*n_list_dev) : n_list)) return;
  const int64_t e = list ? (int64_t)list[li] : li;
  const double* p = b.params + (int64_t)b.epoch_event[e] * kParams;
  const double rho = p[6];
  if (tid == 0) {
    rmin_k = ~0ull;
    rmax_k = 0ull;
    st_sh = 0u;
  }
  if (tid < kBinsTheta) occ_t[tid] = 0;
  if (tid < kBinsR) occ_r[tid] = 0;
  __syncthreads();

  // 1. images of limb point k = tid: w = w_c + rho e^{2 pi i k / N_limb}
  int n = 0;
  if (tid < n_limb) {
    const Lens<N> L = make_lens<N>(p);
    const c64 wc = source_center(p, b.t[e]);
    double sp, cp;
    sincospi(2.0 * tid / n_limb, &sp, &cp);
    const c64 w = mk(wc.x + rho * cp, wc.y + rho * sp);
    c64 img[MI], warm[MI];
    if (roots)
      for (int j = 0; j < MI; ++j) warm[j] = mk(roots[(e * kMaxRoots + j) * 2], roots[(e * kMaxRoots + j) * 2 + 1]);
    uint32_t st = find_images<N, T>(L, w, img, n, sizeof(T) == 8 ? kEAMaxIterFP64 : kEAMaxIterFP32,
                                    roots ? warm : nullptr);
    // a warm-started solve that ends with a forbidden image count or an unconverged root
    // (two iterates settled on one root of a cluster): the epoch is queued for a cold FP64
    // pass, which decides its sectors and its status bits
    if (redo_list && (st & (kStImgCount | kStRootNonconv))) {
      st &= ~(kStImgCount | kStRootNonconv);
      st |= kStRedo;
    }
    if (st) atomicOr(&st_sh, st);
    for (int j = 0; j < n; ++j) {
      const double r = hypot(img[j].x, img[j].y);
      pr[tid * MI + j] = r;
      pth[tid * MI + j] = atan2(img[j].y, img[j].x);
      atomicMin(&rmin_k, dkey(r));
      atomicMax(&rmax_k, dkey(r));
    }
  }
  __syncthreads();

  // 2. occupancy of 64 theta bins on (-pi, pi] and 32 r bins of width
  //    max((r_max - r_min)/32, 2 rho) from r_min
  const double rmin = dkey_inv(rmin_k), rmax = dkey_inv(rmax_k);
  const double wr = fmax((rmax - rmin) / kBinsR, 2.0 * rho);
  for (int j = 0; j < n; ++j) {
    occ_t[theta_bin(pth[tid * MI + j])] = 1;
    occ_r[r_bin(pr[tid * MI + j], rmin, wr)] = 1;
  }
  __syncthreads();

  // 3. runs of occupied bins joined across single empty bins (theta circular), by bit
  //    operations on the occupancy masks in the first wave (one lane per bin).  A bin joins a
  //    run when it is occupied or both its neighbours are (G); runs are the maximal stretches
  //    of G, numbered from the lowest-index start upwards; a stretch that wraps past bin 63
  //    is the last run.  G covering the whole circle is one full-ring run.
  if (tid < 64) {
    const uint64_t M = __ballot(occ_t[tid] != 0);
    const uint64_t G = M | (((M << 1) | (M >> 63)) & ((M >> 1) | (M << 63)));
    const int full = (M != 0ull && G == ~0ull) ? 1 : 0;
    const uint64_t S = full ? 1ull : G & ~((G << 1) | (G >> 63));  // run starts
    const int nt = __popcll(S);
    const uint64_t upto = (tid == 63) ? ~0ull : ((2ull << tid) - 1ull);  // bins 0..tid
    int tr = -1;
    if ((G >> tid) & 1ull) {
      const int c = __popcll(S & upto);
      tr = c > 0 ? c - 1 : nt - 1;
    }
    trun_of[tid] = tr;
    if ((S >> tid) & 1ull) trun_first[__popcll(S & (upto >> 1))] = tid;
    const uint32_t Mr = (uint32_t)__ballot(tid < kBinsR && occ_r[tid] != 0);
    const uint32_t Gr = Mr | ((Mr << 1) & (Mr >> 1));
    const uint32_t Sr = Gr & ~(Gr << 1);
    if (tid < kBinsR) {
      const uint32_t upr = (tid == 31) ? ~0u : ((2u << tid) - 1u);
      rrun_of[tid] = ((Gr >> tid) & 1u) ? __popc(Sr & upr) - 1 : -1;
    }
    if (tid == 0) {
      n_tr = nt;
      n_rr = __popc(Sr);
      full_ring = full;
    }
  }
  __syncthreads();
  const int nc = n_tr * n_rr;
  for (int c = tid; c < nc; c += blockDim.x) {
    ck[c][0] = ~0ull;
    ck[c][1] = 0ull;
    ck[c][2] = ~0ull;
    ck[c][3] = 0ull;
    ccount[c] = 0;
  }
  __syncthreads();

  // 4. candidate boxes: min/max of member r and theta (theta unwrapped inside its run)
  for (int j = 0; j < n; ++j) {
    const double r = pr[tid * MI + j], th = pth[tid * MI + j];
    const int tb = theta_bin(th), rb = r_bin(r, rmin, wr);
    const int tr = trun_of[tb], rr = rrun_of[rb];
    if (tr < 0 || rr < 0) continue;
    const int c = rr * n_tr + tr;
    const double thu = (tb >= trun_first[tr]) ? th : th + 2.0 * kPi;
    atomicMin(&ck[c][0], dkey(r));
    atomicMax(&ck[c][1], dkey(r));
    atomicMin(&ck[c][2], dkey(thu));
    atomicMax(&ck[c][3], dkey(thu));
    atomicAdd(&ccount[c], 1);
  }
  __syncthreads();

  // 5. margins, merge to a fixpoint, cap at 5(N-1), sort (lane 0; a handful of boxes)
  if (tid == 0) {
    uint32_t st = st_sh;
    if (st & kStRedo) {
      st &= ~kStRedo;
      redo_list[atomicAdd(redo_count, 1)] = (int32_t)e;
    }
    int ns = 0;
    for (int rr = 0; rr < n_rr; ++rr)
      for (int tr = 0; tr < n_tr; ++tr) {
        const int c = rr * n_tr + tr;
        if (ccount[c] == 0) continue;
        S[ns++] = candidate_to_sector(dkey_inv(ck[c][0]), dkey_inv(ck[c][1]), dkey_inv(ck[c][2]),
                                      dkey_inv(ck[c][3]), full_ring, rho);
      }
    merge_to_fixpoint(S, ns);
    while (ns > cap) {
      st |= kStCapOverflow;
      int bi = 0, bj = 1;
      double best = 1e300;
      for (int i = 0; i < ns; ++i)
        for (int j = i + 1; j < ns; ++j) {
          const double a = sector_area(sector_union(S[i], S[j]));
          if (a < best) {
            best = a;
            bi = i;
            bj = j;
          }
        }
      S[bi] = sector_union(S[bi], S[bj]);
      for (int m = bj; m + 1 < ns; ++m) S[m] = S[m + 1];
      --ns;
      merge_to_fixpoint(S, ns);
    }
    sort_sectors(S, ns);
    for (int s = 0; s < ns; ++s) {
      double* o = out.sectors + (e * kMaxSectors + s) * 4;
      o[0] = S[s].r_lo;
      o[1] = S[s].r_hi;
      o[2] = S[s].th_lo;
      o[3] = S[s].th_hi;
      out.periodic[e * kMaxSectors + s] = (uint8_t)S[s].periodic;
    }
    out.nsec[e] = ns;
    status[e] |= st;
  }
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_epoch_event(const Batch& b, int32_t* epoch_event, hipStream_t s) {
  if (b.n_epochs == 0) return hipSuccess;
  hipLaunchKernelGGL(epoch_event_kernel, dim3(blocks_for(b.n_epochs, 256)), dim3(256), 0, s, b.offsets, b.n_events,
                     b.n_epochs, epoch_event);
  return hipGetLastError();
}

hipError_t launch_centre_images(int n_lens, int root_fp32, const Batch& b, double* images, int32_t* n_images,
                                double* a_ps, uint32_t* status, hipStream_t s, double* roots) {
  if (b.n_epochs == 0) return hipSuccess;
  const dim3 g(blocks_for(b.n_epochs, 64)), blk(64);
  if (n_lens == 2) {
    if (root_fp32)
      hipLaunchKernelGGL((centre_images_kernel<2, float>), g, blk, 0, s, b, images, n_images, a_ps, status, roots);
    else
      hipLaunchKernelGGL((centre_images_kernel<2, double>), g, blk, 0, s, b, images, n_images, a_ps, status, roots);
  } else {
    if (root_fp32)
      hipLaunchKernelGGL((centre_images_kernel<3, float>), g, blk, 0, s, b, images, n_images, a_ps, status, roots);
    else
      hipLaunchKernelGGL((centre_images_kernel<3, double>), g, blk, 0, s, b, images, n_images, a_ps, status, roots);
  }
  return hipGetLastError();
}

namespace {
template <int N, typename T>
void limb_launch(dim3 g, dim3 blk, size_t lds, hipStream_t s, const Batch& b, int n_limb, const SectorBuf& out,
                 uint32_t* status, const int32_t* list, int64_t n, const int32_t* n_list_dev, const double* roots,
                 int32_t* redo_list, int32_t* redo_count) {
  hipLaunchKernelGGL((limb_sectors_kernel<N, T>), g, blk, lds, s, b, n_limb, out, status, list, n, n_list_dev, roots,
                     redo_list, redo_count);
}
}  // namespace

hipError_t launch_limb_sectors(int n_lens, int root_fp32, int n_limb, const Batch& b, const SectorBuf& out,
                               uint32_t* status, hipStream_t s, const int32_t* list, int64_t n_list,
                               const int32_t* n_list_dev, const double* roots, int32_t* redo_list,
                               int32_t* redo_count) {
  const int64_t n = list ? n_list : b.n_epochs;
  if (n <= 0) return hipSuccess;
  if (roots && (!redo_list || !redo_count)) return hipErrorInvalidValue;
  const int bs = ((n_limb + 63) / 64) * 64;
  // one workgroup per epoch (n is the list's upper bound when its length is on the device)
  if (n > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g((unsigned)n), blk(bs);
  const size_t lds = std::max((size_t)bs * (n_lens * n_lens + 1) * 2 * sizeof(double), kMaxCand * sizeof(Sector));
  if (roots) {
    hipError_t e = launch_fill_i32(redo_count, 1, 0, s);
    if (e != hipSuccess) return e;
  }
  // warm-started pass (or the cold pass when no roots are given)
  if (n_lens == 2) {
    if (root_fp32)
      limb_launch<2, float>(g, blk, lds, s, b, n_limb, out, status, list, n, n_list_dev, roots, redo_list, redo_count);
    else
      limb_launch<2, double>(g, blk, lds, s, b, n_limb, out, status, list, n, n_list_dev, roots, redo_list, redo_count);
  } else {
    if (root_fp32)
      limb_launch<3, float>(g, blk, lds, s, b, n_limb, out, status, list, n, n_list_dev, roots, redo_list, redo_count);
    else
      limb_launch<3, double>(g, blk, lds, s, b, n_limb, out, status, list, n, n_list_dev, roots, redo_list, redo_count);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !roots) return e;
  // the epochs it queued, again from the Cauchy circle in FP64 (a handful per million); the
  // grid covers every epoch and the workgroups past the queue's end leave at once
  const dim3 g2((unsigned)n);
  if (n_lens == 2)
    limb_launch<2, double>(g2, blk, lds, s, b, n_limb, out, status, redo_list, n, redo_count, nullptr, nullptr,
                           nullptr);
  else
    limb_launch<3, double>(g2, blk, lds, s, b, n_limb, out, status, redo_list, n, redo_count, nullptr, nullptr,
                           nullptr);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace icrs
