// icrs_api.hip -- host side of the C ABI declared in include/icrs.h: argument checks,
// workspace carving, and the launch sequence of one call.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "../../include/icrs.h"
#include "icrs_launch.hpp"

struct icrs_handle {
  icrs_config cfg;
  hipStream_t stream;
  int profiling;
  hipEvent_t ev[16];
  icrs_profile prof;
  int64_t prep_events, prep_epochs;  // batch uploaded by icrs_prepare()
  const void* prep_ws;
};

namespace {

using icrs::Batch;
using icrs::RayWork;
using icrs::SectorBuf;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t params, offsets, epoch_event, sectors, periodic, nsec, partial, clip, list_a, list_b, fallback, retake,
      retake_fx, jac, roots, counters, total;
};

// Room for FP32 crossings retaken in FP64 (next to the edge rule's jump at delta_c): the
// benchmark workload lists 6 per epoch at 192 x 512 and 16 at 256 x 1024; a sector whose
// crossings do not fit is redone by the FP64 pass.
constexpr int64_t kRetakePerEpoch = 32;

Layout layout_for(int64_t n_events, int64_t n_epochs) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t E = (size_t)n_epochs, V = (size_t)n_events;
  // per-epoch blocks first (their offsets depend on n_epochs only), event blocks last
  L.sectors = take(E * ICRS_MAX_SECTORS * 4 * sizeof(double));
  L.periodic = take(E * ICRS_MAX_SECTORS);
  L.nsec = take(E * sizeof(int32_t));
  L.partial = take(E * ICRS_MAX_SECTORS * sizeof(double));
  L.clip = take(E * ICRS_MAX_SECTORS);
  L.epoch_event = take(E * sizeof(int32_t));
  L.list_a = take(E * sizeof(int32_t));
  L.list_b = take(E * sizeof(int32_t));
  L.fallback = take(E * ICRS_MAX_SECTORS * sizeof(int32_t));
  L.retake = take(E * kRetakePerEpoch * 2 * sizeof(int32_t));
  L.retake_fx = take(E * ICRS_MAX_SECTORS * sizeof(unsigned long long));
  L.jac = take(E * ICRS_N_PARAMS * sizeof(double));
  L.roots = take(E * 10 * 2 * sizeof(double));  // the source centre's polynomial roots
  L.counters = take(64);
  L.params = take(V * ICRS_N_PARAMS * sizeof(double));
  L.offsets = take((V + 1) * sizeof(int64_t));
  L.total = o;
  return L;
}

// Extra blocks of the learned path, after the plain layout.
struct LearnedLayout {
  size_t cimg, cn, a_c, a_ring, add, flags, ext, feat, y, lists, counts, total;
};

LearnedLayout learned_layout(int n_lens, int64_t n_events, int64_t n_epochs) {
  LearnedLayout L;
  size_t o = layout_for(n_events, n_epochs).total;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t E = (size_t)n_epochs, MI = (size_t)(n_lens * n_lens + 1);
  L.cimg = take(E * ICRS_MAX_SECTORS * 2 * sizeof(double));
  L.cn = take(E * sizeof(int32_t));
  L.a_c = take(E * sizeof(double));
  L.a_ring = take(E * sizeof(double));
  L.add = take(E * sizeof(double));
  L.flags = take(E * sizeof(uint32_t));
  L.ext = take(E * MI * 4 * sizeof(double));
  L.feat = take(E * MI * 10 * sizeof(float));
  L.y = take(E * MI * 4 * sizeof(float));
  L.lists = take(2 * E * sizeof(int32_t));
  L.counts = take(64);
  L.total = o;
  return L;
}

bool config_ok(const icrs_config* c) {
  if (!c || c->abi_version != ICRS_ABI_VERSION) return false;
  if (c->n_lens != 2 && c->n_lens != 3) return false;
  if (c->n_limb < 8 || c->n_limb > 256) return false;
  if (c->n_r < 4 || c->n_r > 4096) return false;
  if (c->n_theta < 64 || c->n_theta > 1024) return false;
  if (c->ray_precision != ICRS_FP64 && c->ray_precision != ICRS_FP32) return false;
  if (c->root_precision != ICRS_FP64 && c->root_precision != ICRS_FP32) return false;
  if (c->max_retries < 0 || c->max_retries > 4) return false;
  if (!(c->delta_c >= 0.0 && c->delta_c <= 1.0)) return false;
  return true;
}

bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(p[i])) return false;
  return true;
}

// host checks of the event parameters and the CSR offsets
bool events_ok(const icrs_config& c, int64_t n_events, const double* params, const int64_t* off, int64_t n_epochs) {
  if (n_events < 0 || n_epochs < 0) return false;
  // FP64-pass work items pack (epoch, sector) as the int32 16 e + slot
  if (n_epochs > ICRS_MAX_EPOCHS) return false;
  if (n_events > 0x7fffffffLL) return false;
  if (n_events > 0 && (!params || !off)) return false;
  if (n_events == 0) return n_epochs == 0;
  if (off[0] != 0 || off[n_events] != n_epochs) return false;
  for (int64_t i = 0; i < n_events; ++i)
    if (off[i + 1] < off[i]) return false;
  for (int64_t i = 0; i < n_events; ++i) {
    const double* p = params + i * ICRS_N_PARAMS;
    if (!finite_all(p, c.n_lens == 3 ? ICRS_N_PARAMS : 8)) return false;
    if (!(p[0] > 0.0 && p[1] > 0.0 && p[5] > 0.0)) return false;
    if (!(p[6] > 0.0 && p[6] <= 1.0)) return false;
    if (!(p[7] >= 0.0 && p[7] < 1.0)) return false;
    if (c.n_lens == 3 && !(p[8] > 0.0 && p[9] >= 0.0)) return false;
  }
  return true;
}

icrs_status hip_status(hipError_t e) { return e == hipSuccess ? ICRS_OK : ICRS_EHIP; }

// Event pair around one launch when profiling is on; elapsed time is added to *acc after
// the stream has been waited for (Timer::flush).
struct Timer {
  icrs_handle* h;
  int n = 0;
  double* acc[8];
  double* acc2[8];
  explicit Timer(icrs_handle* hh) : h(hh) {}
  hipError_t begin() {
    if (!h->profiling || n >= 8) return hipSuccess;
    return hipEventRecord(h->ev[2 * n], h->stream);
  }
  hipError_t end(double* into, double* also = nullptr) {
    if (!h->profiling || n >= 8) return hipSuccess;
    acc[n] = into;
    acc2[n] = also;
    return hipEventRecord(h->ev[2 * n++ + 1], h->stream);
  }
  hipError_t flush() {
    if (!h->profiling) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->stream);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]);
      *acc[i] += ms;
      if (acc2[i]) *acc2[i] += ms;
    }
    n = 0;
    return e;
  }
};

#define ICRS_TRY(expr)                       \
  do {                                       \
    const hipError_t err_ = (expr);          \
    if (err_ != hipSuccess) return ICRS_EHIP; \
  } while (0)

struct Views {
  Batch b;
  SectorBuf sec;
  double* partial;
  uint8_t* clip;
  int32_t* list_a;
  int32_t* list_b;
  int32_t* fallback;
  int32_t* retake;
  unsigned long long* retake_fx;
  int64_t retake_cap;
  double* jac;
  double* roots;       // [n_epochs][10] complex: roots of the centre's lens polynomial
  int32_t* counters;   // [0], [1] retry list counts, [2] cold-redo list count, [4] FP64 fallback
                       // count, [6..7] int64 retake count, [8..9] int64 sector passes, [12..13] int64
                       // work queue
};

icrs_status prepare(icrs_handle* h, int64_t n_events, const double* params, const int64_t* off, int64_t n_epochs,
                    const double* t, void* ws, size_t ws_bytes, Views* v) {
  const Layout L = layout_for(n_events, n_epochs);
  if (!ws || ws_bytes < L.total) return ws ? ICRS_ENOMEM : ICRS_EINVAL;
  if (((uintptr_t)ws & (kAlign - 1)) != 0) return ICRS_EINVAL;
  char* base = (char*)ws;
  v->b.params = (const double*)(base + L.params);
  v->b.offsets = (const int64_t*)(base + L.offsets);
  v->b.epoch_event = (const int32_t*)(base + L.epoch_event);
  v->b.t = t;
  v->b.n_events = n_events;
  v->b.n_epochs = n_epochs;
  v->sec.sectors = (double*)(base + L.sectors);
  v->sec.periodic = (uint8_t*)(base + L.periodic);
  v->sec.nsec = (int32_t*)(base + L.nsec);
  v->partial = (double*)(base + L.partial);
  v->clip = (uint8_t*)(base + L.clip);
  v->list_a = (int32_t*)(base + L.list_a);
  v->list_b = (int32_t*)(base + L.list_b);
  v->fallback = (int32_t*)(base + L.fallback);
  v->retake = (int32_t*)(base + L.retake);
  v->retake_fx = (unsigned long long*)(base + L.retake_fx);
  v->retake_cap = n_epochs * kRetakePerEpoch;
  v->jac = (double*)(base + L.jac);
  v->roots = (double*)(base + L.roots);
  v->counters = (int32_t*)(base + L.counters);
  if (n_events == 0) return ICRS_OK;
  ICRS_TRY(hipMemcpyAsync(base + L.params, params, (size_t)n_events * ICRS_N_PARAMS * sizeof(double),
                          hipMemcpyHostToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(base + L.offsets, off, (size_t)(n_events + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                          h->stream));
  ICRS_TRY(icrs::launch_epoch_event(v->b, (int32_t*)(base + L.epoch_event), h->stream));
  return ICRS_OK;
}

// Views of the batch that icrs_prepare() uploaded into workspace (no host memory is read).
Views prepared_views(const icrs_handle* h, const double* t, void* workspace) {
  const Layout L = layout_for(h->prep_events, h->prep_epochs);
  char* base = (char*)workspace;
  Views v;
  v.b.params = (const double*)(base + L.params);
  v.b.offsets = (const int64_t*)(base + L.offsets);
  v.b.epoch_event = (const int32_t*)(base + L.epoch_event);
  v.b.t = t;
  v.b.n_events = h->prep_events;
  v.b.n_epochs = h->prep_epochs;
  v.sec.sectors = (double*)(base + L.sectors);
  v.sec.periodic = (uint8_t*)(base + L.periodic);
  v.sec.nsec = (int32_t*)(base + L.nsec);
  v.partial = (double*)(base + L.partial);
  v.clip = (uint8_t*)(base + L.clip);
  v.list_a = (int32_t*)(base + L.list_a);
  v.list_b = (int32_t*)(base + L.list_b);
  v.fallback = (int32_t*)(base + L.fallback);
  v.retake = (int32_t*)(base + L.retake);
  v.retake_fx = (unsigned long long*)(base + L.retake_fx);
  v.retake_cap = h->prep_epochs * kRetakePerEpoch;
  v.jac = (double*)(base + L.jac);
  v.roots = (double*)(base + L.roots);
  v.counters = (int32_t*)(base + L.counters);
  return v;
}

// Which epochs and grid one ray call covers: all epochs on the handle's grid by default.
struct RaySet {
  const int32_t* list = nullptr;   // epochs (device), or all when null
  int64_t n = -1;                  // list length, or an upper bound of it when n_dev is set
  const int32_t* n_dev = nullptr;  // device-side list length (read by the kernels only)
  int n_r = 0, n_theta = 0;        // grid; 0 = the handle's
  const double* add_mag = nullptr;
};

// Rays + finalize with up to max_retries widening passes, with no host synchronisation:
// every retry pass is enqueued and finds its work list size on the device (an empty pass
// ends at once).  With profiling on, kernel timings and the main pass's sector count are
// read back after the first pass (the only host waits, and only then).
icrs_status run_rays(icrs_handle* h, const Views& v, int max_retries, double* mag, uint32_t* status,
                     uint32_t extra_status, const RaySet& rs = RaySet{}) {
  icrs_config c = h->cfg;
  if (rs.n_r) c.n_r = rs.n_r;
  if (rs.n_theta) c.n_theta = rs.n_theta;
  RayWork w;
  w.list = rs.list;
  w.n = rs.list ? rs.n : v.b.n_epochs;
  w.n_dev = rs.n_dev;
  if (w.n <= 0) return ICRS_OK;
  const int64_t n_bound = w.n;
  int32_t* lists[2] = {v.list_a, v.list_b};
  int32_t* counts[2] = {v.counters + 0, v.counters + 1};
  unsigned long long* passes = (unsigned long long*)(v.counters + 8);
  icrs::RetakeBuf rb;
  rb.items = v.retake;
  rb.n = (unsigned long long*)(v.counters + 6);
  rb.cap = v.retake_cap;
  rb.fx = v.retake_fx;
  const bool learned = (extra_status & ICRS_ST_LEARNED) != 0;
  if (h->profiling) ICRS_TRY(icrs::launch_fill_i32(v.counters + 8, 2, 0, h->stream));
  Timer tm(h);
  for (int attempt = 0; attempt <= max_retries; ++attempt) {
    // stage 0: the main pass (timed on its own for the first attempt); stage 1: FP64 pass
    // over the sectors the FP32 main pass listed
    for (int stage = 0; stage < 2; ++stage) {
      ICRS_TRY(tm.begin());
      ICRS_TRY(icrs::launch_rays(c.n_lens, c.ray_precision, stage, v.b, v.sec, w, c.n_r, c.n_theta, c.delta_c,
                                 v.partial, v.clip, (unsigned long long*)(v.counters + 12), v.fallback,
                                 v.counters + 4, rb, h->stream));
      double* also = nullptr;
      if (attempt == 0 && stage == 0) also = learned ? &h->prof.ms_rays_learned : &h->prof.ms_rays_main;
      ICRS_TRY(tm.end(&h->prof.ms_rays, also));
    }
    h->prof.n_rays_launches += 1;
    int32_t* nxt = lists[attempt & 1];
    int32_t* ncount = counts[attempt & 1];
    ICRS_TRY(icrs::launch_fill_i32(ncount, 1, 0, h->stream));
    ICRS_TRY(tm.begin());
    ICRS_TRY(icrs::launch_finalize(v.b, v.sec, w, v.partial, v.clip, attempt, max_retries, nxt, ncount, mag, status,
                                   extra_status, h->profiling ? passes : nullptr, h->stream, rs.add_mag));
    ICRS_TRY(tm.end(&h->prof.ms_finalize));
    ICRS_TRY(tm.flush());
    if (h->profiling && attempt == 0) {
      // sectors the main pass shot: all first-attempt sectors less those sent to FP64
      unsigned long long np = 0;
      int32_t nfb = 0;
      ICRS_TRY(hipMemcpyAsync(&np, passes, sizeof(np), hipMemcpyDeviceToHost, h->stream));
      ICRS_TRY(hipMemcpyAsync(&nfb, v.counters + 4, sizeof(nfb), hipMemcpyDeviceToHost, h->stream));
      ICRS_TRY(hipStreamSynchronize(h->stream));
      const int64_t main = (int64_t)np - (c.ray_precision == ICRS_FP32 ? (int64_t)nfb : 0);
      if (learned) {
        h->prof.n_learned_launches += 1;
        h->prof.n_learned_sectors += main;
        h->prof.n_learned_rays += main * (int64_t)c.n_r * c.n_theta;
      } else {
        h->prof.n_main_launches += 1;
        h->prof.n_main_sectors += main;
        h->prof.n_main_rays += main * (int64_t)c.n_r * c.n_theta;
      }
    }
    w = RayWork{};
    w.list = nxt;
    w.n = n_bound;
    w.n_dev = ncount;
  }
  if (h->profiling) {
    unsigned long long np = 0;
    int64_t ne = rs.list ? rs.n : v.b.n_epochs;
    int32_t nd = 0;
    ICRS_TRY(hipMemcpyAsync(&np, passes, sizeof(np), hipMemcpyDeviceToHost, h->stream));
    if (rs.n_dev) ICRS_TRY(hipMemcpyAsync(&nd, rs.n_dev, sizeof(nd), hipMemcpyDeviceToHost, h->stream));
    ICRS_TRY(hipStreamSynchronize(h->stream));
    if (rs.n_dev) ne = nd;
    h->prof.n_sector_passes += (int64_t)np;
    h->prof.n_epochs += ne;
    h->prof.n_calls += 1;
  }
  return ICRS_OK;
}

// The plain path: centre images (the limb solves' warm start), limb sectors, rays.
icrs_status run_plain(icrs_handle* h, const Views& v, double* mag, uint32_t* status) {
  const icrs_config& c = h->cfg;
  const int fp32_roots = c.root_precision == ICRS_FP32;
  Timer tm(h);
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_centre_images(c.n_lens, fp32_roots, v.b, nullptr, nullptr, nullptr, status, h->stream,
                                      v.roots));
  ICRS_TRY(tm.end(&h->prof.ms_centre));
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_limb_sectors(c.n_lens, fp32_roots, c.n_limb, v.b, v.sec, status, h->stream, nullptr, 0,
                                     nullptr, v.roots, v.list_b, v.counters + 2));
  ICRS_TRY(tm.end(&h->prof.ms_limb_sectors));
  ICRS_TRY(tm.flush());
  return run_rays(h, v, c.max_retries, mag, status, 0u);
}

bool learned_config_ok(const icrs_learned_config* lc) {
  return lc && lc->n_check >= 8 && lc->n_check <= 64 && lc->n_r >= 4 && lc->n_r <= 4096 && lc->n_theta >= 64 &&
         lc->n_theta <= 1024 && lc->prune_ratio >= 0.0 && lc->prune_ratio < 0.1 && lc->vary_max > 0.0 &&
         lc->gate_rel > 0.0 && fabs(lc->log_safety) < 10.0 && lc->margin_frac >= 0.0 && lc->margin_frac <= 1.0 &&
         lc->gate_slack >= 0.0 && lc->gate_slack <= 10.0;
}

// The learned path on an uploaded batch (views v over workspace): no host memory is read
// and, without stats and profiling, nothing waits for the stream.
icrs_status run_learned(icrs_handle* h, const Views& v, const icrs_learned_config* lc, const uint16_t* packed,
                        const float* mlp_params, const float* norm, double* mag, uint32_t* status,
                        icrs_learned_stats* stats, void* workspace) {
  if (stats) memset(stats, 0, sizeof(*stats));
  const int64_t n_epochs = v.b.n_epochs;
  if (n_epochs == 0) return ICRS_OK;
  const LearnedLayout LL = learned_layout(h->cfg.n_lens, v.b.n_events, n_epochs);
  char* base = (char*)workspace;
  const icrs_config& c = h->cfg;
  const int fp32_roots = c.root_precision == ICRS_FP32;
  const int MI = c.n_lens * c.n_lens + 1;
  double* cimg = (double*)(base + LL.cimg);
  int32_t* cn = (int32_t*)(base + LL.cn);
  double* a_c = (double*)(base + LL.a_c);
  double* a_ring = (double*)(base + LL.a_ring);
  double* add = (double*)(base + LL.add);
  uint32_t* flags = (uint32_t*)(base + LL.flags);
  double* ext = (double*)(base + LL.ext);
  float* feat = (float*)(base + LL.feat);
  float* y = (float*)(base + LL.y);
  int32_t* lists = (int32_t*)(base + LL.lists);
  int32_t* counts = (int32_t*)(base + LL.counts);
  Timer tm(h);
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_centre_images(c.n_lens, fp32_roots, v.b, cimg, cn, a_c, status, h->stream, v.roots));
  ICRS_TRY(tm.end(&h->prof.ms_centre));
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_image_extents(c.n_lens, fp32_roots, lc->n_check, v.b, cimg, cn, ext, feat, nullptr, a_ring,
                                      flags, h->stream, v.roots));
  ICRS_TRY(icrs::mlp::launch_forward(packed, mlp_params, norm, n_epochs * MI, feat, y, h->stream));
  ICRS_TRY(icrs::launch_fill_i32(counts, 4, 0, h->stream));
  ICRS_TRY(icrs::launch_learned_sectors(c.n_lens, v.b, cimg, cn, a_c, a_ring, ext, y, lc->log_safety,
                                        lc->margin_frac, lc->prune_ratio, lc->vary_max, flags, v.sec, add, lists,
                                        counts, counts + 2, h->stream));
  ICRS_TRY(tm.end(&h->prof.ms_limb_sectors));
  ICRS_TRY(tm.flush());
  // learned epochs: counts[0] of them at lists[0..]; fallback epochs at lists[E..], counts[1]
  RaySet rs;
  rs.list = lists;
  rs.n = n_epochs;
  rs.n_dev = counts;
  rs.n_r = lc->n_r;
  rs.n_theta = lc->n_theta;
  rs.add_mag = add;
  icrs_status st = run_rays(h, v, c.max_retries, mag, status, ICRS_ST_LEARNED, rs);
  if (st != ICRS_OK) return st;
  // the gate appends the learned epochs it rejects to the fallback list (and counts them
  // in counts[3])
  ICRS_TRY(icrs::launch_learned_gate(v.b, lists, counts, n_epochs, a_c, a_ring, mag, status, lc->gate_rel,
                                     lc->gate_slack, flags,
                                     lists, counts, h->stream));
  const int32_t* fb = lists + n_epochs;
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_limb_sectors(c.n_lens, fp32_roots, c.n_limb, v.b, v.sec, status, h->stream, fb, n_epochs,
                                     counts + 1, v.roots, v.list_b, v.counters + 2));
  ICRS_TRY(tm.end(&h->prof.ms_limb_sectors));
  ICRS_TRY(tm.flush());
  RaySet fs;
  fs.list = fb;
  fs.n = n_epochs;
  fs.n_dev = counts + 1;
  st = run_rays(h, v, c.max_retries, mag, status, ICRS_ST_FALLBACK, fs);
  if (st != ICRS_OK) return st;
  if (stats) {
    // the only host wait of this entry point, and only when statistics are asked for
    int32_t cnt[4] = {0, 0, 0, 0};
    ICRS_TRY(hipMemcpyAsync(cnt, counts, sizeof(cnt), hipMemcpyDeviceToHost, h->stream));
    ICRS_TRY(hipStreamSynchronize(h->stream));
    stats->n_epochs = n_epochs;
    stats->n_fallback = cnt[1];
    stats->n_gate_rejected = cnt[3];
    stats->n_learned = cnt[0] - stats->n_gate_rejected;
    stats->n_pruned_images = cnt[2];
  }
  return ICRS_OK;
}


// Device scratch of icrs_magnification_noalloc: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device memory: its device
// address is taken once per device with hipGetSymbolAddress (with that device current) and
// only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[ICRS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (resolved on the first call on that device).
hipError_t scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr || ((uintptr_t)ptr & (kAlign - 1)) != 0) return hipErrorInvalidValue;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

void icrs_default_config(icrs_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->abi_version = ICRS_ABI_VERSION;
  cfg->n_lens = 2;
  cfg->n_limb = 64;
  cfg->n_r = 64;
  cfg->n_theta = 256;
  cfg->ray_precision = ICRS_FP64;
  cfg->root_precision = ICRS_FP64;
  cfg->max_retries = 2;
  cfg->delta_c = 0.1;
}

icrs_status icrs_create(const icrs_config* cfg, void* hip_stream, icrs_handle** out) {
  if (!out || !config_ok(cfg)) return ICRS_EINVAL;
  icrs_handle* h = new (std::nothrow) icrs_handle;
  if (!h) return ICRS_ENOMEM;
  h->cfg = *cfg;
  h->stream = (hipStream_t)hip_stream;
  h->profiling = 0;
  memset(&h->prof, 0, sizeof(h->prof));
  h->prep_events = h->prep_epochs = 0;
  h->prep_ws = nullptr;
  for (auto& e : h->ev) e = nullptr;
  *out = h;
  return ICRS_OK;
}

void icrs_destroy(icrs_handle* h) {
  if (!h) return;
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

icrs_status icrs_set_profiling(icrs_handle* h, int on) {
  if (!h) return ICRS_EINVAL;
  if (on && !h->ev[0])
    for (auto& e : h->ev) ICRS_TRY(hipEventCreate(&e));
  h->profiling = on ? 1 : 0;
  return ICRS_OK;
}

icrs_status icrs_get_profile(icrs_handle* h, icrs_profile* out, int reset) {
  if (!h || !out) return ICRS_EINVAL;
  *out = h->prof;
  if (reset) memset(&h->prof, 0, sizeof(h->prof));
  return ICRS_OK;
}

size_t icrs_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs) {
  (void)h;
  if (n_events < 0 || n_epochs < 0) return 0;
  return layout_for(n_events, n_epochs).total;
}

icrs_status icrs_magnification(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                               int64_t n_epochs, const double* t, double* mag, uint32_t* status, void* workspace,
                               size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !mag || !status)) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  return run_plain(h, v, mag, status);
}

icrs_status icrs_magnification_noalloc(icrs_handle* h, int64_t n_events, const double* params,
                                       const int64_t* epoch_offsets, int64_t n_epochs, const double* t, double* mag,
                                       uint32_t* status) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !mag || !status)) return ICRS_EINVAL;
  const size_t need = layout_for(n_events, n_epochs).total;
  if (need > (size_t)ICRS_NOALLOC_SCRATCH_BYTES) return ICRS_ENOMEM;
  if (n_epochs == 0) return ICRS_OK;
  void* ws = nullptr;
  ICRS_TRY(scratch_for_current_device(&ws));
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, ws, need, &v);
  if (ps != ICRS_OK) return ps;
  // no host waits and no event timers here
  const int prof = h->profiling;
  h->profiling = 0;
  const icrs_status st = run_plain(h, v, mag, status);
  h->profiling = prof;
  return st;
}

icrs_status icrs_prepare(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                         int64_t n_epochs, void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, nullptr, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK) return ps;
  h->prep_events = n_events;
  h->prep_epochs = n_epochs;
  h->prep_ws = workspace;
  return ICRS_OK;
}

icrs_status icrs_run(icrs_handle* h, const double* t, double* mag, uint32_t* status, void* workspace,
                     size_t workspace_bytes) {
  if (!h || !workspace || workspace != h->prep_ws) return ICRS_EINVAL;
  if (h->prep_epochs > 0 && (!t || !mag || !status)) return ICRS_EINVAL;
  const Layout L = layout_for(h->prep_events, h->prep_epochs);
  if (workspace_bytes < L.total) return ICRS_ENOMEM;
  if (h->prep_epochs == 0) return ICRS_OK;
  const Views v = prepared_views(h, t, workspace);
  // no host waits: the profiling timers (which wait for the stream) are off here
  const int prof = h->profiling;
  h->profiling = 0;
  const icrs_status st = run_plain(h, v, mag, status);
  h->profiling = prof;
  return st;
}

icrs_status icrs_magnification_given(icrs_handle* h, int64_t n_events, const double* params,
                                     const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                     const double* sectors, const uint8_t* periodic, const int32_t* n_sectors,
                                     double* mag, uint32_t* status, void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !mag || !status || !sectors || !periodic || !n_sectors)) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  const size_t E = (size_t)n_epochs;
  ICRS_TRY(hipMemcpyAsync(v.sec.sectors, sectors, E * ICRS_MAX_SECTORS * 4 * sizeof(double),
                          hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.periodic, periodic, E * ICRS_MAX_SECTORS, hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.nsec, n_sectors, E * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(icrs::launch_fill_u32(status, n_epochs, 0u, h->stream));
  return run_rays(h, v, 0, mag, status, ICRS_ST_GIVEN);
}

icrs_status icrs_magnification_vjp(icrs_handle* h, int64_t n_events, const double* params,
                                   const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                   const double* sectors, const uint8_t* periodic, const int32_t* n_sectors,
                                   const double* cotangent, double* grad, double* jac, double* mag, void* workspace,
                                   size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !sectors || !periodic || !n_sectors)) return ICRS_EINVAL;
  if ((grad && !cotangent) || (!grad && !jac && !mag)) return ICRS_EINVAL;
  if (h->cfg.n_theta > 1024) return ICRS_EUNSUPPORTED;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  const size_t E = (size_t)n_epochs;
  ICRS_TRY(hipMemcpyAsync(v.sec.sectors, sectors, E * ICRS_MAX_SECTORS * 4 * sizeof(double),
                          hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.periodic, periodic, E * ICRS_MAX_SECTORS, hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.nsec, n_sectors, E * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  double* J = jac ? jac : v.jac;
  return hip_status(icrs::launch_adjoint(h->cfg.n_lens, v.b, v.sec, h->cfg.n_r, h->cfg.n_theta, h->cfg.delta_c,
                                         cotangent, J, grad, mag, (unsigned long long*)(v.counters + 12),
                                         h->stream));
}

icrs_status icrs_get_sectors(icrs_handle* h, const void* workspace, int64_t n_epochs, double* sectors,
                             uint8_t* periodic, int32_t* n_sectors) {
  if (!h || !workspace || n_epochs < 0) return ICRS_EINVAL;
  if (n_epochs == 0) return ICRS_OK;
  if (!sectors || !periodic || !n_sectors) return ICRS_EINVAL;
  const Layout L = layout_for(0, n_epochs);
  const char* base = (const char*)workspace;
  const size_t E = (size_t)n_epochs;
  ICRS_TRY(hipMemcpyAsync(sectors, base + L.sectors, E * ICRS_MAX_SECTORS * 4 * sizeof(double),
                          hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(periodic, base + L.periodic, E * ICRS_MAX_SECTORS, hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(n_sectors, base + L.nsec, E * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  return ICRS_OK;
}

icrs_status icrs_point_images(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                              int64_t n_epochs, const double* t, double* images, int32_t* n_images, double* a_ps,
                              void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && !t) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  const icrs_config& c = h->cfg;
  return hip_status(icrs::launch_centre_images(c.n_lens, c.root_precision == ICRS_FP32, v.b, images, n_images, a_ps,
                                               nullptr, h->stream));
}

icrs_status icrs_mlp_pack(icrs_handle* h, const float* params, uint16_t* packed) {
  if (!h || !params || !packed || ((uintptr_t)packed & 15u)) return ICRS_EINVAL;
  return hip_status(icrs::mlp::launch_pack(params, packed, h->stream));
}

icrs_status icrs_mlp_forward(icrs_handle* h, const uint16_t* packed, const float* params, const float* norm,
                             int64_t n_rows, const float* x, float* y) {
  if (!h || n_rows < 0) return ICRS_EINVAL;
  if (n_rows == 0) return ICRS_OK;
  if (!packed || !params || !norm || !x || !y || ((uintptr_t)packed & 15u)) return ICRS_EINVAL;
  if (n_rows > ((int64_t)1 << 36)) return ICRS_EUNSUPPORTED;
  return hip_status(icrs::mlp::launch_forward(packed, params, norm, n_rows, x, y, h->stream));
}

size_t icrs_mlp_workspace_bytes(int64_t n_rows) {
  if (n_rows < 1) return 0;
  return icrs::mlp::train_workspace_bytes(n_rows);
}

icrs_status icrs_mlp_loss_grad(icrs_handle* h, const uint16_t* packed, const float* params, const float* norm,
                               int64_t n_rows, const float* x, const float* target, float* grad, float* loss,
                               void* workspace, size_t workspace_bytes) {
  if (!h || n_rows < 1 || !packed || !params || !norm || !x || !target || !grad || !workspace) return ICRS_EINVAL;
  if (((uintptr_t)packed & 15u) || ((uintptr_t)workspace & 3u)) return ICRS_EINVAL;
  if (workspace_bytes < icrs::mlp::train_workspace_bytes(n_rows)) return ICRS_ENOMEM;
  return hip_status(icrs::mlp::launch_loss_grad(packed, params, norm, n_rows, x, target, grad, loss, workspace,
                                                h->stream));
}

icrs_status icrs_mlp_adamw(icrs_handle* h, float* params, const float* grad, float* m, float* v, int64_t step,
                           float lr, float beta1, float beta2, float eps, float weight_decay, uint16_t* packed) {
  if (!h || !params || !grad || !m || !v || step < 1) return ICRS_EINVAL;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f)) return ICRS_EINVAL;
  if (packed && ((uintptr_t)packed & 15u)) return ICRS_EINVAL;
  return hip_status(icrs::mlp::launch_adamw(params, grad, m, v, step, lr, beta1, beta2, eps, weight_decay, packed,
                                            h->stream));
}

size_t icrs_learned_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs) {
  if (!h || n_events < 0 || n_epochs < 0) return 0;
  return learned_layout(h->cfg.n_lens, n_events, n_epochs).total;
}

void icrs_default_learned_config(icrs_learned_config* lc) {
  if (!lc) return;
  memset(lc, 0, sizeof(*lc));
  lc->n_check = 16;
  lc->n_r = 128;
  lc->n_theta = 512;
  lc->log_safety = 0.0;
  lc->prune_ratio = 1e-6;
  lc->vary_max = 0.1;
  lc->gate_rel = 1e-3;
  lc->gate_slack = 0.0;
  lc->margin_frac = 0.02;
}

icrs_status icrs_image_bounds(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                              int64_t n_epochs, const double* t, float* features, float* targets,
                              int32_t* n_images, uint32_t* flags, void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !features || !targets || !n_images || !flags)) return ICRS_EINVAL;
  const LearnedLayout LL = learned_layout(h->cfg.n_lens, n_events, n_epochs);
  if (workspace && workspace_bytes < LL.total) return ICRS_ENOMEM;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  char* base = (char*)workspace;
  const icrs_config& c = h->cfg;
  const int fp32_roots = c.root_precision == ICRS_FP32;
  double* cimg = (double*)(base + LL.cimg);
  ICRS_TRY(icrs::launch_centre_images(c.n_lens, fp32_roots, v.b, cimg, n_images, (double*)(base + LL.a_c), nullptr,
                                      h->stream, v.roots));
  return hip_status(icrs::launch_image_extents(c.n_lens, fp32_roots, c.n_limb, v.b, cimg, n_images,
                                               (double*)(base + LL.ext), features, targets,
                                               (double*)(base + LL.a_ring), flags, h->stream, v.roots));
}

icrs_status icrs_magnification_learned(icrs_handle* h, int64_t n_events, const double* params,
                                       const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                       const icrs_learned_config* lc, const uint16_t* packed,
                                       const float* mlp_params, const float* norm, double* mag, uint32_t* status,
                                       icrs_learned_stats* stats, void* workspace, size_t workspace_bytes) {
  if (!h || !learned_config_ok(lc) || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs))
    return ICRS_EINVAL;
  if (h->cfg.n_lens != 2) return ICRS_EUNSUPPORTED;
  if (n_epochs > 0 && (!t || !mag || !status || !packed || !mlp_params || !norm)) return ICRS_EINVAL;
  if (packed && ((uintptr_t)packed & 15u)) return ICRS_EINVAL;
  const LearnedLayout LL = learned_layout(h->cfg.n_lens, n_events, n_epochs);
  if (workspace && workspace_bytes < LL.total) return ICRS_ENOMEM;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK) return ps;
  return run_learned(h, v, lc, packed, mlp_params, norm, mag, status, stats, workspace);
}

icrs_status icrs_run_learned(icrs_handle* h, const double* t, const icrs_learned_config* lc, const uint16_t* packed,
                             const float* mlp_params, const float* norm, double* mag, uint32_t* status,
                             icrs_learned_stats* stats, void* workspace, size_t workspace_bytes) {
  if (!h || !workspace || workspace != h->prep_ws || !learned_config_ok(lc)) return ICRS_EINVAL;
  if (h->cfg.n_lens != 2) return ICRS_EUNSUPPORTED;
  if (h->prep_epochs > 0 && (!t || !mag || !status || !packed || !mlp_params || !norm)) return ICRS_EINVAL;
  if (packed && ((uintptr_t)packed & 15u)) return ICRS_EINVAL;
  if (workspace_bytes < learned_layout(h->cfg.n_lens, h->prep_events, h->prep_epochs).total) return ICRS_ENOMEM;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (h->prep_epochs == 0) return ICRS_OK;
  const Views v = prepared_views(h, t, workspace);
  // no host waits: the profiling timers (which wait for the stream) are off here
  const int prof = h->profiling;
  h->profiling = 0;
  const icrs_status st = run_learned(h, v, lc, packed, mlp_params, norm, mag, status, stats, workspace);
  h->profiling = prof;
  return st;
}

void icrs_default_hybrid_config(icrs_hybrid_config* hc) {
  if (!hc) return;
  memset(hc, 0, sizeof(*hc));
  hc->n_check = 16;
  hc->guard = 2.0;
  hc->tol = 1e-4;
  hc->vary_max = 0.1;
}

size_t icrs_hybrid_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs) {
  if (!h || n_events < 0 || n_epochs < 0) return 0;
  return learned_layout(h->cfg.n_lens, n_events, n_epochs).total;
}

icrs_status icrs_magnification_hybrid(icrs_handle* h, int64_t n_events, const double* params,
                                      const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                      const icrs_hybrid_config* hc, double* mag, uint32_t* status, void* workspace,
                                      size_t workspace_bytes) {
  if (!h || !hc || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (hc->n_check < 4 || hc->n_check > 64 || !(hc->guard >= 1.0 && hc->guard <= 100.0) || !(hc->tol > 0.0) ||
      !(hc->vary_max > 0.0))
    return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !mag || !status)) return ICRS_EINVAL;
  const LearnedLayout LL = learned_layout(h->cfg.n_lens, n_events, n_epochs);
  if (workspace && workspace_bytes < LL.total) return ICRS_ENOMEM;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  char* base = (char*)workspace;
  const icrs_config& c = h->cfg;
  const int fp32_roots = c.root_precision == ICRS_FP32;
  int32_t* cn = (int32_t*)(base + LL.cn);
  double* a_c = (double*)(base + LL.a_c);
  int32_t* ext = (int32_t*)(base + LL.lists);
  int32_t* counts = (int32_t*)(base + LL.counts);
  Timer tm(h);
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_centre_images(c.n_lens, fp32_roots, v.b, nullptr, cn, a_c, status, h->stream, v.roots));
  ICRS_TRY(icrs::launch_fill_i32(counts, 1, 0, h->stream));
  ICRS_TRY(icrs::launch_hybrid_select(c.n_lens, fp32_roots, hc->n_check, hc->guard, hc->tol, hc->vary_max, v.b, cn,
                                      a_c, v.roots, mag, status, v.sec.nsec, ext, counts, h->stream));
  ICRS_TRY(tm.end(&h->prof.ms_centre));
  ICRS_TRY(tm.begin());
  ICRS_TRY(icrs::launch_limb_sectors(c.n_lens, fp32_roots, c.n_limb, v.b, v.sec, status, h->stream, ext, n_epochs,
                                     counts, v.roots, v.list_b, v.counters + 2));
  ICRS_TRY(tm.end(&h->prof.ms_limb_sectors));
  ICRS_TRY(tm.flush());
  RaySet rs;
  rs.list = ext;
  rs.n = n_epochs;
  rs.n_dev = counts;
  return run_rays(h, v, c.max_retries, mag, status, 0u, rs);
}

icrs_status icrs_point_jacobian(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                                int64_t n_epochs, const double* t, double* a_ps, double* jac, uint32_t* status,
                                void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !jac)) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  return hip_status(icrs::launch_point_jacobian(h->cfg.n_lens, h->cfg.root_precision == ICRS_FP32, v.b, a_ps, jac,
                                                status, nullptr, 0u, h->stream));
}

icrs_status icrs_disk_magnification(icrs_handle* h, int64_t n_events, const double* params,
                                    const int64_t* epoch_offsets, int64_t n_epochs, const double* t, int n_x,
                                    int n_phi, double* mag, int32_t* count_changes, void* workspace,
                                    size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_x < 1 || n_x > 64 || n_phi < 1 || n_phi > 4096) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !mag || !count_changes)) return ICRS_EINVAL;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  // centre images in FP64 (their roots warm-start every disk node); the partial-flux area
  // of the workspace holds the centre's status words
  ICRS_TRY(icrs::launch_centre_images(h->cfg.n_lens, 0, v.b, nullptr, count_changes, nullptr, (uint32_t*)v.partial,
                                      h->stream, v.roots));
  return hip_status(icrs::launch_disk_mag(h->cfg.n_lens, n_x, n_phi, v.b, count_changes, (const uint32_t*)v.partial,
                                          v.roots, mag, h->stream));
}

icrs_status icrs_hybrid_vjp(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                            int64_t n_epochs, const double* t, const uint32_t* status, const double* sectors,
                            const uint8_t* periodic, const int32_t* n_sectors, const double* cotangent, double* grad,
                            double* jac, void* workspace, size_t workspace_bytes) {
  if (!h || !events_ok(h->cfg, n_events, params, epoch_offsets, n_epochs)) return ICRS_EINVAL;
  if (n_epochs > 0 && (!t || !status || !sectors || !periodic || !n_sectors)) return ICRS_EINVAL;
  if ((grad && !cotangent) || (!grad && !jac)) return ICRS_EINVAL;
  if (h->cfg.n_theta > 1024) return ICRS_EUNSUPPORTED;
  Views v;
  const icrs_status ps = prepare(h, n_events, params, epoch_offsets, n_epochs, t, workspace, workspace_bytes, &v);
  if (ps != ICRS_OK || n_epochs == 0) return ps;
  const size_t E = (size_t)n_epochs;
  ICRS_TRY(hipMemcpyAsync(v.sec.sectors, sectors, E * ICRS_MAX_SECTORS * 4 * sizeof(double),
                          hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.periodic, periodic, E * ICRS_MAX_SECTORS, hipMemcpyDeviceToDevice, h->stream));
  ICRS_TRY(hipMemcpyAsync(v.sec.nsec, n_sectors, E * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
  double* J = jac ? jac : v.jac;
  // extended epochs on their frozen sectors (point epochs carry no sectors and get zero
  // rows here), then the point epochs' rows through their images, then the contraction
  ICRS_TRY(icrs::launch_adjoint(h->cfg.n_lens, v.b, v.sec, h->cfg.n_r, h->cfg.n_theta, h->cfg.delta_c, nullptr, J,
                                nullptr, nullptr, (unsigned long long*)(v.counters + 12), h->stream));
  ICRS_TRY(icrs::launch_point_jacobian(h->cfg.n_lens, h->cfg.root_precision == ICRS_FP32, v.b, nullptr, J, nullptr,
                                       status, ICRS_ST_POINT, h->stream));
  if (grad) ICRS_TRY(icrs::launch_contract(v.b, J, cotangent, grad, h->stream));
  return ICRS_OK;
}

size_t icrs_marginal_nll_workspace_bytes(int64_t n_events) {
  if (n_events < 0) return 0;
  return align_up((size_t)(n_events + 1) * sizeof(int64_t)) + align_up((size_t)n_events * 4 * sizeof(double));
}

icrs_status icrs_marginal_nll(icrs_handle* h, int64_t n_events, const int64_t* epoch_offsets, int64_t n_epochs,
                              const double* mag, const double* flux, const double* sigma, const double* prior,
                              double* nll, double* beta, double* dnll_dmag, void* workspace,
                              size_t workspace_bytes) {
  if (!h || n_events < 0 || n_epochs < 0 || n_epochs > ICRS_MAX_EPOCHS || n_events > 0x7fffffffLL)
    return ICRS_EINVAL;
  if (n_events == 0) return n_epochs == 0 ? ICRS_OK : ICRS_EINVAL;
  if (!epoch_offsets || !prior || !nll || !workspace) return ICRS_EINVAL;
  if (n_epochs > 0 && (!mag || !flux || !sigma)) return ICRS_EINVAL;
  if (epoch_offsets[0] != 0 || epoch_offsets[n_events] != n_epochs) return ICRS_EINVAL;
  for (int64_t i = 0; i < n_events; ++i)
    if (epoch_offsets[i + 1] < epoch_offsets[i]) return ICRS_EINVAL;
  for (int64_t i = 0; i < n_events; ++i) {
    const double* q = prior + 4 * i;
    if (!finite_all(q, 4) || !(q[2] > 0.0) || !(q[3] > 0.0)) return ICRS_EINVAL;
  }
  if (((uintptr_t)workspace & (kAlign - 1)) != 0) return ICRS_EINVAL;
  if (workspace_bytes < icrs_marginal_nll_workspace_bytes(n_events)) return ICRS_ENOMEM;
  char* base = (char*)workspace;
  int64_t* off = (int64_t*)base;
  double* pr = (double*)(base + align_up((size_t)(n_events + 1) * sizeof(int64_t)));
  ICRS_TRY(hipMemcpyAsync(off, epoch_offsets, (size_t)(n_events + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                          h->stream));
  ICRS_TRY(hipMemcpyAsync(pr, prior, (size_t)n_events * 4 * sizeof(double), hipMemcpyHostToDevice, h->stream));
  return hip_status(icrs::launch_nll(n_events, off, mag, flux, sigma, pr, nll, beta, dnll_dmag, h->stream));
}

const char* icrs_status_string(icrs_status s) {
  switch (s) {
    case ICRS_OK:
      return "ok";
    case ICRS_EINVAL:
      return "invalid argument";
    case ICRS_ENOMEM:
      return "workspace too small";
    case ICRS_EHIP:
      return "HIP runtime error";
    case ICRS_EUNSUPPORTED:
      return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
