// icrs_launch.hpp -- host-side launchers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icrs {

// Device views of one call's inputs and workspace.
struct Batch {
  const double* params;        // [n_events][11] (device copy)
  const int64_t* offsets;      // [n_events + 1] (device copy)
  const int32_t* epoch_event;  // [n_epochs]
  const double* t;             // [n_epochs]
  int64_t n_events;
  int64_t n_epochs;
};

struct SectorBuf {
  double* sectors;   // [n_epochs][10][4]
  uint8_t* periodic; // [n_epochs][10]
  int32_t* nsec;     // [n_epochs]
};

hipError_t launch_epoch_event(const Batch& b, int32_t* epoch_event, hipStream_t s);

// point images of every epoch's source centre; writes status[e] (assigns).  roots, if given,
// receives the polynomial's roots ([n_epochs][kMaxRoots] complex).
hipError_t launch_centre_images(int n_lens, int root_fp32, const Batch& b, double* images, int32_t* n_images,
                                double* a_ps, uint32_t* status, hipStream_t s, double* roots = nullptr);

// limb images + sectors (one workgroup per epoch); ORs status bits.  With list, only the
// n_list epochs it names (with n_list_dev, the list's length is read on the device and
// n_list is only its upper bound).  With roots (the centre polynomial's, from
// launch_centre_images), the limb points' root solves start there, and an epoch where such
// a solve ends with a forbidden image count or an unconverged root is queued in redo_list
// (count in *redo_count, zeroed here; n_epochs entries) and redone from the Cauchy circle
// in FP64 by a second launch.
hipError_t launch_limb_sectors(int n_lens, int root_fp32, int n_limb, const Batch& b, const SectorBuf& out,
                               uint32_t* status, hipStream_t s, const int32_t* list = nullptr, int64_t n_list = 0,
                               const int32_t* n_list_dev = nullptr, const double* roots = nullptr,
                               int32_t* redo_list = nullptr, int32_t* redo_count = nullptr);

struct RayWork {
  const int32_t* list = nullptr;    // epochs to process (all their sectors), or nullptr = 0..n-1
  int64_t n = 0;                    // number of epochs in the list (an upper bound with n_dev)
  const int32_t* n_dev = nullptr;   // device-side count of the list, when only the device knows it
  const int32_t* items = nullptr;   // instead: single sectors 16 e + slot, count in *n_items
  const int32_t* n_items = nullptr;
  int32_t* fallback = nullptr;      // FP32 pass: sectors sent to the FP64 pass
  int32_t* n_fallback = nullptr;
  int32_t* retake = nullptr;        // FP32 pass: crossings retaken in FP64, pairs (16 e + slot, queue flags)
  unsigned long long* n_retake = nullptr;  // their count (may pass retake_cap; pairs beyond it are not stored)
  int64_t retake_cap = 0;
  unsigned long long* retake_fx = nullptr;  // per sector slot: the retaken terms' sum, two's complement, 2^-40 units
};

// Buffers of the FP64 retake of FP32 crossings next to the edge rule's jump at delta_c.
struct RetakeBuf {
  int32_t* items = nullptr;  // [cap][2]
  unsigned long long* n = nullptr;  // 8-byte aligned
  int64_t cap = 0;
  unsigned long long* fx = nullptr;  // [n_epochs * 10]
};

// persistent ray kernel; queue: 16 bytes of device scratch (zeroed here) for the work
// counter; fallback/n_fallback: [n_epochs * 10] list + counter for FP32 -> FP64 sectors.
// stage 0 is the main pass over w (FP32 or FP64); stage 1 is the FP64 pass over the sectors
// the FP32 main pass listed (nothing to do when ray_fp32 == 0).  Both stages are always
// launched, in order, before the finalize kernel.  rb: the FP32 pass lists its crossings
// whose edge-rule branch rounding could flip, and stage 0 retakes them in FP64 and adds
// them to partial before it returns (sectors whose crossings do not fit go to the FP64 pass).
hipError_t launch_rays(int n_lens, int ray_fp32, int stage, const Batch& b, const SectorBuf& sec, const RayWork& w,
                       int n_r, int n_theta, double delta_c, double* partial, uint8_t* clip,
                       unsigned long long* queue, int32_t* fallback, int32_t* n_fallback, const RetakeBuf& rb,
                       hipStream_t s);

// sums sector fluxes into magnifications; epochs with edge touches and retries left get
// widened sectors and are appended to next_list (count in *next_count).  add_mag (or null):
// a per-epoch term added to the magnification (images given no grid).
hipError_t launch_finalize(const Batch& b, const SectorBuf& sec, const RayWork& w, const double* partial,
                           const uint8_t* clip, int attempt, int max_retries, int32_t* next_list,
                           int32_t* next_count, double* mag, uint32_t* status, uint32_t extra_status,
                           unsigned long long* passes, hipStream_t s, const double* add_mag = nullptr);

// frozen-structure Jacobian jac[n_epochs][11] (and mag if non-null) on the given sectors;
// with cot and grad non-null also grad[n_events][11] = sum_e cot[e] jac[e]
hipError_t launch_adjoint(int n_lens, const Batch& b, const SectorBuf& sec, int n_r, int n_theta, double delta_c,
                          const double* cot, double* jac, double* grad, double* mag, unsigned long long* queue,
                          hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// learned-bounds path (icrs_learned.hip)
hipError_t launch_image_extents(int n_lens, int root_fp32, int n_pts, const Batch& b, const double* cimg,
                                const int32_t* cn, double* ext, float* feat, float* tgt, double* a_ring,
                                uint32_t* flags, hipStream_t s, const double* roots = nullptr);
hipError_t launch_learned_sectors(int n_lens, const Batch& b, const double* cimg, const int32_t* cn,
                                  const double* a_c, const double* a_ring, const double* ext, const float* y,
                                  double log_safety, double margin_frac, double prune_ratio, double vary_max,
                                  uint32_t* flags, const SectorBuf& sec, double* add_mag, int32_t* lists,
                                  int32_t* counts, int32_t* n_pruned, hipStream_t s);
hipError_t launch_learned_gate(const Batch& b, const int32_t* learned, const int32_t* n_learned, int64_t n_max,
                               const double* a_c, const double* a_ring, const double* mag, uint32_t* status,
                               double gate_rel, double gate_slack, uint32_t* flags, int32_t* lists,
                               int32_t* counts, hipStream_t s);

// hybrid light curve (icrs_hybrid.hip): epochs whose check circle shows no caustic and a
// point-source magnification flat to tol get mag = A_ps and ICRS_ST_POINT; the others are
// appended to ext_list (count in *ext_count, zeroed by the caller); nsec[e] = 0 for all.
hipError_t launch_hybrid_select(int n_lens, int root_fp32, int n_check, double guard, double tol, double vary_max,
                                const Batch& b, const int32_t* cn, const double* a_c, const double* roots,
                                double* mag, uint32_t* status, int32_t* nsec, int32_t* ext_list, int32_t* ext_count,
                                hipStream_t s);
// A_ps and dA_ps/dparams [n_epochs][11] of every epoch (with only_status, only epochs whose
// status_in has that bit); status_out (or null) gets the image-finding bits.
// Grid-free disk reference: cn_changes holds each epoch's centre image count on entry and
// the number of disk nodes whose image count or status differs (plus one for a flagged
// centre) on return.
hipError_t launch_disk_mag(int n_lens, int n_x, int n_phi, const Batch& b, int32_t* cn_changes,
                           const uint32_t* centre_status, const double* roots, double* mag, hipStream_t s);
hipError_t launch_point_jacobian(int n_lens, int root_fp32, const Batch& b, double* a_ps, double* jac,
                                 uint32_t* status_out, const uint32_t* status_in, uint32_t only_status,
                                 hipStream_t s);
// grad[ev][k] = sum over the event's epochs of cot[e] jac[e][k] (fixed order)
hipError_t launch_contract(const Batch& b, const double* jac, const double* cot, double* grad, hipStream_t s);

// marginalised likelihood (icrs_likelihood.hip): per event NLL, posterior moments (or null)
// and dNLL/dmag per epoch (or null); offsets and prior are device arrays
hipError_t launch_nll(int64_t n_events, const int64_t* offsets, const double* mag, const double* flux,
                      const double* sigma, const double* prior, double* nll, double* beta, double* dnll,
                      hipStream_t s);

namespace mlp {
// learned-bounds network: FP32 master blob (param_floats()), packed bf16 weights
// (packed_halfs()), norm[32] = in_mean[10], in_std[10], out_mean[4], out_std[4]
int param_floats();
int packed_halfs();
size_t train_workspace_bytes(int64_t m_rows);
hipError_t launch_pack(const float* prm, uint16_t* wb, hipStream_t s);
hipError_t launch_forward(const uint16_t* wb, const float* prm, const float* norm, int64_t m_rows, const float* x,
                          float* y, hipStream_t s);
hipError_t launch_loss_grad(const uint16_t* wb, const float* prm, const float* norm, int64_t m_rows, const float* x,
                            const float* tgt, float* grad, float* loss, void* ws, hipStream_t s);
hipError_t launch_adamw(float* prm, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                        float beta2, float eps, float wd, uint16_t* wb, hipStream_t s);
}  // namespace mlp
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

}  // namespace icrs
