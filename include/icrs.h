/* icrs.h -- C ABI of the MI355X (gfx950) image-centred ray-shooting library.
 *
 * Computes finite-source magnifications of binary- and triple-lens microlensing events
 * with a uniform or linearly limb-darkened source, by the image-centred ray-shooting (ICRS)
 * method of Miyazaki & Kawahara, "microJAX" (arXiv 2510.02639):
 *   - source centre on a straight trajectory (t0, u0, tE, alpha)            -- Sec. 3.5
 *   - N_limb points on the source limb, images by Ehrlich-Aberth roots of the
 *     lens polynomial (degree 5 or 10), validated against the lens equation -- Secs. 2.1, 3.1, 3.2
 *   - polar sectors around the images from 1-D binning of image-limb points -- Sec. 3.2
 *   - an N_r x N_theta polar grid per sector, every node shot back through the
 *     lens equation, row quadrature with cubic boundary crossings and the
 *     uniform / limb-darkened edge rules, radial sum, normalisation          -- Sec. 3.3, App. A
 *
 * Conventions shared by every entry point
 *   - Units: t, t0, tE in days; alpha, psi in radians; s, u0, rho, r3 in Einstein radii of
 *     the total lens mass.
 *   - Event parameters are a HOST array of ICRS_N_PARAMS doubles per event:
 *       [s, q, u0, alpha, t0, tE, rho, u_ld, q3, r3, psi]
 *     q = m2/m1 and the primary sits at -q s/(1+q) on the real axis, the secondary at
 *     s/(1+q) (centre of mass of the pair at the origin).  Triple lenses (n_lens = 3) add
 *     q3 = m3/m1 at r3 e^{i psi} from the M1-M2 midpoint (paper Fig. 3); binary events
 *     ignore the last three entries.  u_ld = 0 selects the uniform-source rule.
 *   - Epochs are grouped by event in CSR form: a HOST array epoch_offsets[n_events + 1]
 *     (non-decreasing, offsets[0] = 0, offsets[n_events] = n_epochs) and a DEVICE array
 *     t[n_epochs]; epoch e belongs to the event i with offsets[i] <= e < offsets[i+1].
 *   - Outputs mag[n_epochs] (double) and status[n_epochs] (uint32, ICRS_ST_* bits) are
 *     DEVICE arrays owned by the caller.
 *   - The caller owns all memory.  The library allocates nothing inside a call: device
 *     scratch comes from a caller workspace of icrs_workspace_bytes() bytes (device memory,
 *     256-byte aligned).  Results stay valid in the workspace until the next call using it.
 *   - Argument errors (bad sizes, NULL pointers, out-of-range parameters, unsorted offsets)
 *     return ICRS_EINVAL before anything is enqueued.  A workspace that is too small gives
 *     ICRS_ENOMEM.  A HIP runtime failure gives ICRS_EHIP.
 *   - Work is enqueued asynchronously on the handle's stream.  Work list sizes (clip
 *     retries, learned and fallback epochs) stay on the device, so no call waits for the
 *     stream unless profiling is on or host statistics are asked for.  Data-dependent
 *     failures never fail a call: they set status bits, and an epoch without a usable result
 *     gets NaN.
 *   - A handle must not be used from two threads at once.
 */
#ifndef ICRS_H_
#define ICRS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ICRS_ABI_VERSION 1u
#define ICRS_N_PARAMS 11
#define ICRS_MAX_SECTORS 10 /* 5(N-1) for N = 3: the sector cap per epoch (Sec. 3.2) */
#define ICRS_MAX_EPOCHS (1LL << 27) /* epochs per call; more returns ICRS_EINVAL */

typedef enum {
  ICRS_OK = 0,
  ICRS_EINVAL = -1,
  ICRS_ENOMEM = -2,
  ICRS_EHIP = -3,
  ICRS_EUNSUPPORTED = -4
} icrs_status;

/* Per-epoch status bits. */
#define ICRS_ST_ROOT_NONCONV 1u   /* an Ehrlich-Aberth solve reached its iteration cap */
#define ICRS_ST_IMG_COUNT 2u      /* an image count outside {N+1, N+3, ..., 5(N-1)} after seeding */
#define ICRS_ST_CAP_OVERFLOW 4u   /* more sector candidates than the cap: pairs were merged */
#define ICRS_ST_CLIP 8u           /* inside rays still touch a sector edge after the retries */
#define ICRS_ST_NAN 16u           /* the magnification is not finite */
#define ICRS_ST_GIVEN 64u         /* sectors were supplied by the caller */
#define ICRS_ST_IMG_RECHECK 512u  /* a kept image failed the final substitution check and was dropped */
#define ICRS_ST_BAD_SECTORS 1024u /* a given sector count outside 0..ICRS_MAX_SECTORS; result NaN */

/* Ray-loop precision. */
#define ICRS_FP64 0
#define ICRS_FP32 1

typedef struct icrs_config {
  uint32_t abi_version;  /* must be ICRS_ABI_VERSION */
  int32_t n_lens;        /* 2 (binary, degree-5 polynomial) or 3 (triple, degree 10) */
  int32_t n_limb;        /* limb points per epoch for image finding, 8..256 (Sec. 3.2) */
  int32_t n_r;           /* radial grid nodes per sector, 4..4096 (Sec. 3.3) */
  int32_t n_theta;       /* angular grid nodes per sector, 64..1024 (Sec. 3.3) */
  int32_t ray_precision; /* ICRS_FP64 or ICRS_FP32 (FP32 rays relative to an FP64 anchor) */
  int32_t root_precision;/* ICRS_FP64: FP64 Ehrlich-Aberth; ICRS_FP32: FP32 EA then FP64 polish */
  int32_t max_retries;   /* sector-widening retries after an edge touch, 0..4 */
  double delta_c;        /* threshold of the limb-darkened edge rule (App. A.2), 0 <= delta_c <= 1 */
} icrs_config;

typedef struct icrs_handle icrs_handle;

/* Fill *cfg with the defaults: binary, N_limb 64, 64 x 256 grid, FP64 everywhere,
 * 2 retries, delta_c = 0.1. */
void icrs_default_config(icrs_config* cfg);

/* Create a handle bound to a HIP stream (hipStream_t passed as void*, NULL = default
 * stream) on the current device.  Validates the configuration (ICRS_EINVAL if invalid).
 * The handle holds no device memory. */
icrs_status icrs_create(const icrs_config* cfg, void* hip_stream, icrs_handle** out);
void icrs_destroy(icrs_handle* h);

/* Device workspace needed for a call over n_events events and n_epochs epochs. */
size_t icrs_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs);

/* Plain ICRS light curves (the full path: trajectory, limb images, sectors, rays,
 * quadrature, retries).  params: HOST [n_events][ICRS_N_PARAMS]; epoch_offsets: HOST
 * [n_events + 1]; t: DEVICE [n_epochs]; mag, status: DEVICE [n_epochs] outputs;
 * workspace: DEVICE, workspace_bytes >= icrs_workspace_bytes(h, n_events, n_epochs).
 * Valid parameter ranges: s > 0, q > 0, tE > 0, 0 < rho <= 1, 0 <= u_ld < 1, and for
 * triples q3 > 0, r3 >= 0; all finite.  After the call the final sectors of every epoch
 * can be read with icrs_get_sectors(). */
icrs_status icrs_magnification(icrs_handle* h, int64_t n_events, const double* params,
                               const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                               double* mag, uint32_t* status, void* workspace,
                               size_t workspace_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): icrs_magnification without a caller
 * workspace.  The device scratch is a library-owned array of ICRS_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, resolved on the first call on each device and held until the process
 * ends; the call allocates nothing (no hipMalloc/hipFree, no allocating library routine).
 * Inputs and outputs as for icrs_magnification, on the current device (the handle's stream
 * must belong to it).  A batch whose workspace (icrs_workspace_bytes) exceeds the scratch --
 * about 63 000 epochs -- returns ICRS_ENOMEM before anything is enqueued.  Every call on a
 * GPU uses that GPU's one scratch array: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialised by the caller.  Each call initialises every part of
 * the scratch it reads, so the contents left by an earlier call do not matter; final
 * sectors are not exported (icrs_get_sectors needs a caller workspace). */
#define ICRS_NOALLOC_SCRATCH_BYTES (64u << 20)
icrs_status icrs_magnification_noalloc(icrs_handle* h, int64_t n_events, const double* params,
                                       const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                       double* mag, uint32_t* status);

/* The plain path split for stream capture (hipGraph) and repeated runs over one batch:
 * icrs_prepare() checks and uploads the events (host arrays as for icrs_magnification)
 * into the workspace and records the batch in the handle; icrs_run() then enqueues the whole
 * path on the handle's stream with no host synchronisation and no host-memory access, so it
 * can be captured into a graph and replayed.  Every clip-retry pass is enqueued; its work
 * list size is read on the device, and an empty pass ends at once.  t, mag, status as for
 * icrs_magnification (n_epochs given to icrs_prepare()); workspace must be the one passed
 * to icrs_prepare().  Profiling does not apply to icrs_run(). */
icrs_status icrs_prepare(icrs_handle* h, int64_t n_events, const double* params,
                         const int64_t* epoch_offsets, int64_t n_epochs, void* workspace,
                         size_t workspace_bytes);
icrs_status icrs_run(icrs_handle* h, const double* t, double* mag, uint32_t* status,
                     void* workspace, size_t workspace_bytes);

/* The same quadrature on caller-given sectors: one pass, no retries (status gets
 * ICRS_ST_GIVEN, plus ICRS_ST_CLIP if inside rays touch an edge).  sectors: DEVICE
 * [n_epochs][ICRS_MAX_SECTORS][4] doubles (r_lo, r_hi, theta_lo, theta_hi) with
 * 0 <= r_lo < r_hi and theta_lo < theta_hi; periodic: DEVICE [n_epochs][ICRS_MAX_SECTORS]
 * bytes (1 = full ring, theta range 2 pi wrapped); n_sectors: DEVICE [n_epochs] int32 in
 * 0..ICRS_MAX_SECTORS.  Entries past n_sectors[e] are ignored.  A count outside that range
 * (it lives on the device, so the call cannot reject it) shoots no rays and gives the epoch
 * NaN with ICRS_ST_BAD_SECTORS. */
icrs_status icrs_magnification_given(icrs_handle* h, int64_t n_events, const double* params,
                                     const int64_t* epoch_offsets, int64_t n_epochs,
                                     const double* t, const double* sectors,
                                     const uint8_t* periodic, const int32_t* n_sectors,
                                     double* mag, uint32_t* status, void* workspace,
                                     size_t workspace_bytes);

/* Derivatives of the magnification on a frozen structure (the adjoint of the plain path):
 * the caller-given sectors (normally those icrs_get_sectors() returns after
 * icrs_magnification()), and the inside/outside pattern, crossing stencils and edge-factor
 * branches of the primal evaluation on them, are held fixed; the rays are recomputed in FP64
 * and differentiated exactly (crossings by implicit differentiation of the cubic
 * interpolant, App. A).  This replaces the paper's forward-mode AD (Sec. 3.5), which needs
 * a sigmoid surrogate for chi and cannot run in reverse mode (Sec. 6).
 * Inputs as icrs_magnification_given(); cotangent: DEVICE [n_epochs] (may be NULL when grad
 * is NULL).  Outputs (DEVICE, any may be NULL but not all): grad [n_events][ICRS_N_PARAMS]
 * = sum over the event's epochs of cotangent[e] * dA_e/dparams; jac [n_epochs][ICRS_N_PARAMS]
 * = dA_e/dparams; mag [n_epochs] = A_e.  Parameter order as in params; entries that do not
 * apply (q3, r3, psi for binaries) are 0.  n_theta must be <= 1024.  An epoch whose
 * n_sectors entry lies outside 0..ICRS_MAX_SECTORS gets NaN in jac and mag. */
icrs_status icrs_magnification_vjp(icrs_handle* h, int64_t n_events, const double* params,
                                   const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                   const double* sectors, const uint8_t* periodic,
                                   const int32_t* n_sectors, const double* cotangent, double* grad,
                                   double* jac, double* mag, void* workspace, size_t workspace_bytes);

/* Copy the final sectors of the last icrs_magnification() on this workspace into DEVICE
 * arrays laid out as in icrs_magnification_given(). */
icrs_status icrs_get_sectors(icrs_handle* h, const void* workspace, int64_t n_epochs,
                             double* sectors, uint8_t* periodic, int32_t* n_sectors);

/* Point-source images of every epoch's source centre (Sec. 2.1, eqs. amp_point and detJ):
 * images: DEVICE [n_epochs][10][2] doubles (re, im), n_images: DEVICE [n_epochs] int32,
 * a_ps: DEVICE [n_epochs] doubles = sum_j 1/|det J(z_j)|.  Any of the three may be NULL. */
icrs_status icrs_point_images(icrs_handle* h, int64_t n_events, const double* params,
                              const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                              double* images, int32_t* n_images, double* a_ps, void* workspace,
                              size_t workspace_bytes);

/* Opt-in timing of the library's kernels (the benchmark's live measurement).  With
 * profiling on, every call records HIP events around each kernel class on the handle's
 * stream and waits for them at the end of the call; totals accumulate in the handle.
 * n_sector_passes counts (epoch, sector) grids shot (each is n_r x n_theta rays), summed
 * over the clip retries.  ms_rays covers every ray kernel; ms_rays_main only the main-pass
 * kernel of each call's first attempt (FP32 or FP64 per ray_precision, one launch per
 * call, n_main_launches of them), which shot n_main_sectors grids in total (first-attempt
 * sectors less those the FP32 pass handed to the FP64 pass). */
typedef struct icrs_profile {
  double ms_centre;        /* centre images (point-source magnification)   */
  double ms_limb_sectors;  /* limb images + sector construction            */
  double ms_rays;          /* ray shooting + row quadrature                */
  double ms_finalize;      /* sums, clip retries                           */
  int64_t n_calls;
  int64_t n_rays_launches;
  int64_t n_sector_passes;
  int64_t n_epochs;
  double ms_rays_main;     /* main ray pass of the first attempt over plain  */
  int64_t n_main_launches; /* sectors (the plain path, the learned path's     */
  int64_t n_main_sectors;  /* fallback epochs, caller-given sectors)          */
  int64_t n_main_rays;     /* n_main_sectors x that call's n_r x n_theta     */
  double ms_rays_learned;  /* the same for the learned path's own boxes      */
  int64_t n_learned_launches;
  int64_t n_learned_sectors;
  int64_t n_learned_rays;  /* n_learned_sectors x the learned n_r x n_theta  */
} icrs_profile;

icrs_status icrs_set_profiling(icrs_handle* h, int on);
/* Copy the accumulated totals into *out; reset them when reset != 0. */
icrs_status icrs_get_profile(icrs_handle* h, icrs_profile* out, int reset);

/* ---- learned-bounds network (not in the paper) ---------------------------------------
 * A multilayer perceptron 10 -> 128 -> 128 -> 128 -> 4 with GELU (tanh form) after each
 * hidden layer, 34 948 parameters, run on the matrix cores with bfloat16 operands and FP32
 * accumulation.  It maps the features of one point-source image to four standardised
 * outputs (the learned path turns them into a polar box).  Parameters live in a padded
 * FP32 master blob of ICRS_MLP_PARAM_FLOATS floats (DEVICE, caller-owned):
 *   W1 [128][32] (input columns 10..31 zero), b1 [128], W2 [128][128], b2 [128],
 *   W3 [128][128], b3 [128], W4 [16][128] (rows 4..15 zero), b4 [16] (entries 4..15 zero),
 * W[n][k] multiplying input k into output n.  The matrix products read a packed bfloat16
 * copy of ICRS_MLP_PACKED_HALFS halfs (DEVICE, 16-byte aligned) that icrs_mlp_pack and
 * icrs_mlp_adamw write.  norm (DEVICE, ICRS_MLP_NORM_FLOATS floats): in_mean[10],
 * in_std[10], out_mean[4], out_std[4]; inputs are standardised with it, and outputs are
 * returned de-standardised (icrs_mlp_forward) or compared with standardised targets
 * (icrs_mlp_loss_grad).  All run on the handle's stream; row-major FP32 x [n_rows][10],
 * y / target [n_rows][4]. */
#define ICRS_MLP_PARAM_FLOATS 39312
#define ICRS_MLP_PACKED_HALFS 75776
#define ICRS_MLP_NORM_FLOATS 32

/* packed = bfloat16 (round to nearest even) of the weight matrices and their transposes */
icrs_status icrs_mlp_pack(icrs_handle* h, const float* params, uint16_t* packed);
/* y = network(x) for n_rows rows (n_rows >= 0) */
icrs_status icrs_mlp_forward(icrs_handle* h, const uint16_t* packed, const float* params, const float* norm,
                             int64_t n_rows, const float* x, float* y);
/* Bytes of workspace icrs_mlp_loss_grad needs for n_rows rows. */
size_t icrs_mlp_workspace_bytes(int64_t n_rows);
/* loss[0] = mean over rows and the 4 outputs of (y - (target - out_mean) / out_std)^2 with y
 * the standardised output; grad = d loss / d params in the blob layout (padding entries 0).
 * Deterministic (fixed-order reductions).  n_rows >= 1. */
icrs_status icrs_mlp_loss_grad(icrs_handle* h, const uint16_t* packed, const float* params, const float* norm,
                               int64_t n_rows, const float* x, const float* target, float* grad, float* loss,
                               void* workspace, size_t workspace_bytes);
/* One AdamW step (bias-corrected moments, decoupled decay on weight matrices only) on
 * params with moments m, v (zero before step 1); step >= 1; repacks into packed when it
 * is non-NULL. */
icrs_status icrs_mlp_adamw(icrs_handle* h, float* params, const float* grad, float* m, float* v, int64_t step,
                           float lr, float beta1, float beta2, float eps, float weight_decay, uint16_t* packed);

/* ---- learned-bounds path (not in the paper) -------------------------------------------
 * Training data: for every epoch, the point-source images of the source centre and, per
 * image, the extent of the limb images the plain sector step assigns to it (n_limb limb
 * points of the handle's config, each limb image given to the nearest centre image).
 * Outputs (DEVICE): features [n_epochs][MI][10] (MI = n_lens^2 + 1; rows j >= n_images[e]
 * are zero): log10 s, log10 q, w_c.x, w_c.y, log10 rho, z.x, z.y, parity, log10 mu,
 * log10(sigma/rho), with mu = 1/|det J| and sigma = rho/|1 - |kappa|| the image's
 * linearised size; targets [n_epochs][MI][4] = ln(offset/sigma) of the four extents
 * (|z| - r_min, r_max - |z|, |z| (theta_z - theta_min), |z| (theta_max - theta_z)),
 * offsets floored at 1e-3 sigma; n_images [n_epochs]; flags [n_epochs], 0 when every limb
 * point has as many images as the centre, every image received limb images and none
 * spans half a turn (only such epochs are training data). */
icrs_status icrs_image_bounds(icrs_handle* h, int64_t n_events, const double* params, const int64_t* epoch_offsets,
                              int64_t n_epochs, const double* t, float* features, float* targets,
                              int32_t* n_images, uint32_t* flags, void* workspace, size_t workspace_bytes);

/* Learned path settings.  n_check limb points (8..64) confirm the image count and sample
 * each image's extent; the learned boxes get n_r x n_theta grids; network offsets are
 * scaled by exp(log_safety); images with mu < prune_ratio x A_ps get no grid and add mu;
 * epochs whose ring-average point-source magnification differs from the centre's by more
 * than vary_max (relative) go to the plain path before any ray; the drift gate sends back
 * results with |A - A_est| > gate_rel A_ps + gate_slack |A_ring - A_ps| (A_est = A_ps +
 * w2 (A_ring - A_ps), w2 the limb-darkened profile's mean squared radius); each box is widened by
 * margin_frac of its extent plus the plain floors (rho/100 in r, rho/(100 r_mid) in theta).
 * icrs_default_learned_config: 16, 128, 512, 0, 0.0, 1e-6, 0.1, 1e-3, 0.02, 0.0. */
typedef struct icrs_learned_config {
  int32_t n_check;
  int32_t n_r;
  int32_t n_theta;
  int32_t reserved;
  double log_safety;
  double prune_ratio;
  double vary_max;
  double gate_rel;
  double margin_frac;
  double gate_slack;  /* >= 0 */
} icrs_learned_config;

typedef struct icrs_learned_stats {
  int64_t n_epochs;
  int64_t n_learned;        /* epochs whose result comes from learned boxes         */
  int64_t n_fallback;       /* epochs recomputed by the plain path                  */
  int64_t n_gate_rejected;  /* of those, rejected after the learned rays             */
  int64_t n_pruned_images;  /* images given no grid                                 */
} icrs_learned_stats;

#define ICRS_ST_LEARNED 128u  /* result from learned boxes                         */
#define ICRS_ST_FALLBACK 256u /* the learned path handed this epoch to the plain path */

void icrs_default_learned_config(icrs_learned_config* lc);
size_t icrs_learned_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs);
/* Magnifications through the learned path (binary lenses; n_lens = 3 returns
 * ICRS_EUNSUPPORTED).  Same inputs and outputs as icrs_magnification plus the network
 * (packed, params, norm as for icrs_mlp_forward) and optional host stats.  Epochs that
 * fail a check are computed by the plain path of the handle's config inside the call.
 * The learned, fallback and retry lists keep their sizes on the device: with stats == NULL
 * (and profiling off) the call only enqueues work on the handle's stream, so it can be
 * captured into a HIP graph; with stats (HOST) it waits for the stream at the end to fill
 * them. */
icrs_status icrs_magnification_learned(icrs_handle* h, int64_t n_events, const double* params,
                                       const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                       const icrs_learned_config* lc, const uint16_t* packed,
                                       const float* mlp_params, const float* norm, double* mag, uint32_t* status,
                                       icrs_learned_stats* stats, void* workspace, size_t workspace_bytes);

/* The learned path on the batch that icrs_prepare() uploaded into workspace (which must be
 * at least icrs_learned_workspace_bytes() long): no host memory is read and, with
 * stats == NULL and profiling off, nothing waits for the stream, so the call can be
 * captured into a HIP graph and replayed (Sec. 3.4's batching of many epochs and events in
 * one pass, with every list size kept on the device).  Arguments otherwise as for
 * icrs_magnification_learned; n_epochs is the prepared batch's. */
icrs_status icrs_run_learned(icrs_handle* h, const double* t, const icrs_learned_config* lc,
                             const uint16_t* packed, const float* mlp_params, const float* norm,
                             double* mag, uint32_t* status, icrs_learned_stats* stats, void* workspace,
                             size_t workspace_bytes);

/* ---- hybrid light curve (Sec. 3.4, item iii) -----------------------------------------
 * The paper computes finite-source magnifications only on a preselected set of epochs
 * (e.g. near caustics) and the point-source magnification of eq. amp_point elsewhere; it
 * gives no selection rule.  The rule here: n_check points on the circle of radius
 * guard x rho around the source centre are solved like the centre; an epoch is "extended"
 * when one of them changes the image count or carries a root flag (a caustic crosses the
 * circle), when their mean point-source magnification differs from the centre's A_ps by
 * more than tol x A_ps (the Laplacian of A_ps, which leads the finite-source correction),
 * or when one of them differs by more than vary_max x A_ps.  Extended epochs go through the
 * plain path with the handle's config; every other epoch gets mag = A_ps and status
 * ICRS_ST_POINT.  icrs_default_hybrid_config: 16, 0, 2.0, 1e-4, 0.1. */
typedef struct icrs_hybrid_config {
  int32_t n_check;  /* 4..64 */
  int32_t reserved;
  double guard;     /* >= 1 */
  double tol;
  double vary_max;
} icrs_hybrid_config;

#define ICRS_ST_POINT 2048u /* the epoch took the point-source magnification (hybrid curve) */

void icrs_default_hybrid_config(icrs_hybrid_config* hc);
/* Workspace of icrs_magnification_hybrid (device, 256-byte aligned). */
size_t icrs_hybrid_workspace_bytes(const icrs_handle* h, int64_t n_events, int64_t n_epochs);
/* Hybrid light curves.  Inputs and outputs as for icrs_magnification; workspace of
 * icrs_hybrid_workspace_bytes().  The extended epochs' list size stays on the device (no
 * host wait).  Final sectors can be read with icrs_get_sectors() (0 sectors for point
 * epochs), as the input of icrs_hybrid_vjp. */
icrs_status icrs_magnification_hybrid(icrs_handle* h, int64_t n_events, const double* params,
                                      const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                      const icrs_hybrid_config* hc, double* mag, uint32_t* status,
                                      void* workspace, size_t workspace_bytes);
/* Point-source magnification of every epoch's source centre and its derivatives: a_ps
 * [n_epochs] (DEVICE, may be NULL), jac [n_epochs][ICRS_N_PARAMS] (DEVICE) = dA_ps/dparams
 * through the images (Sec. 3.5's implicit root derivative, taken on eq. lens_eq, whose
 * solutions are the validated roots), status [n_epochs] (DEVICE, may be NULL) the image-
 * finding bits.  rho and u_ld columns are 0.  Workspace as for icrs_magnification. */
icrs_status icrs_point_jacobian(icrs_handle* h, int64_t n_events, const double* params,
                                const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                                double* a_ps, double* jac, uint32_t* status, void* workspace,
                                size_t workspace_bytes);
/* Grid-free reference magnification (Sec. 2.2: the finite-source magnification is the
 * brightness-weighted mean of the point-source magnification, eq. amp_point, over the source
 * disk), for checking and tuning the ray quadrature's accuracy.  n_x Gauss-Legendre nodes in
 * x on [0, pi/2] with r = sin x (1 <= n_x <= 64) times n_phi midpoint angles (1 <= n_phi <=
 * 4096) per epoch, each a point-source solve in FP64 started from the centre's roots, linear
 * limb darkening.  The mean is a valid quadrature only while no caustic crosses the disk:
 * count_changes[e] counts the nodes whose image count differs from the centre's or whose solve
 * set a status bit (plus one when the centre's solve did); use mag[e] only where it is 0.  Events and epochs as for
 * icrs_magnification (params/epoch_offsets host, t device); mag [n_epochs] float64 and
 * count_changes [n_epochs] int32 are device arrays written on the handle's stream; workspace
 * as for icrs_magnification (icrs_workspace_bytes).  Cost: n_x n_phi point-source solves per
 * epoch.  Errors: EINVAL (bad sizes or pointers), ENOMEM (workspace too small). */
icrs_status icrs_disk_magnification(icrs_handle* h, int64_t n_events, const double* params,
                                    const int64_t* epoch_offsets, int64_t n_epochs, const double* t, int n_x,
                                    int n_phi, double* mag, int32_t* count_changes, void* workspace,
                                    size_t workspace_bytes);

/* Reverse mode of the hybrid curve: status (DEVICE [n_epochs]) from the forward call selects
 * the rule per epoch -- ICRS_ST_POINT epochs are differentiated through their images, the
 * others on their frozen sectors (as icrs_magnification_vjp; point epochs must have
 * n_sectors 0, as the forward leaves them).  cotangent, grad, jac as for
 * icrs_magnification_vjp (grad needs cotangent; at least one of grad, jac).  Workspace as
 * for icrs_magnification. */
icrs_status icrs_hybrid_vjp(icrs_handle* h, int64_t n_events, const double* params,
                            const int64_t* epoch_offsets, int64_t n_epochs, const double* t,
                            const uint32_t* status, const double* sectors, const uint8_t* periodic,
                            const int32_t* n_sectors, const double* cotangent, double* grad, double* jac,
                            void* workspace, size_t workspace_bytes);

/* ---- marginalised light-curve likelihood (App. B, eq. NLL) ------------------------------
 * Each event is one data set: fluxes F = (A - 1) F_S + F_base with independent Gaussian noise
 * sigma, and a Gaussian prior on the linear parameters beta = (F_S, F_base) with mean
 * (mu_S, mu_B) and standard deviations (sigma_S, sigma_B).  Marginalising beta gives
 *   NLL = 1/2 r^T (C + M Lambda M^T)^{-1} r + 1/2 ln |C + M Lambda M^T|,  r = F - M mu,
 * M = [A - 1, 1], evaluated through the appendix's Woodbury forms (the constant n/2 ln 2 pi
 * is left out, as in eq. NLL).  mag, flux, sigma: DEVICE [n_epochs]; epoch_offsets: HOST
 * [n_events + 1] CSR as elsewhere; prior: HOST [n_events][4] = (mu_S, mu_B, sigma_S,
 * sigma_B), sigma_S, sigma_B > 0.  Outputs (DEVICE): nll [n_events]; beta [n_events][5]
 * (may be NULL) = posterior mean (F_S, F_base) and covariance (SS, SB, BB); dnll_dmag
 * [n_epochs] (may be NULL) = dNLL/dA per epoch, the cotangent for icrs_magnification_vjp
 * or icrs_hybrid_vjp.  Workspace: DEVICE, icrs_marginal_nll_workspace_bytes(n_events). */
size_t icrs_marginal_nll_workspace_bytes(int64_t n_events);
icrs_status icrs_marginal_nll(icrs_handle* h, int64_t n_events, const int64_t* epoch_offsets, int64_t n_epochs,
                              const double* mag, const double* flux, const double* sigma, const double* prior,
                              double* nll, double* beta, double* dnll_dmag, void* workspace,
                              size_t workspace_bytes);

const char* icrs_status_string(icrs_status s);

#ifdef __cplusplus
}
#endif
#endif /* ICRS_H_ */
