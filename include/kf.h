/*
 * kf.h - C ABI of the keyframe depth-update library (gfx950 / MI355X).
 *
 * The library keeps one keyframe's depth state resident in device memory and
 * updates it with every new frame, as in DeepFusion (Laidlow, Czarnowski,
 * Leutenegger, arxiv 2207.12244):
 *   - semi-dense estimation (Sec. II-B): per textured keyframe pixel, an SSD
 *     search along the epipolar line of the new frame, interpolation between
 *     two steps, the variance (J^T J)^-1 of eq. (semi), and an inverse-depth
 *     Gaussian filter;
 *   - optimisation (Sec. II-C): the cost c(d, s) = c_semi + c_net + c_grad with
 *     Huber on every term, minimised by Gauss-Newton iterations that alternate
 *     between the log-depth map and the scale, the depth step solved with
 *     Jacobi-preconditioned conjugate gradients on the grid's 5-point system.
 *
 * Conventions
 *   - Images and maps are H x W, row-major, pixel i = v * W + u; integer pixel
 *     coordinates are pixel centres; depth is z-depth.
 *   - Device pointers are hipMalloc'd (or torch) memory on the context's
 *     device. Host pointers are marked "host".
 *   - Poses are host double[16], row-major 4x4 camera-to-world SE(3) matrices
 *     T_WC; they are copied at call time.
 *   - Map element type follows cfg.precision: KF_F64 -> double, otherwise
 *     float. Images are always uint8 grey levels.
 *   - Every call except kf_read_depth, kf_read_stats, kf_export_state and
 *     kf_import_state only enqueues work on cfg.stream and returns; those four
 *     synchronise the stream before returning.
 *   - Ownership: the caller owns the workspace and every buffer passed in.
 *     kf_set_prior copies the image and priors into the workspace (they may be
 *     freed once the stream has passed the call); image1 of kf_fuse_frame must
 *     stay alive until the stream has passed that call.
 *   - Errors: a call returns KF_OK or a negative kf_status and never throws.
 *     Argument and state errors are detected on the host before any device
 *     work is enqueued. Input errors found on the device (non-finite values,
 *     variances <= 0) and a solver synchronisation timeout raise a device flag
 *     that the next synchronising call returns (KF_ERR_INPUT, KF_ERR_TIMEOUT).
 *     kf_last_error gives a message for the last failure on the context.
 *   - Threading: a context is externally synchronised; distinct contexts are
 *     independent (each has its own workspace).
 */
#ifndef KF_H
#define KF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kf_ctx kf_ctx;

typedef enum {
  KF_OK = 0,
  KF_ERR_ARG = -1,      /* invalid argument or configuration */
  KF_ERR_OOM = -2,      /* workspace too small */
  KF_ERR_HIP = -3,      /* a HIP runtime call failed (message in kf_last_error) */
  KF_ERR_STATE = -4,    /* call out of order (e.g. kf_fuse_frame before kf_set_prior) */
  KF_ERR_INPUT = -5,    /* device found a non-finite input or a variance <= 0 */
  KF_ERR_TIMEOUT = -6   /* a solver workgroup waited too long for its team (never expected) */
} kf_status;

/* Storage / arithmetic form. */
typedef enum {
  KF_F64 = 0,       /* double maps, double arithmetic, double images */
  KF_F32 = 1,       /* float maps and arithmetic, float images */
  KF_BF16_F32 = 2   /* float maps and arithmetic; keyframe image and patch buffers bf16 */
} kf_precision;

/* The optimisation of Sec. II-C, or one of the two ablations of Sec. III. */
typedef enum {
  KF_VARIANT_FULL = 0,          /* c_semi + c_net + c_grad, alternating depth and scale (Sec. II-C) */
  KF_VARIANT_NO_PAIRWISE = 1,   /* Table III: no gradient (pairwise) terms; each depth step is the
                                   per-pixel weighted mean of the network and semi-dense log-depths */
  KF_VARIANT_SCALE_POSTFIT = 2  /* Table II: a scale-ambiguous log-depth y from c_semi + c_grad alone
                                   (scale held fixed), then the least-squares fit of the scale to the
                                   network log-depth, tau = mean(mu - y) over all pixels, x = y + tau;
                                   gradient variances must be finite */
} kf_variant;

/* Robust cost on every term's whitened residual r (Sec. II-C uses Huber; Sec. V
   names Tukey's biweight as the alternative to try). Both use huber_delta as the
   threshold c. */
typedef enum {
  KF_ROBUST_HUBER = 0,   /* IRLS weight min(1, c / |r|) */
  KF_ROBUST_TUKEY = 1    /* IRLS weight (1 - (r/c)^2)^2 for |r| <= c, 0 beyond (non-convex: a term far
                            off is ignored; a pixel whose every term is ignored keeps its value) */
} kf_robust;

/* Matching pattern of the epipolar search (Sec. II-B). */
typedef enum {
  KF_PAT_LINE5 = 0, /* five points, 1 px apart, along the epipolar lines of both images */
  KF_PAT_SQ5X5 = 1  /* 5x5 square patch, translation-only warp */
} kf_pattern;

typedef struct {
  int32_t width, height;        /* keyframe size; 8 <= width, height <= 8192 */
  double fx, fy, cx, cy;        /* pinhole intrinsics K */
  int32_t n_samples;            /* epipolar samples per pixel: a power of two in [4, 1024] */
  int32_t pattern;              /* kf_pattern */
  int32_t n_gn;                 /* Gauss-Newton iterations per frame (paper: 10), >= 1 */
  int32_t n_cg;                 /* PCG iterations per GN iteration when cg_rtol == 0, >= 1 */
  double cg_rtol;               /* > 0: PCG until ||r|| <= cg_rtol ||b||, at most cg_max */
  int32_t cg_max;               /* cap of the tolerance mode, >= 1 */
  int32_t cg_variant;           /* 0 automatic (pipelined when cg_rtol == 0), 1 textbook PCG,
                                   2 pipelined PCG: same iterates in exact arithmetic, one team
                                   synchronisation per iteration instead of two */
  double huber_delta;           /* threshold c of the robust cost on whitened residuals (> 0; INFINITY
                                   gives plain least squares with Huber) */
  double d_near, d_far;         /* depth range of a full-line search, 0 < d_near < d_far */
  double grad_gate;             /* texture gate: |grad I0| >= grad_gate grey levels per pixel */
  double sigma_photo;           /* photometric noise (grey levels) in eq. (semi), > 0 */
  double r_floor;               /* floor of the log-space semi-dense variance, > 0 */
  int32_t precision;            /* kf_precision */
  int32_t solver_tiles_x;       /* solver workgroup grid (0, 0 = automatic) */
  int32_t solver_tiles_y;
  int32_t solver_threads;       /* threads per solver workgroup: 0 = automatic, 256, 512 or 1024 */
  int32_t solver_cooperative;   /* 1: hipLaunchCooperativeKernel; 0: plain launch whose grid is
                                   checked against the device's co-resident capacity */
  int32_t pipeline_frames;      /* 1: the solve runs on a second, internal stream and the filter state
                                   is double-buffered, so the next frame's stereo update overlaps the
                                   current frame's solve (same results); 0: one stream. A context with
                                   1 cannot join a batch. */
  int32_t variant;              /* kf_variant (default KF_VARIANT_FULL) */
  int32_t robust;               /* kf_robust (default KF_ROBUST_HUBER) */
  double lambda_trans;          /* Sec. II keyframe rule: a frame whose camera centre is more than
                                   lambda_trans (pose units) from the keyframe's asks for a new
                                   keyframe; 0 disables the test */
  int32_t lambda_inliers;       /* ... or whose semi-dense update produced fewer than lambda_inliers
                                   measurements ("inliers"); 0 disables the test. A frame that asks
                                   for a new keyframe updates the semi-dense filter but is not fused:
                                   the depth map keeps its last fused state, and
                                   kf_frame_stats.new_keyframe reports why (the caller creates the
                                   new keyframe with kf_set_prior and the network's outputs) */
  double solver_timeout_ms;     /* longest a solver workgroup waits for its team before the whole
                                   team gives up and flags KF_ERR_TIMEOUT (0 = default 2000 ms).
                                   After a timeout the state is undefined: call kf_set_prior. */
  void* stream;                 /* hipStream_t the context enqueues on (NULL = null stream) */
  void* workspace;              /* device buffer of at least kf_workspace_bytes(cfg) bytes */
  size_t workspace_bytes;
} kf_config;

/* Per-frame statistics, valid after kf_read_stats. */
typedef struct {
  int32_t n_searched;       /* textured pixels searched by the last stereo update */
  int32_t n_updated;        /* of which produced a measurement ("inliers", Sec. II) */
  int32_t n_valid;          /* pixels with a semi-dense estimate after the last solve */
  int32_t cg_iterations;    /* PCG iterations of the last solve, summed over GN iterations */
  double scale;             /* s = exp(tau) after the last solve */
  double cg_rel_residual;   /* ||r|| / ||b|| at the end of the last PCG solve (tolerance mode) */
  int32_t team_syncs;       /* team synchronisations of the last solver launch (or probe) */
  int32_t new_keyframe;     /* KF_NEW_KEYFRAME_* bits of the last frame (0: it was fused) */
} kf_frame_stats;

#define KF_NEW_KEYFRAME_TRANSLATION 1   /* camera centre moved more than lambda_trans */
#define KF_NEW_KEYFRAME_INLIERS 2       /* fewer than lambda_inliers semi-dense measurements */

/* Fills *cfg with the defaults of the readings documented with the library:
   n_samples 32, LINE5, n_gn 10, n_cg 20, cg_rtol 0, cg_max 4000, huber 1.345,
   d_near 0.4, d_far 10, grad_gate 6, sigma_photo 1, r_floor 1e-6, KF_F32,
   fx = fy = 0.8 width, cx = width / 2, cy = height / 2. */
void kf_config_default(kf_config* cfg, int32_t width, int32_t height);

/* Device bytes a context with this configuration needs; 0 if cfg is invalid. */
size_t kf_workspace_bytes(const kf_config* cfg);

/* Validates cfg and binds the workspace. No device work. *out = NULL on error.
   The paper defines no such call (it runs one keyframe at a time); the context
   is this library's unit of resident state. cfg and the workspace are the
   caller's; the context keeps a copy of cfg and a pointer to the workspace,
   which must outlive it. */
kf_status kf_create(const kf_config* cfg, kf_ctx** out);

/* Frees the host-side context (not the workspace). NULL is allowed. */
void kf_destroy(kf_ctx* ctx);

/* Message of the last failure on ctx ("" if none); static text if ctx is NULL. */
const char* kf_last_error(const kf_ctx* ctx);

/* Name of a status code. */
const char* kf_status_string(int32_t status);

/* New keyframe (Sec. II): the keyframe image (device uint8, H x W), the network's
   log-depth and its variance, the x / y log-depth gradients and their variances
   (device, map element type), and the keyframe pose (host double[16]).
   Resets the state: log-depth x := prior log-depth, scale := 1, semi-dense filter
   empty; computes the texture mask (grad_gate, 2-pixel border). */
kf_status kf_set_prior(kf_ctx* ctx, const uint8_t* image0,
                       const void* logdepth, const void* logdepth_var,
                       const void* grad_x, const void* grad_x_var,
                       const void* grad_y, const void* grad_y_var,
                       const double T_wc0[16]);

/* kf_set_prior from the network's outputs at the network's own resolution
   (Sec. II-A: the network's inputs and outputs are 256 x 192). The six maps are
   net_width x net_height (device, map element type, >= 2 x 2), in kf_set_prior's
   order. They are resampled to the keyframe size bilinearly, with pixel centres
   aligned: keyframe pixel u samples the network map at (u + 1/2) net_width /
   width - 1/2, clamped. The network's log-depth is normalised by the focal length
   of the camera it was trained with, so the log-depth is shifted by
   ln(fx net_width / width / focal_ref): focal_ref is that training focal length in
   pixels at the network's resolution, and fx net_width / width is this camera's
   at the same resolution. The gradients are per network pixel; they are
   rescaled to keyframe pixels by net_width / width (x) and net_height / height
   (y), and their variances by the squares. The log-depth variance is resampled
   unchanged (the paper scales neither gradients nor uncertainties by the focal
   length). The maps may be freed once the stream has passed the call.
   KF_ERR_ARG for a NULL map, a network size outside [2, 8192] or a focal_ref
   that is not finite and > 0. */
kf_status kf_set_prior_network(kf_ctx* ctx, const uint8_t* image0,
                               const void* logdepth, const void* logdepth_var,
                               const void* grad_x, const void* grad_x_var,
                               const void* grad_y, const void* grad_y_var,
                               int32_t net_width, int32_t net_height, double focal_ref,
                               const double T_wc0[16]);

/* Semi-dense update only (Sec. II-B) with a new frame (device uint8 image, host pose). */
kf_status kf_stereo_update(kf_ctx* ctx, const uint8_t* image1, const double T_wc1[16]);

/* Optimisation only (Sec. II-C): n_gn Gauss-Newton iterations from the current state. */
kf_status kf_solve(kf_ctx* ctx);

/* The per-frame update of Sec. II: the semi-dense update of Sec. II-B (epipolar
   search, interpolation between two steps, variance of eq. (semi), inverse-depth
   filter) followed by the optimisation of Sec. II-C (c_semi + c_net + c_grad with
   Huber terms, n_gn Gauss-Newton iterations alternating depth and scale, warm
   started from the current state). Same as kf_stereo_update then kf_solve.
   image1: device uint8, H x W, row-major, owned by the caller, alive until the
   stream has passed this call; T_wc1: host double[16], copied. Returns
   KF_ERR_STATE before kf_set_prior, KF_ERR_ARG for a NULL image or a pose that is
   not finite or has a last row other than 0 0 0 1. */
kf_status kf_fuse_frame(kf_ctx* ctx, const uint8_t* image1, const double T_wc1[16]);

/* The result of Sec. II-C: the keyframe depth map d = exp(x) (x = ln d is the
   optimised log-depth) and the scale s = exp(tau) of the semi-dense term.
   Writes depth (device, H x W, map element type, caller-owned) and, if var_out is
   not NULL, the inverse-depth filter variance of Sec. II-B (0 where no estimate);
   *scale_out (host, nullable) receives s. Synchronises the stream; returns a
   pending device error (KF_ERR_INPUT, KF_ERR_TIMEOUT) or KF_ERR_STATE before
   kf_set_prior. */
kf_status kf_read_depth(kf_ctx* ctx, void* depth_out, void* var_out, double* scale_out);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops and harnesses that forbid allocation): kf_fuse_frame
   with the same results, whose kernels take their scratch -- the staged new
   frame and the solver team's exchange words -- from a fixed array inside the
   library (4 MiB per device, held until the process ends) instead of the
   context's workspace. Allocates nothing and calls no allocating routine.
   KF_ERR_ARG if the keyframe needs more scratch than the array holds
   ((height + 1) x row stride of the staged frame, rows padded to a multiple of
   64 bytes >= width + 8, plus the exchange words: 640 x 480 needs 2.8 MB);
   KF_ERR_STATE before kf_set_prior or with pipeline_frames. Every call on a
   device shares that device's array and clears what must start at zero, so
   calls that overlap on one device (contexts on different streams) race. */
kf_status kf_fuse_frame_static(kf_ctx* ctx, const uint8_t* image1, const double T_wc1[16]);

/* Statistics of the last stereo update and solve (host struct). Synchronises. */
kf_status kf_read_stats(kf_ctx* ctx, kf_frame_stats* out);

/* Measurement aid, not part of the method: enqueues on cfg.stream one launch
   of the solver's workgroup team (same tiling, workgroup size and exchange
   words as kf_solve) that makes `rounds` team synchronisations of the kind one
   pipelined PCG iteration makes (`nvalues` inner-product partials, 1..3, plus
   the tile boundary of the stencil operand) and no arithmetic. The caller times
   it (events on cfg.stream); time / rounds is the synchronisation latency that
   bounds the solve. rounds in [1, 20000]. KF_ERR_STATE before kf_set_prior or
   with pipeline_frames; the resident depth state is not touched. */
kf_status kf_probe_sync(kf_ctx* ctx, int32_t rounds, int32_t nvalues);

/* The internal stream the solves run on when cfg.pipeline_frames = 1 (NULL
   otherwise), for callers that time or order work against the solve. */
void* kf_solve_stream(const kf_ctx* ctx);

/* Solver decomposition chosen for ctx: tiles_x, tiles_y, tile_w, tile_h, threads. */
kf_status kf_solver_layout(const kf_ctx* ctx, int32_t out[5]);

/* Copies the resident state out (device buffers, each nullable): log-depth x,
   inverse depth rho and its variance (0 = no estimate), the last match index per
   pixel (int32: -2 = not textured, -1 = searched without a valid sample), and
   tau = ln s (host). Synchronises. */
kf_status kf_export_state(kf_ctx* ctx, void* x, void* rho, void* rho_var, int32_t* match,
                          double* tau);

/* Overwrites parts of the resident state (device buffers, each nullable; tau
   host, nullable). Requires kf_set_prior first. Synchronises. */
kf_status kf_import_state(kf_ctx* ctx, const void* x, const void* rho, const void* rho_var,
                          const double* tau);

/* ------------------------------------------------------------------ batched form

   A batch fuses one new frame into each of n keyframe contexts (the per-frame
   update of Sec. II-B and II-C, unchanged) with three launches for the whole
   batch: frame staging, stereo over the union of the keyframes' textured
   pixels, and one persistent solver launch in which every keyframe's team of
   workgroups runs concurrently with the others. Each keyframe keeps its own
   tiling, so a member's results are bit-identical to kf_fuse_frame on it. */

typedef struct kf_batch kf_batch;

#define KF_BATCH_MAX_MEMBERS 256

typedef struct {
  void* stream;            /* hipStream_t; every member context must use this stream */
  int32_t use_graph;       /* 1 (default): replay the launches from one captured HIP graph; 0: direct launches */
  void* workspace;         /* device buffer of at least kf_batch_workspace_bytes bytes, 256-byte aligned */
  size_t workspace_bytes;
} kf_batch_config;

/* Defaults: stream 0, use_graph 1, no workspace. */
void kf_batch_config_default(kf_batch_config* cfg);

/* Device bytes the batch of these n member contexts (host array) needs; 0 if invalid. */
size_t kf_batch_workspace_bytes(kf_ctx* const* members, int32_t n);

/* Binds n distinct contexts (1 <= n <= KF_BATCH_MAX_MEMBERS). Members must share
   precision, pattern, n_samples, the solver workgroup size and CG variant, the
   device and cfg->stream, and run without pipeline_frames; they may differ in
   size, intrinsics, tiling and iteration counts. Schedules the solver teams, uploads the static tables and
   (use_graph) captures the graph; allocates two small pinned host buffers.
   KF_ERR_ARG if the members are incompatible or a team cannot be co-resident.
   Members must outlive the batch; they stay usable on their own between
   batch calls. *out = NULL on error. */
kf_status kf_batch_create(kf_ctx* const* members, int32_t n, const kf_batch_config* cfg, kf_batch** out);

/* One frame for every member: images is a host array of n device uint8 images
   (member i's H x W), poses a host array of n row-major 4 x 4 T_WC (n x 16
   doubles). Every member needs a prior (kf_set_prior). Enqueues work only; the
   results are read per member (kf_read_depth, kf_read_stats), which also
   report device errors. Blocks the host only while the descriptor buffer it
   reuses (that of the call before last) is still being uploaded. */
kf_status kf_batch_fuse(kf_batch* batch, const uint8_t* const* images, const double* poses);

/* kf_batch_fuse for a subset: members[0 .. n_active) are distinct member
   indices (host int32, positions in the array given to kf_batch_create), and
   images / poses hold one entry per listed member, in that order. Members not
   listed are left untouched. n_active = 0 is a no-op. This is the call a
   serving loop makes with whichever streams have a frame ready. */
kf_status kf_batch_fuse_subset(kf_batch* batch, int32_t n_active, const int32_t* members,
                               const uint8_t* const* images, const double* poses);

/* The two halves of kf_batch_fuse, for callers that time or interleave them:
   the stereo update of every member (staging + stereo launches), and the
   optimisation of every member (the persistent solver launch). Same
   arguments, conditions and results as the corresponding parts of
   kf_batch_fuse. */
kf_status kf_batch_stereo_update(kf_batch* batch, const uint8_t* const* images, const double* poses);
kf_status kf_batch_solve(kf_batch* batch);

/* Solver launch of the batch: workgroups, threads per workgroup, pixels per
   thread, and the longest per-workgroup team queue. */
kf_status kf_batch_layout(const kf_batch* batch, int32_t out[4]);

/* Message of the last failure on the batch ("" if none). */
const char* kf_batch_last_error(const kf_batch* batch);

/* Waits for the batch's pending descriptor uploads and frees its host state
   (not the workspace, not the members). NULL is allowed. */
void kf_batch_destroy(kf_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* KF_H */
