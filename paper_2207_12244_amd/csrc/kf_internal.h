// Internal declarations of the keyframe depth-update library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>

#include "kf.h"

namespace kf {

// Global address space. Pointers loaded from memory (argument tables) are
// generic to the compiler, which then emits flat instructions: those also
// count against the LDS wait counter, so every LDS wait would drain the
// outstanding global accesses too. Kernels convert their buffer pointers once.
// (The qualifier only exists in the device pass of the single-source build.)
#if defined(__HIP_DEVICE_COMPILE__)
#define KF_GLOBAL __attribute__((address_space(1)))
#else
#define KF_GLOBAL
#endif
template <typename P>
__device__ inline KF_GLOBAL P* gp(P* p) { return (KF_GLOBAL P*)p; }

// ------------------------------------------------------------------ storage types

// bfloat16 stored as its 16 raw bits; conversions round to nearest even.
struct bf16 {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16 h) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)h.bits << 16;
  return c.f;
}

__host__ __device__ inline bf16 float_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t u = c.u;
  bf16 h;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    h.bits = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    h.bits = (uint16_t)(u >> 16);
  }
  return h;
}

template <typename TI, typename T> __device__ inline T load_img(const TI* p, size_t i);
template <> __device__ inline double load_img<double, double>(const double* p, size_t i) { return p[i]; }
template <> __device__ inline float load_img<float, float>(const float* p, size_t i) { return p[i]; }
template <> __device__ inline float load_img<bf16, float>(const bf16* p, size_t i) { return bf16_to_float(p[i]); }

// Value of one stored image element in the arithmetic type.
__device__ inline double img_value(double v) { return v; }
__device__ inline float img_value(float v) { return v; }
__device__ inline float img_value(bf16 v) { return bf16_to_float(v); }

template <typename TI, typename T> __device__ inline TI to_img(T v);
template <> __device__ inline double to_img<double, double>(double v) { return v; }
template <> __device__ inline float to_img<float, float>(float v) { return v; }
template <> __device__ inline bf16 to_img<bf16, float>(float v) { return float_to_bf16(v); }

// v rounded to the storage type TI and read back (identity for float/double storage).
template <typename TI, typename T> __device__ inline T round_to_img(T v) {
  const TI s = to_img<TI, T>(v);
  return load_img<TI, T>(&s, 0);
}

// Form traits: T = map and arithmetic type, TI = keyframe image / patch storage type.
template <int PREC> struct Form;
template <> struct Form<KF_F64> { using T = double; using TI = double; };
template <> struct Form<KF_F32> { using T = float; using TI = float; };
template <> struct Form<KF_BF16_F32> { using T = float; using TI = bf16; };

// ------------------------------------------------------------------ device scalars block

// Device-side counters and flags (one 256-byte block in the workspace).
struct DevScalars {
  double tau;             // ln s
  double cg_rel_residual;
  double frame_trans[2];  // camera-centre distance of the frame behind filter-state buffer b from the keyframe
  int32_t mask_count;     // textured pixels (length of the search list)
  int32_t n_updated[2];   // measurements of the stereo update that wrote filter-state buffer b
  int32_t n_valid;        // pixels with a filter estimate (computed by the solver)
  int32_t cg_iterations;
  int32_t err;            // bit flags, ERR_*
  uint32_t epoch;         // next synchronisation epoch of the solver team (never 0)
  int32_t team_syncs;     // team synchronisations of the last solve
  int32_t new_keyframe;   // KF_NEW_KEYFRAME_* bits of the last solve (0: fused)
};
static_assert(sizeof(DevScalars) <= 256, "device scalars take one 256-byte block of the workspace");
enum : int32_t { ERR_INPUT = 1, ERR_TIMEOUT = 2 };

// ------------------------------------------------------------------ workspace layout

struct Layout {
  size_t i0, list, chunk, prior, x, rho, var, rho2, var2, match, i1s, scal, parts, halo, total;
  size_t elt;       // sizeof(T)
  size_t elt_img;   // sizeof(TI)
};

// Solver decomposition: tiles_x x tiles_y workgroups, each owning one tile.
struct Tiling {
  int tiles_x, tiles_y, tile_w, tile_h, blocks, ppt, threads;
};

constexpr int NV_MAX = 3;            // values reduced per synchronisation
constexpr int PART_REPLICAS = 8;     // copies of each published partial (readers spread over them)
constexpr int MAX_TEAM = 256;        // workgroups per keyframe team
constexpr int CHUNK = 256;           // pixels per compaction chunk
#define KF_BATCH_MAX KF_BATCH_MAX_MEMBERS

bool choose_tiling(int W, int H, int tx_req, int ty_req, int threads_req, int prec, Tiling* t);
double iteration_us(const Tiling& t);   // latency model of one PCG iteration
// Workgroups of this tiling the device can hold at once (0 if unknown).
// kind: bit 0 pipelined CG, bit 1 the solver instantiation that handles the
// Sec. III variants and the keyframe rule (solve_kind)
int solve_max_coresident(int prec, const Tiling& t, int kind, int device);
bool layout_for(const kf_config& cfg, const Tiling& t, Layout* lay);
int stage_stride(int W);

// ------------------------------------------------------------------ kernel arguments

struct PriorArgs {
  int W, H;
  const uint8_t* image0;
  const void* mu; const void* var_n; const void* gx; const void* var_gx; const void* gy; const void* var_gy;
  void* i0;                  // TI[N]
  void* prior;               // T[6][N]: mu, isd_n, gx, isd_gx, gy, isd_gy (isd = 1/sigma)
  void* x; void* rho; void* var; int32_t* match;
  int32_t* chunk_counts;     // [nchunks + 1]
  int32_t* list;             // [N]
  DevScalars* scal;
  double grad_gate;
  int border;
};

struct ResampleArgs {        // network outputs at the network's size -> keyframe priors
  int W, H, Wn, Hn;
  const void* src[6];        // mu, var_mu, g_x, var_gx, g_y, var_gy (Wn x Hn, map element type)
  void* dst;                 // T[6][W H], same order
  double shift;              // ln(focal length at the network's size / reference focal length)
};

struct FrameConst {          // epipolar constants of one frame (host FP64)
  double Hm[9];              // K R K^-1
  double b[3];               // K t
  double e0[3];              // keyframe epipole K c1 (homogeneous)
  double rho_min, rho_max;
  double sigma_photo;
  double trans;              // |t|: distance between the two camera centres
};

struct StereoArgs {
  int W, H;
  const void* i0;            // TI[N]
  const uint8_t* i1;         // new frame (caller's buffer)
  uint8_t* i1s;              // new frame staged with padded rows (H + 1 rows of i1_stride bytes)
  int i1_stride;
  const int32_t* list;
  const DevScalars* scal_ro;
  DevScalars* scal;
  void* rho; void* var;       // filter state read
  void* rho_out; void* var_out;   // filter state written (== rho / var: in place)
  int32_t* match;
  int buf;                   // filter-state buffer written (its counters: n_updated[buf], frame_trans[buf])
  FrameConst fc;
};

struct SolveArgs {
  int W, H;
  int tiles_x, tiles_y, tile_w, tile_h;
  const void* prior;         // T[6][N]
  const void* rho; const void* var;
  void* x;
  DevScalars* scal;
  uint64_t* parts;           // [2][NV_MAX][PART_REPLICAS][blocks][2] exchange words
  uint64_t* halo;            // [2][blocks][2 perim][2]: first, then second row / column per side
  int perim;                 // 2 tile_w + 2 tile_h
  int ghost_z;               // 1: fixed-count pipelined CG on tiles >= 2 x 2 without the
                             // initial-residual synchronisation (x shipped two pixels deep)
  uint32_t epoch_span;       // epochs one launch may use (the base lives in DevScalars::epoch)
  int packed;                // 1: one-word partials (48-bit values, 16-bit epochs)
  int n_gn, n_cg, cg_max;
  int variant;               // kf_variant
  int robust;                // kf_robust
  int lambda_inliers;        // keyframe rule (0: off)
  int buf;                   // filter-state buffer read (the counters its stereo update wrote)
  double lambda_trans;       // keyframe rule (0: off)
  double cg_rtol;
  double huber_delta, r_floor;
  uint64_t timeout_ticks;    // wall-clock ticks a workgroup may wait for its team
};

struct ReadArgs {
  int N;
  const void* x; const void* var;
  void* depth_out; void* var_out;
};

struct ImportArgs {
  int N;
  const void* x; const void* rho; const void* var;
  void* dx; void* drho; void* dvar;
  DevScalars* scal;
};

// ------------------------------------------------------------------ launchers (return hipError_t)

hipError_t launch_prior(int prec, const PriorArgs& a, hipStream_t s);
hipError_t launch_resample_priors(int prec, const ResampleArgs& a, hipStream_t s);
// Staging + stereo update of one keyframe on `cus` compute units: as many
// workgroups as the device holds at once, or one per unit beside a running solve.
hipError_t launch_stereo(int prec, int pattern, int ns, const StereoArgs& a, int cus, bool beside_solve,
                         hipStream_t s);
// Batched stereo: the active count *n (device, <= nmax) and the table entries
// are read by the kernels, so the launches can be captured once.
hipError_t launch_stereo_batch(int prec, int pattern, int ns, const StereoArgs* tab, const int32_t* n, int nmax,
                               int cus, hipStream_t s);
hipError_t launch_solve(int prec, const Tiling& t, const SolveArgs& a, bool cooperative, int kind, hipStream_t s);
// Batched solver: workgroup g runs the team members queue[qoff[g] .. qoff[g+1])
// in order, each entry (keyframe << 8) | member; all `grid` workgroups must be
// co-resident.
hipError_t launch_solve_batch(int prec, int threads, int ppt, int kind, const SolveArgs* tab,
                              const int32_t* queue, const int32_t* qoff, int grid, size_t smem, hipStream_t s);
// Team-synchronisation probe on the layout of `a` (see k_sync_probe).
hipError_t launch_sync_probe(int prec, const Tiling& t, const SolveArgs& a, int rounds, int nv, hipStream_t s);
int solve_batch_coresident(int prec, int threads, int ppt, int kind, size_t smem, int device);
bool solve_batch_supported(int prec, int threads, int ppt);
hipError_t launch_read(int prec, const ReadArgs& a, hipStream_t s);
hipError_t launch_import(int prec, const ImportArgs& a, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);
size_t solve_smem_bytes(int prec, const Tiling& t);
// Compute units of the device (256 if the query fails).
int device_cus(int device);

}  // namespace kf

// Host state of one keyframe context (opaque to callers).
struct kf_ctx {
  kf_config cfg;
  kf::Tiling tiling;
  kf::Layout lay;
  hipStream_t stream;
  int device;
  uint32_t epoch;      // host mirror of the device-side epoch base
  uint32_t frame;
  bool has_prior;
  double T_wc0[16];
  std::string err;
  char* ws;
  uint64_t timeout_ticks;
  int cus;                    // compute units of the device (stereo grids)
  int coresident;      // workgroups of the solver tiling the device holds at once (-1: not checked)
  // frame pipelining (cfg.pipeline_frames): the solve runs on solve_stream, the
  // filter state alternates between two buffers, cur = the one the last stereo
  // update wrote (and the next solve reads)
  int cur = 0;
  hipStream_t solve_stream = nullptr;
  hipEvent_t ev_user = nullptr;           // user stream's tail when a solve is enqueued
  hipEvent_t ev_solve[2] = {nullptr, nullptr};   // last solve that read buffer b
  bool solve_pending[2] = {false, false};
  int last_solve = -1;                    // buffer of the last enqueued solve
  bool solves_waited = true;              // the user stream waits for every enqueued solve
};

namespace kf {

// Shared by the single-keyframe calls and the batched executor, so that both
// hand the kernels the same arguments.
bool pose_ok(const double* T);
bool stereo_args(kf_ctx* c, const uint8_t* image1, const double* T_wc1, StereoArgs* a);
uint32_t solve_epoch_bound(const kf_config& g);
bool solve_pipelined(const kf_config& g);
int solve_kind(const kf_config& g);
void solve_args(kf_ctx* c, SolveArgs* a);
hipError_t epoch_wrap_if_needed(kf_ctx* c, uint32_t bound);   // restart epochs before they could wrap

}  // namespace kf
