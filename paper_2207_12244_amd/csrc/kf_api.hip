// C ABI of the keyframe depth-update library: validation, workspace layout,
// per-frame epipolar constants (host FP64) and kernel launches.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "kf_internal.h"


namespace kf {

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Row stride of the staged new frame: >= W + 8 bytes (room for dword reads past
// the last pixel), a multiple of 64.
int stage_stride_impl(int W) { return ((W + 8 + 63) / 64) * 64; }

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

const char* validate(const kf_config& c) {
  if (c.width < 8 || c.height < 8 || c.width > 8192 || c.height > 8192) return "width/height must be in [8, 8192]";
  if (!finite_pos(c.fx) || !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
    return "intrinsics must be finite with fx, fy > 0";
  if (!is_pow2(c.n_samples) || c.n_samples < 4 || c.n_samples > 1024)
    return "n_samples must be a power of two in [4, 1024]";
  if (c.pattern != KF_PAT_LINE5 && c.pattern != KF_PAT_SQ5X5) return "pattern must be KF_PAT_LINE5 or KF_PAT_SQ5X5";
  if (c.n_gn < 1 || c.n_gn > 1000) return "n_gn must be in [1, 1000]";
  if (c.n_cg < 1 || c.n_cg > 100000) return "n_cg must be in [1, 100000]";
  if (!(c.cg_rtol >= 0.0) || !std::isfinite(c.cg_rtol)) return "cg_rtol must be finite and >= 0";
  if (c.cg_max < 1 || c.cg_max > 100000) return "cg_max must be in [1, 100000]";
  if (!(c.huber_delta > 0.0)) return "huber_delta must be > 0 (INFINITY allowed)";
  if (!finite_pos(c.d_near) || !finite_pos(c.d_far) || !(c.d_near < c.d_far)) return "need 0 < d_near < d_far";
  if (!(c.grad_gate >= 0.0) || !std::isfinite(c.grad_gate)) return "grad_gate must be finite and >= 0";
  if (!finite_pos(c.sigma_photo)) return "sigma_photo must be finite and > 0";
  if (!finite_pos(c.r_floor)) return "r_floor must be finite and > 0";
  if (c.precision != KF_F64 && c.precision != KF_F32 && c.precision != KF_BF16_F32) return "unknown precision";
  if ((c.solver_tiles_x == 0) != (c.solver_tiles_y == 0) || c.solver_tiles_x < 0 || c.solver_tiles_y < 0)
    return "solver_tiles_x/y must both be 0 (automatic) or both positive";
  if (c.solver_threads != 0 && c.solver_threads != 256 && c.solver_threads != 512 && c.solver_threads != 1024)
    return "solver_threads must be 0, 256, 512 or 1024";
  if (c.solver_cooperative != 0 && c.solver_cooperative != 1) return "solver_cooperative must be 0 or 1";
  if (c.pipeline_frames != 0 && c.pipeline_frames != 1) return "pipeline_frames must be 0 or 1";
  if (c.cg_variant < 0 || c.cg_variant > 2) return "cg_variant must be 0, 1 or 2";
  if (c.variant < KF_VARIANT_FULL || c.variant > KF_VARIANT_SCALE_POSTFIT) return "unknown variant";
  if (c.robust != KF_ROBUST_HUBER && c.robust != KF_ROBUST_TUKEY) return "unknown robust cost";
  if (c.robust == KF_ROBUST_TUKEY && !std::isfinite(c.huber_delta)) return "Tukey's threshold must be finite";
  if (!(c.lambda_trans >= 0.0) || !std::isfinite(c.lambda_trans)) return "lambda_trans must be finite and >= 0";
  if (c.lambda_inliers < 0) return "lambda_inliers must be >= 0";
  if (c.cg_variant == 2 && c.cg_rtol > 0.0) return "the pipelined CG variant runs a fixed iteration count (cg_rtol = 0)";
  if (!(c.solver_timeout_ms >= 0.0) || !std::isfinite(c.solver_timeout_ms) || c.solver_timeout_ms > 3.6e6)
    return "solver_timeout_ms must be in [0, 3.6e6]";
  return nullptr;
}

// Largest pixels-per-thread whose solver instantiation keeps every value in
// registers (VGPRs, or AGPRs as spill space for 256-thread workgroups).
int ppt_max(int prec, int threads) {
  if (prec == KF_F64) return threads == 256 ? 6 : (threads == 512 ? 4 : 1);
  return threads == 256 ? 8 : (threads == 512 ? 10 : 3);
}

int ppt_for(int px, int threads, int prec) {
  const int need = (px + threads - 1) / threads;
  static const int opts[] = {1, 2, 3, 4, 6, 8, 10};
  for (int o : opts)
    if (o >= need) return o <= ppt_max(prec, threads) ? o : 0;
  return 0;
}

bool tiling_ok(int W, int H, int tx, int ty, int threads, int prec, Tiling* t) {
  if (tx < 1 || ty < 1 || tx > W || ty > H || tx * ty > MAX_TEAM) return false;
  const int tw = (W + tx - 1) / tx, th = (H + ty - 1) / ty;
  if ((tx - 1) * tw >= W || (ty - 1) * th >= H) return false;   // no empty tiles
  if (tw + th > threads) return false;                          // ghost ring fits 2 slots per thread
  const int ppt = ppt_for(tw * th, threads, prec);
  if (ppt == 0) return false;
  t->tiles_x = tx;
  t->tiles_y = ty;
  t->tile_w = tw;
  t->tile_h = th;
  t->blocks = tx * ty;
  t->ppt = ppt;
  t->threads = threads;
  return true;
}

}  // namespace

// Latency model of one PCG iteration of a team (microseconds), fitted to
// MI355X measurements of the 640 x 480 solve (200-256 workgroups): ~1.27 us
// per synchronisation plus 4 ns per workgroup polled, and ~1.25 ns per tile
// pixel at 512 threads (1.45 at 1024, 2.4 at 256, whose single wavefront per
// SIMD hides little latency), with a small penalty for long tile perimeters.
double iteration_us(const Tiling& c) {
  const double per_px = c.threads == 256 ? 2.4e-3 : (c.threads == 512 ? 1.25e-3 : 1.45e-3);
  return 1.27 + 0.004 * c.blocks + (double)c.tile_w * c.tile_h * per_px + (c.tile_w + c.tile_h) * 1e-4;
}

// Picks the tile grid (and workgroup size, unless given) minimising iteration_us.
bool choose_tiling(int W, int H, int tx_req, int ty_req, int threads_req, int prec, Tiling* t) {
  const int thr_opts[3] = {512, 256, 1024};
  if (tx_req > 0 && ty_req > 0) {
    for (int nt : thr_opts) {
      if (threads_req && nt != threads_req) continue;
      if (tiling_ok(W, H, tx_req, ty_req, nt, prec, t)) return true;
    }
    return false;
  }
  double best = 1e300;
  Tiling bt{};
  bool found = false;
  for (int nt : thr_opts) {
    if (threads_req && nt != threads_req) continue;
    for (int tx = 1; tx <= 64 && tx <= W; ++tx) {
      for (int ty = 1; ty <= 64 && ty <= H; ++ty) {
        if (tx * ty > MAX_TEAM) break;
        Tiling c;
        if (!tiling_ok(W, H, tx, ty, nt, prec, &c)) continue;
        const double cost = iteration_us(c);
        if (cost < best) {
          best = cost;
          bt = c;
          found = true;
        }
      }
    }
  }
  if (found) *t = bt;
  return found;
}

int stage_stride(int W) { return stage_stride_impl(W); }

bool layout_for(const kf_config& c, const Tiling& t, Layout* L) {
  const size_t N = (size_t)c.width * c.height;
  const size_t elt = c.precision == KF_F64 ? 8 : 4;
  const size_t elt_img = c.precision == KF_F64 ? 8 : (c.precision == KF_F32 ? 4 : 2);
  const size_t nchunks = (N + CHUNK - 1) / CHUNK;
  size_t off = 0;
  L->elt = elt;
  L->elt_img = elt_img;
  L->i0 = off; off += align256(N * elt_img);
  L->list = off; off += align256(N * 4);
  L->chunk = off; off += align256((nchunks + 1) * 4);
  L->prior = off; off += align256(6 * N * elt);
  L->x = off; off += align256(N * elt);
  L->rho = off; off += align256(N * elt);
  L->var = off; off += align256(N * elt);
  // second filter-state buffer for frame pipelining (adjacent, cleared together)
  L->rho2 = off; off += c.pipeline_frames ? align256(N * elt) : 0;
  L->var2 = off; off += c.pipeline_frames ? align256(N * elt) : 0;
  L->match = off; off += align256(N * 4);
  L->i1s = off; off += align256((size_t)(c.height + 1) * stage_stride(c.width));
  L->scal = off; off += 256;
  L->parts = off; off += align256((size_t)2 * NV_MAX * PART_REPLICAS * t.blocks * 2 * 8);
  L->halo = off; off += align256((size_t)2 * t.blocks * 2 * (2 * t.tile_w + 2 * t.tile_h) * 2 * 8);
  L->total = off;
  return true;
}

}  // namespace kf

using namespace kf;

namespace {

kf_status fail(kf_ctx* ctx, kf_status s, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return s;
}

kf_status hip_fail(kf_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, KF_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

template <typename P>
P* ws_ptr(kf_ctx* c, size_t off) { return reinterpret_cast<P*>(c->ws + off); }

DevScalars* scal_ptr(kf_ctx* c) { return ws_ptr<DevScalars>(c, c->lay.scal); }

// Filter-state buffer b (b = 1 exists only with frame pipelining).
char* rho_buf(kf_ctx* c, int b) { return c->ws + (b ? c->lay.rho2 : c->lay.rho); }
char* var_buf(kf_ctx* c, int b) { return c->ws + (b ? c->lay.var2 : c->lay.var); }

// With frame pipelining: the user stream waits for the solves enqueued on the
// solve stream (they run in order, so waiting for the last one suffices).
hipError_t wait_solves(kf_ctx* c) {
  if (c->last_solve < 0) return hipSuccess;
  const hipError_t e = hipStreamWaitEvent(c->stream, c->ev_solve[c->last_solve], 0);
  if (e == hipSuccess) c->solves_waited = true;
  return e;
}

// General 4x4 inverse (Gauss-Jordan, partial pivoting), row-major.
bool inv4(const double* m, double* out) {
  double a[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) a[i][j] = j < 4 ? m[i * 4 + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int p = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
    if (a[p][c] == 0.0) return false;
    if (p != c)
      for (int j = 0; j < 8; ++j) std::swap(a[p][j], a[c][j]);
    const double d = a[c][c];
    for (int j = 0; j < 8; ++j) a[c][j] /= d;
    for (int r = 0; r < 4; ++r) {
      if (r == c) continue;
      const double f = a[r][c];
      if (f == 0.0) continue;
      for (int j = 0; j < 8; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[i * 4 + j] = a[i][j + 4];
  return true;
}

// Epipolar constants of the photometric error (Sec. II-B): [R|t] = T_WC1^-1 T_WC0,
// H = K R K^-1, b = K t, keyframe epipole K (-R^T t).
bool frame_constants(const kf_ctx* c, const double* T1, FrameConst* fc) {
  double T1i[16];
  if (!inv4(T1, T1i)) return false;
  double T[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += T1i[i * 4 + k] * c->T_wc0[k * 4 + j];
      T[i * 4 + j] = s;
    }
  const kf_config& g = c->cfg;
  const double K[9] = {g.fx, 0, g.cx, 0, g.fy, g.cy, 0, 0, 1};
  const double Ki[9] = {1.0 / g.fx, 0, -g.cx / g.fx, 0, 1.0 / g.fy, -g.cy / g.fy, 0, 0, 1};
  double R[9], t[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[i * 3 + j] = T[i * 4 + j];
    t[i] = T[i * 4 + 3];
  }
  double KR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += K[i * 3 + k] * R[k * 3 + j];
      KR[i * 3 + j] = s;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += KR[i * 3 + k] * Ki[k * 3 + j];
      fc->Hm[i * 3 + j] = s;
    }
  double c1[3];
  for (int i = 0; i < 3; ++i) {
    double s = 0.0, s2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      s += K[i * 3 + k] * t[k];
      s2 -= R[k * 3 + i] * t[k];
    }
    fc->b[i] = s;
    c1[i] = s2;
  }
  fc->trans = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += K[i * 3 + k] * c1[k];
    fc->e0[i] = s;
  }
  fc->rho_min = 1.0 / g.d_far;
  fc->rho_max = 1.0 / g.d_near;
  fc->sigma_photo = g.sigma_photo;
  return true;
}

}  // namespace

namespace kf {

bool pose_ok(const double* T) {
  if (!T) return false;
  for (int i = 0; i < 16; ++i)
    if (!std::isfinite(T[i])) return false;
  return T[12] == 0.0 && T[13] == 0.0 && T[14] == 0.0 && T[15] == 1.0;
}

bool stereo_args(kf_ctx* c, const uint8_t* image1, const double* T_wc1, StereoArgs* a) {
  if (!frame_constants(c, T_wc1, &a->fc)) return false;
  a->W = c->cfg.width;
  a->H = c->cfg.height;
  a->i0 = c->ws + c->lay.i0;
  a->i1 = image1;
  a->i1s = ws_ptr<uint8_t>(c, c->lay.i1s);
  a->i1_stride = stage_stride(c->cfg.width);
  a->list = ws_ptr<int32_t>(c, c->lay.list);
  a->scal_ro = scal_ptr(c);
  a->scal = scal_ptr(c);
  a->rho = rho_buf(c, c->cur);
  a->var = var_buf(c, c->cur);
  a->rho_out = a->rho;
  a->var_out = a->var;
  a->match = ws_ptr<int32_t>(c, c->lay.match);
  a->buf = c->cur;
  return true;
}

// Epochs one solver launch may consume: per GN iteration at most 2 per CG
// iteration plus the initial and the scale synchronisation, plus slack.
uint32_t solve_epoch_bound(const kf_config& g) {
  const uint64_t limit = g.cg_rtol > 0.0 ? (uint64_t)g.cg_max : (uint64_t)g.n_cg;
  return (uint32_t)((uint64_t)g.n_gn * (2 * limit + 2) + 2);
}

bool solve_pipelined(const kf_config& g) { return g.cg_variant == 2 || (g.cg_variant == 0 && g.cg_rtol == 0.0); }

int solve_kind(const kf_config& g) {
  const bool var = g.variant != KF_VARIANT_FULL || g.robust != KF_ROBUST_HUBER || g.lambda_trans > 0.0 ||
                   g.lambda_inliers > 0;
  return (solve_pipelined(g) ? 1 : 0) | (var ? 2 : 0);
}

void solve_args(kf_ctx* c, SolveArgs* a) {
  const kf_config& g = c->cfg;
  const uint32_t bound = solve_epoch_bound(g);
  a->W = g.width;
  a->H = g.height;
  a->tiles_x = c->tiling.tiles_x;
  a->tiles_y = c->tiling.tiles_y;
  a->tile_w = c->tiling.tile_w;
  a->tile_h = c->tiling.tile_h;
  a->prior = c->ws + c->lay.prior;
  a->rho = rho_buf(c, c->cur);
  a->var = var_buf(c, c->cur);
  a->x = c->ws + c->lay.x;
  a->scal = scal_ptr(c);
  a->parts = ws_ptr<uint64_t>(c, c->lay.parts);
  a->halo = ws_ptr<uint64_t>(c, c->lay.halo);
  a->perim = 2 * c->tiling.tile_w + 2 * c->tiling.tile_h;
  // the second-ring cells (perimeter + 4 corners) fit one slot per thread
  a->ghost_z = (solve_pipelined(g) && g.cg_rtol == 0.0 && c->tiling.tile_w >= 2 && c->tiling.tile_h >= 2 &&
                a->perim + 4 <= c->tiling.threads) ? 1 : 0;
  a->epoch_span = bound;
  a->packed = (g.precision != KF_F64 && bound < 30000) ? 1 : 0;
  a->n_gn = g.n_gn;
  a->n_cg = g.n_cg;
  a->cg_max = g.cg_max;
  a->variant = g.variant;
  a->robust = g.robust;
  a->lambda_inliers = g.lambda_inliers;
  a->buf = c->cur;
  a->lambda_trans = g.lambda_trans;
  a->cg_rtol = g.cg_rtol;
  a->huber_delta = g.huber_delta;
  a->r_floor = g.r_floor;
  a->timeout_ticks = c->timeout_ticks;
}

// c->epoch mirrors the device-side base (both advance by `bound` per launch);
// before the 32-bit epochs could wrap, clear the exchange words and restart at 1.
hipError_t epoch_wrap_if_needed(kf_ctx* c, uint32_t bound) {
  if ((uint64_t)c->epoch + bound < 0xfff00000ull) return hipSuccess;
  hipError_t e = launch_zero(c->ws + c->lay.parts, c->lay.total - c->lay.parts, c->stream);
  if (e == hipSuccess) e = launch_set_u32(&scal_ptr(c)->epoch, 1u, c->stream);
  if (e == hipSuccess) c->epoch = 1;
  return e;
}

}  // namespace kf

namespace {

// Scratch of kf_fuse_frame_static: the staged frame and the solver team's
// exchange words live here instead of the context's workspace. Each device
// holds its own copy for the life of the process; host code uses only the
// per-device address that hipGetSymbolAddress returns, never the symbol.
constexpr size_t KF_STATIC_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) unsigned char scratch[KF_STATIC_SCRATCH_BYTES];

constexpr int KF_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[KF_MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
hipError_t static_scratch(int device, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= KF_MAX_DEVICES) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

kf_status check_device_flags(kf_ctx* c) {
  DevScalars h;
  hipError_t e = hipMemcpyAsync(&h, scal_ptr(c), sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronising the stream");
  if (h.err & ERR_TIMEOUT) return fail(c, KF_ERR_TIMEOUT, "solver workgroups timed out waiting for their team");
  if (h.err & ERR_INPUT) return fail(c, KF_ERR_INPUT, "device found a non-finite input or a variance <= 0");
  return KF_OK;
}

}  // namespace


extern "C" {

void kf_config_default(kf_config* cfg, int32_t width, int32_t height) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->width = width;
  cfg->height = height;
  cfg->fx = cfg->fy = 0.8 * width;
  cfg->cx = width / 2.0;
  cfg->cy = height / 2.0;
  cfg->n_samples = 32;
  cfg->pattern = KF_PAT_LINE5;
  cfg->n_gn = 10;
  cfg->n_cg = 20;
  cfg->cg_rtol = 0.0;
  cfg->cg_max = 4000;
  cfg->huber_delta = 1.345;
  cfg->d_near = 0.4;
  cfg->d_far = 10.0;
  cfg->grad_gate = 6.0;
  cfg->sigma_photo = 1.0;
  cfg->r_floor = 1e-6;
  cfg->precision = KF_F32;
}

size_t kf_workspace_bytes(const kf_config* cfg) {
  if (!cfg || validate(*cfg)) return 0;
  Tiling t;
  if (!choose_tiling(cfg->width, cfg->height, cfg->solver_tiles_x, cfg->solver_tiles_y, cfg->solver_threads, cfg->precision, &t)) return 0;
  Layout L;
  layout_for(*cfg, t, &L);
  return L.total;
}

kf_status kf_create(const kf_config* cfg, kf_ctx** out) {
  if (!out) return KF_ERR_ARG;
  *out = nullptr;
  if (!cfg) return KF_ERR_ARG;
  if (validate(*cfg)) return KF_ERR_ARG;
  Tiling t;
  if (!choose_tiling(cfg->width, cfg->height, cfg->solver_tiles_x, cfg->solver_tiles_y, cfg->solver_threads, cfg->precision, &t)) return KF_ERR_ARG;
  Layout L;
  layout_for(*cfg, t, &L);
  if (!cfg->workspace) return KF_ERR_ARG;
  if (cfg->workspace_bytes < L.total) return KF_ERR_OOM;
  if (reinterpret_cast<uintptr_t>(cfg->workspace) % 256 != 0) return KF_ERR_ARG;
  kf_ctx* c = new (std::nothrow) kf_ctx();
  if (!c) return KF_ERR_OOM;
  c->cfg = *cfg;
  c->tiling = t;
  c->lay = L;
  c->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  c->ws = reinterpret_cast<char*>(cfg->workspace);
  c->epoch = 1;
  c->frame = 0;
  c->has_prior = false;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  int rate_khz = 100000;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device) != hipSuccess || rate_khz <= 0)
    rate_khz = 100000;
  const double timeout_ms = cfg->solver_timeout_ms > 0.0 ? cfg->solver_timeout_ms : 2000.0;
  c->timeout_ticks = (uint64_t)((double)rate_khz * timeout_ms);   // wall-clock ticks
  c->cus = device_cus(c->device);
  c->coresident = -1;
  if (cfg->pipeline_frames) {
    // the two streams' events order work on this device only (the host reads
    // results through the user stream), so they skip the system-scope fence
    const unsigned ev_flags = hipEventDisableTiming | hipEventDisableSystemFence;
    hipError_t e = hipStreamCreateWithFlags(&c->solve_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_user, ev_flags);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipEventCreateWithFlags(&c->ev_solve[b], ev_flags);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      kf_destroy(c);
      return KF_ERR_HIP;
    }
  }
  *out = c;
  return KF_OK;
}

void kf_destroy(kf_ctx* ctx) {
  if (!ctx) return;
  if (ctx->solve_stream) (void)hipStreamSynchronize(ctx->solve_stream);
  for (hipEvent_t ev : ctx->ev_solve)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->ev_user) (void)hipEventDestroy(ctx->ev_user);
  if (ctx->solve_stream) (void)hipStreamDestroy(ctx->solve_stream);
  delete ctx;
}

const char* kf_last_error(const kf_ctx* ctx) {
  if (!ctx) return "no context";
  return ctx->err.c_str();
}

const char* kf_status_string(int32_t s) {
  switch (s) {
    case KF_OK: return "KF_OK";
    case KF_ERR_ARG: return "KF_ERR_ARG";
    case KF_ERR_OOM: return "KF_ERR_OOM";
    case KF_ERR_HIP: return "KF_ERR_HIP";
    case KF_ERR_STATE: return "KF_ERR_STATE";
    case KF_ERR_INPUT: return "KF_ERR_INPUT";
    case KF_ERR_TIMEOUT: return "KF_ERR_TIMEOUT";
  }
  return "unknown status";
}

}  // extern "C"

namespace {

// New keyframe: clears the state, then (with `rs`) resamples the network's maps
// into the prior region and initialises from there in place, else initialises
// from the six caller maps.
kf_status set_prior_impl(kf_ctx* c, const uint8_t* image0, const void* const maps[6], const double* T_wc0,
                         const ResampleArgs* rs) {
  std::memcpy(c->T_wc0, T_wc0, sizeof(c->T_wc0));
  // exchange words and device scalars start from zero (epoch 0 is never used)
  hipError_t e = wait_solves(c);
  if (e == hipSuccess) e = launch_zero(c->ws + c->lay.scal, c->lay.total - c->lay.scal, c->stream);
  if (e == hipSuccess && c->lay.match > c->lay.rho2)   // second filter-state buffer
    e = launch_zero(c->ws + c->lay.rho2, c->lay.match - c->lay.rho2, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_set_prior (clear)");
  c->cur = 0;
  c->epoch = 1;
  PriorArgs a;
  a.W = c->cfg.width;
  a.H = c->cfg.height;
  a.image0 = image0;
  const void* src[6];
  const size_t N = (size_t)a.W * a.H;
  if (rs) {
    ResampleArgs r = *rs;
    r.W = a.W;
    r.H = a.H;
    r.dst = c->ws + c->lay.prior;
    e = launch_resample_priors(c->cfg.precision, r, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "kf_set_prior_network (resample)");
    for (int k = 0; k < 6; ++k) src[k] = c->ws + c->lay.prior + k * N * c->lay.elt;
  } else {
    for (int k = 0; k < 6; ++k) src[k] = maps[k];
  }
  a.mu = src[0]; a.var_n = src[1]; a.gx = src[2]; a.var_gx = src[3]; a.gy = src[4]; a.var_gy = src[5];
  a.i0 = c->ws + c->lay.i0;
  a.prior = c->ws + c->lay.prior;
  a.x = c->ws + c->lay.x;
  a.rho = rho_buf(c, 0);
  a.var = var_buf(c, 0);
  a.match = ws_ptr<int32_t>(c, c->lay.match);
  a.chunk_counts = ws_ptr<int32_t>(c, c->lay.chunk);
  a.list = ws_ptr<int32_t>(c, c->lay.list);
  a.scal = scal_ptr(c);
  a.grad_gate = c->cfg.grad_gate;
  a.border = 2;
  e = launch_prior(c->cfg.precision, a, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_set_prior");
  c->has_prior = true;
  c->err.clear();
  return KF_OK;
}

}  // namespace

extern "C" {

kf_status kf_set_prior(kf_ctx* c, const uint8_t* image0, const void* logdepth, const void* logdepth_var,
                       const void* grad_x, const void* grad_x_var, const void* grad_y, const void* grad_y_var,
                       const double T_wc0[16]) {
  if (!c) return KF_ERR_ARG;
  if (!image0 || !logdepth || !logdepth_var || !grad_x || !grad_x_var || !grad_y || !grad_y_var)
    return fail(c, KF_ERR_ARG, "kf_set_prior: NULL buffer");
  if (!pose_ok(T_wc0)) return fail(c, KF_ERR_ARG, "kf_set_prior: pose must be finite with last row 0 0 0 1");
  const void* maps[6] = {logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var};
  return set_prior_impl(c, image0, maps, T_wc0, nullptr);
}

kf_status kf_set_prior_network(kf_ctx* c, const uint8_t* image0, const void* logdepth, const void* logdepth_var,
                               const void* grad_x, const void* grad_x_var, const void* grad_y, const void* grad_y_var,
                               int32_t net_width, int32_t net_height, double focal_ref, const double T_wc0[16]) {
  if (!c) return KF_ERR_ARG;
  if (!image0 || !logdepth || !logdepth_var || !grad_x || !grad_x_var || !grad_y || !grad_y_var)
    return fail(c, KF_ERR_ARG, "kf_set_prior_network: NULL buffer");
  if (net_width < 2 || net_height < 2 || net_width > 8192 || net_height > 8192)
    return fail(c, KF_ERR_ARG, "kf_set_prior_network: network size must be in [2, 8192]");
  if (!(focal_ref > 0.0) || !std::isfinite(focal_ref))
    return fail(c, KF_ERR_ARG, "kf_set_prior_network: focal_ref must be finite and > 0");
  if (!pose_ok(T_wc0)) return fail(c, KF_ERR_ARG, "kf_set_prior_network: pose must be finite with last row 0 0 0 1");
  ResampleArgs r{};
  r.Wn = net_width;
  r.Hn = net_height;
  const void* maps[6] = {logdepth, logdepth_var, grad_x, grad_x_var, grad_y, grad_y_var};
  for (int k = 0; k < 6; ++k) r.src[k] = maps[k];
  r.shift = std::log(c->cfg.fx * ((double)net_width / c->cfg.width) / focal_ref);
  return set_prior_impl(c, image0, maps, T_wc0, &r);
}

kf_status kf_stereo_update(kf_ctx* c, const uint8_t* image1, const double T_wc1[16]) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_stereo_update before kf_set_prior");
  if (!image1) return fail(c, KF_ERR_ARG, "kf_stereo_update: NULL image");
  if (!pose_ok(T_wc1)) return fail(c, KF_ERR_ARG, "kf_stereo_update: pose must be finite with last row 0 0 0 1");
  StereoArgs a;
  if (!stereo_args(c, image1, T_wc1, &a)) return fail(c, KF_ERR_ARG, "kf_stereo_update: singular pose");
  hipError_t e = hipSuccess;
  const int nxt = c->cur ^ 1;
  if (c->cfg.pipeline_frames) {
    // read the state the last update wrote, write the other buffer, which the
    // solve before last may still be reading
    a.rho_out = rho_buf(c, nxt);
    a.var_out = var_buf(c, nxt);
    a.buf = nxt;
    if (c->solve_pending[nxt]) e = hipStreamWaitEvent(c->stream, c->ev_solve[nxt], 0);
  }
  // beside a solve still in flight the update takes one workgroup per compute
  // unit; with none in flight (the user stream waited for them all) the
  // resident grid
  const bool beside = c->cfg.pipeline_frames && !c->solves_waited;
  if (e == hipSuccess) e = launch_stereo(c->cfg.precision, c->cfg.pattern, c->cfg.n_samples, a, c->cus, beside, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_stereo_update");
  if (c->cfg.pipeline_frames) c->cur = nxt;
  ++c->frame;
  return KF_OK;
}

kf_status kf_solve(kf_ctx* c) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_solve before kf_set_prior");
  const kf_config& g = c->cfg;
  const uint32_t bound = solve_epoch_bound(g);
  hipError_t e = hipSuccess;
  // the epoch restart clears words the previous solve may still use
  if (g.pipeline_frames && (uint64_t)c->epoch + bound >= 0xfff00000ull) e = wait_solves(c);
  if (e == hipSuccess) e = epoch_wrap_if_needed(c, bound);
  if (e != hipSuccess) return hip_fail(c, e, "kf_solve (epoch wrap)");
  SolveArgs a;
  solve_args(c, &a);
  const int kind = solve_kind(g);
  if (c->coresident < 0) c->coresident = solve_max_coresident(g.precision, c->tiling, kind, c->device);
  if (c->coresident < c->tiling.blocks)
    return fail(c, KF_ERR_ARG, "solver tiling needs " + std::to_string(c->tiling.blocks) +
                               " co-resident workgroups, the device holds " + std::to_string(c->coresident));
  hipStream_t s = c->stream;
  if (g.pipeline_frames) {
    // the solve waits for everything enqueued on the user stream so far (this
    // frame's stereo update included), not the other way round
    s = c->solve_stream;
    e = hipEventRecord(c->ev_user, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_user, 0);
    if (e != hipSuccess) return hip_fail(c, e, "kf_solve (ordering)");
  }
  e = launch_solve(g.precision, c->tiling, a, g.solver_cooperative != 0, kind, s);
  if (e == hipSuccess && g.pipeline_frames) {
    e = hipEventRecord(c->ev_solve[c->cur], s);
    c->solve_pending[c->cur] = true;
    c->last_solve = c->cur;
    c->solves_waited = false;
  }
  if (e != hipSuccess) return hip_fail(c, e, "kf_solve");
  c->epoch += bound;
  return KF_OK;
}

kf_status kf_fuse_frame(kf_ctx* c, const uint8_t* image1, const double T_wc1[16]) {
  kf_status s = kf_stereo_update(c, image1, T_wc1);
  if (s != KF_OK) return s;
  return kf_solve(c);
}

kf_status kf_read_depth(kf_ctx* c, void* depth_out, void* var_out, double* scale_out) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_read_depth before kf_set_prior");
  if (hipError_t e = wait_solves(c); e != hipSuccess) return hip_fail(c, e, "kf_read_depth");
  if (depth_out || var_out) {
    if (!depth_out) return fail(c, KF_ERR_ARG, "kf_read_depth: var_out needs depth_out");
    ReadArgs a;
    a.N = c->cfg.width * c->cfg.height;
    a.x = c->ws + c->lay.x;
    a.var = var_buf(c, c->cur);
    a.depth_out = depth_out;
    a.var_out = var_out;
    hipError_t e = launch_read(c->cfg.precision, a, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "kf_read_depth");
  }
  kf_status s = check_device_flags(c);
  if (s != KF_OK) return s;
  if (scale_out) {
    double tau;
    hipError_t e = hipMemcpy(&tau, &scal_ptr(c)->tau, sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "kf_read_depth (scale)");
    *scale_out = std::exp(tau);
  }
  return KF_OK;
}

kf_status kf_read_stats(kf_ctx* c, kf_frame_stats* out) {
  if (!c || !out) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_read_stats before kf_set_prior");
  DevScalars h;
  hipError_t e = wait_solves(c);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, scal_ptr(c), sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_read_stats");
  out->n_searched = h.mask_count;
  out->n_updated = h.n_updated[c->cur];
  out->n_valid = h.n_valid;
  out->cg_iterations = h.cg_iterations;
  out->scale = std::exp(h.tau);
  out->cg_rel_residual = h.cg_rel_residual;
  out->team_syncs = h.team_syncs;
  out->new_keyframe = h.new_keyframe;
  if (h.err & ERR_TIMEOUT) return fail(c, KF_ERR_TIMEOUT, "solver workgroups timed out waiting for their team");
  if (h.err & ERR_INPUT) return fail(c, KF_ERR_INPUT, "device found a non-finite input or a variance <= 0");
  return KF_OK;
}

kf_status kf_fuse_frame_static(kf_ctx* c, const uint8_t* image1, const double T_wc1[16]) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_fuse_frame_static before kf_set_prior");
  if (c->cfg.pipeline_frames) return fail(c, KF_ERR_STATE, "kf_fuse_frame_static needs a context without pipeline_frames");
  if (!image1) return fail(c, KF_ERR_ARG, "kf_fuse_frame_static: NULL image");
  if (!pose_ok(T_wc1)) return fail(c, KF_ERR_ARG, "kf_fuse_frame_static: pose must be finite with last row 0 0 0 1");
  const size_t stage = align256((size_t)(c->cfg.height + 1) * stage_stride(c->cfg.width));
  const size_t exch = c->lay.total - c->lay.parts;   // exchange words of the solver team
  if (stage + exch > KF_STATIC_SCRATCH_BYTES)
    return fail(c, KF_ERR_ARG, "kf_fuse_frame_static: this keyframe needs " + std::to_string(stage + exch) +
                                   " bytes of scratch, the static array holds " +
                                   std::to_string(KF_STATIC_SCRATCH_BYTES));
  char* base = nullptr;
  hipError_t e = static_scratch(c->device, &base);
  if (e != hipSuccess) return hip_fail(c, e, "kf_fuse_frame_static (static scratch address)");
  StereoArgs a;
  if (!stereo_args(c, image1, T_wc1, &a)) return fail(c, KF_ERR_ARG, "kf_fuse_frame_static: singular pose");
  a.i1s = reinterpret_cast<uint8_t*>(base);
  const kf_config& g = c->cfg;
  const uint32_t bound = solve_epoch_bound(g);
  e = epoch_wrap_if_needed(c, bound);
  // the array holds whatever the last call on this device left: its exchange
  // words start from zero (epoch 0 is never used), cleared by a fill kernel
  if (e == hipSuccess) e = launch_zero(base + stage, exch, c->stream);
  if (e == hipSuccess) e = launch_stereo(g.precision, g.pattern, g.n_samples, a, c->cus, false, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_fuse_frame_static (stereo)");
  ++c->frame;
  SolveArgs sa;
  solve_args(c, &sa);
  sa.parts = reinterpret_cast<uint64_t*>(base + stage);
  sa.halo = reinterpret_cast<uint64_t*>(base + stage + (c->lay.halo - c->lay.parts));
  const int kind = solve_kind(g);
  if (c->coresident < 0) c->coresident = solve_max_coresident(g.precision, c->tiling, kind, c->device);
  if (c->coresident < c->tiling.blocks)
    return fail(c, KF_ERR_ARG, "solver tiling needs " + std::to_string(c->tiling.blocks) +
                               " co-resident workgroups, the device holds " + std::to_string(c->coresident));
  e = launch_solve(g.precision, c->tiling, sa, g.solver_cooperative != 0, kind, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_fuse_frame_static (solve)");
  c->epoch += bound;
  return KF_OK;
}

kf_status kf_probe_sync(kf_ctx* c, int32_t rounds, int32_t nvalues) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_probe_sync before kf_set_prior");
  if (c->cfg.pipeline_frames) return fail(c, KF_ERR_STATE, "kf_probe_sync needs a context without pipeline_frames");
  if (rounds < 1 || rounds > 20000) return fail(c, KF_ERR_ARG, "kf_probe_sync: rounds must be in [1, 20000]");
  if (nvalues < 1 || nvalues > NV_MAX) return fail(c, KF_ERR_ARG, "kf_probe_sync: nvalues must be in [1, 3]");
  const uint32_t bound = (uint32_t)rounds + 2;
  hipError_t e = epoch_wrap_if_needed(c, bound);
  if (e != hipSuccess) return hip_fail(c, e, "kf_probe_sync (epoch wrap)");
  SolveArgs a;
  solve_args(c, &a);
  a.epoch_span = bound;
  a.packed = (c->cfg.precision != KF_F64 && bound < 30000) ? 1 : 0;
  if (c->coresident < 0) c->coresident = solve_max_coresident(c->cfg.precision, c->tiling, solve_kind(c->cfg), c->device);
  if (c->coresident < c->tiling.blocks) return fail(c, KF_ERR_ARG, "kf_probe_sync: tiling not co-resident");
  e = launch_sync_probe(c->cfg.precision, c->tiling, a, rounds, nvalues, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_probe_sync");
  c->epoch += bound;
  return KF_OK;
}

void* kf_solve_stream(const kf_ctx* c) { return c ? reinterpret_cast<void*>(c->solve_stream) : nullptr; }

kf_status kf_solver_layout(const kf_ctx* c, int32_t out[5]) {
  if (!c || !out) return KF_ERR_ARG;
  out[0] = c->tiling.tiles_x;
  out[1] = c->tiling.tiles_y;
  out[2] = c->tiling.tile_w;
  out[3] = c->tiling.tile_h;
  out[4] = c->tiling.threads;
  return KF_OK;
}

kf_status kf_export_state(kf_ctx* c, void* x, void* rho, void* rho_var, int32_t* match, double* tau) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_export_state before kf_set_prior");
  const size_t N = (size_t)c->cfg.width * c->cfg.height;
  const size_t nb = N * c->lay.elt;
  hipError_t e = wait_solves(c);
  if (x && e == hipSuccess) e = hipMemcpyAsync(x, c->ws + c->lay.x, nb, hipMemcpyDeviceToDevice, c->stream);
  if (rho && e == hipSuccess) e = hipMemcpyAsync(rho, rho_buf(c, c->cur), nb, hipMemcpyDeviceToDevice, c->stream);
  if (rho_var && e == hipSuccess)
    e = hipMemcpyAsync(rho_var, var_buf(c, c->cur), nb, hipMemcpyDeviceToDevice, c->stream);
  if (match && e == hipSuccess)
    e = hipMemcpyAsync(match, c->ws + c->lay.match, N * 4, hipMemcpyDeviceToDevice, c->stream);
  double t = 0.0;
  if (tau && e == hipSuccess) e = hipMemcpyAsync(&t, &scal_ptr(c)->tau, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_export_state");
  if (tau) *tau = t;
  return KF_OK;
}

kf_status kf_import_state(kf_ctx* c, const void* x, const void* rho, const void* rho_var, const double* tau) {
  if (!c) return KF_ERR_ARG;
  if (!c->has_prior) return fail(c, KF_ERR_STATE, "kf_import_state before kf_set_prior");
  if ((rho == nullptr) != (rho_var == nullptr)) return fail(c, KF_ERR_ARG, "kf_import_state: rho and rho_var go together");
  if (tau && !std::isfinite(*tau)) return fail(c, KF_ERR_ARG, "kf_import_state: tau must be finite");
  hipError_t e = wait_solves(c);
  if ((x || rho) && e == hipSuccess) {
    ImportArgs a;
    a.N = c->cfg.width * c->cfg.height;
    a.x = x; a.rho = rho; a.var = rho_var;
    a.dx = c->ws + c->lay.x;
    a.drho = rho_buf(c, c->cur);
    a.dvar = var_buf(c, c->cur);
    a.scal = scal_ptr(c);
    e = launch_import(c->cfg.precision, a, c->stream);
  }
  double t = tau ? *tau : 0.0;
  if (tau && e == hipSuccess) e = hipMemcpyAsync(&scal_ptr(c)->tau, &t, 8, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "kf_import_state");
  return check_device_flags(c);
}

}  // extern "C"
