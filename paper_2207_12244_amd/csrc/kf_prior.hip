// Keyframe initialisation (texture mask, priors, state reset), read-out and state import.
#include "kf_internal.h"

namespace kf {

namespace {

__device__ inline bool finite_d(double v) { return isfinite(v); }

// Texture gate (Sec. II-B "sufficient texture"): central differences of the
// uint8 keyframe image, (a/2)^2 + (b/2)^2 >= gate^2, exact for integer images;
// pixels within `border` of the edge are never searched.
__device__ inline bool textured(const uint8_t* img, int W, int H, int u, int v, double gate, int border) {
  if (u < border || v < border || u > W - 1 - border || v > H - 1 - border) return false;
  if (u < 1 || v < 1 || u > W - 2 || v > H - 2) return false;
  const size_t i = (size_t)v * W + u;
  const double a = 0.5 * ((double)img[i + 1] - (double)img[i - 1]);
  const double b = 0.5 * ((double)img[i + W] - (double)img[i - W]);
  return a * a + b * b >= gate * gate;
}

template <typename T, typename TI>
__global__ __launch_bounds__(CHUNK) void k_prior_init(PriorArgs a) {
  const int N = a.W * a.H;
  const int i = blockIdx.x * CHUNK + threadIdx.x;
  bool m = false;
  if (i < N) {
    const int u = i % a.W, v = i / a.W;
    m = textured(a.image0, a.W, a.H, u, v, a.grad_gate, a.border);
    static_cast<TI*>(a.i0)[i] = to_img<TI, T>((T)a.image0[i]);
    const T* mu = static_cast<const T*>(a.mu);
    const T* vn = static_cast<const T*>(a.var_n);
    const T* gx = static_cast<const T*>(a.gx);
    const T* vgx = static_cast<const T*>(a.var_gx);
    const T* gy = static_cast<const T*>(a.gy);
    const T* vgy = static_cast<const T*>(a.var_gy);
    T* pr = static_cast<T*>(a.prior);
    const T mui = mu[i], vni = vn[i], gxi = gx[i], vgxi = vgx[i], gyi = gy[i], vgyi = vgy[i];
    // network depth variance must be finite and positive (it makes the scale
    // observable, Sec. II-C); gradient variances may be +inf (term disabled)
    bool ok = finite_d((double)mui) && finite_d((double)gxi) && finite_d((double)gyi) &&
              finite_d((double)vni) && vni > (T)0 && vgxi > (T)0 && vgyi > (T)0 &&
              !isnan((double)vgxi) && !isnan((double)vgyi);
    if (!ok) atomicOr(&a.scal->err, ERR_INPUT);
    pr[0 * (size_t)N + i] = mui;
    pr[1 * (size_t)N + i] = (T)1 / sqrt(vni);
    pr[2 * (size_t)N + i] = gxi;
    pr[3 * (size_t)N + i] = (T)1 / sqrt(vgxi);
    pr[4 * (size_t)N + i] = gyi;
    pr[5 * (size_t)N + i] = (T)1 / sqrt(vgyi);
    static_cast<T*>(a.x)[i] = mui;
    static_cast<T*>(a.rho)[i] = (T)0;
    static_cast<T*>(a.var)[i] = (T)0;
    a.match[i] = m ? -1 : -2;   // -2: not textured, never searched
  }
  const int cnt = __syncthreads_count(m ? 1 : 0);
  if (threadIdx.x == 0) a.chunk_counts[blockIdx.x] = cnt;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal->epoch = 1u;
    a.scal->tau = 0.0;
    a.scal->cg_rel_residual = 0.0;
    a.scal->n_updated[0] = a.scal->n_updated[1] = 0;
    a.scal->n_valid = 0;
    a.scal->cg_iterations = 0;
  }
}

// Network outputs (Sec. II-A) to keyframe priors: bilinear resampling with pixel
// centres aligned (keyframe pixel u samples the network map at
// (u + 1/2) Wn / W - 1/2, clamped), the focal-length shift of the log-depth, and
// the gradients and their variances rescaled from network to keyframe pixel
// spacing. Positions, weights and sums in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_resample_priors(ResampleArgs r) {
  const int N = r.W * r.H;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const int u = i % r.W, v = i / r.W;
  const double sx = (double)r.Wn / r.W, sy = (double)r.Hn / r.H;
  double un = (u + 0.5) * sx - 0.5, vn = (v + 0.5) * sy - 0.5;
  un = un < 0.0 ? 0.0 : (un > r.Wn - 1.0 ? r.Wn - 1.0 : un);
  vn = vn < 0.0 ? 0.0 : (vn > r.Hn - 1.0 ? r.Hn - 1.0 : vn);
  const int u0 = min((int)floor(un), r.Wn - 2), v0 = min((int)floor(vn), r.Hn - 2);
  const double f = un - u0, g = vn - v0;
  const double scale[6] = {1.0, 1.0, sx, sx * sx, sy, sy * sy};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T* m = static_cast<const T*>(r.src[k]);
    const size_t a = (size_t)v0 * r.Wn + u0, b = a + r.Wn;
    const double top = (1.0 - f) * (double)m[a] + f * (double)m[a + 1];
    const double bot = (1.0 - f) * (double)m[b] + f * (double)m[b + 1];
    double val = (1.0 - g) * top + g * bot;
    val = k == 0 ? val + r.shift : val * scale[k];
    static_cast<T*>(r.dst)[(size_t)k * N + i] = (T)val;
  }
}

// Exclusive scan of the per-chunk counts (one workgroup), total -> mask_count.
__global__ __launch_bounds__(1024) void k_scan_chunks(int32_t* counts, int nchunks, DevScalars* scal) {
  __shared__ int32_t part[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nchunks; base += 1024) {
    const int c = base + threadIdx.x;
    const int32_t v = c < nchunks ? counts[c] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (c < nchunks) counts[c] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[nchunks] = carry;
    scal->mask_count = carry;
  }
}

// Writes the textured pixels, in row-major order, into the search list.
__global__ __launch_bounds__(CHUNK) void k_write_list(PriorArgs a) {
  __shared__ int32_t wave_cnt[CHUNK / 64];
  const int N = a.W * a.H;
  const int i = blockIdx.x * CHUNK + threadIdx.x;
  bool m = false;
  if (i < N) m = textured(a.image0, a.W, a.H, i % a.W, i / a.W, a.grad_gate, a.border);
  const uint64_t ballot = __ballot(m);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = lane ? (ballot & ((~0ull) >> (64 - lane))) : 0ull;
  const int rank = __popcll(below);
  if (lane == 0) wave_cnt[wave] = __popcll(ballot);
  __syncthreads();
  int off = a.chunk_counts[blockIdx.x];
  for (int w = 0; w < wave; ++w) off += wave_cnt[w];
  if (m) a.list[off + rank] = i;
}

template <typename T>
__global__ void k_read(ReadArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const T* x = static_cast<const T*>(a.x);
  static_cast<T*>(a.depth_out)[i] = exp(x[i]);
  if (a.var_out) static_cast<T*>(a.var_out)[i] = static_cast<const T*>(a.var)[i];
}

template <typename T>
__global__ void k_import(ImportArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  bool ok = true;
  if (a.x) {
    const T v = static_cast<const T*>(a.x)[i];
    ok = ok && finite_d((double)v);
    static_cast<T*>(a.dx)[i] = v;
  }
  if (a.rho && a.var) {
    const T r = static_cast<const T*>(a.rho)[i];
    const T w = static_cast<const T*>(a.var)[i];
    // var == 0 marks "no estimate"; an estimate needs rho > 0 and a finite var
    ok = ok && finite_d((double)r) && finite_d((double)w) && w >= (T)0 && (w == (T)0 || r > (T)0);
    static_cast<T*>(a.drho)[i] = r;
    static_cast<T*>(a.dvar)[i] = w;
  }
  if (!ok) atomicOr(&a.scal->err, ERR_INPUT);
}

template <int PREC>
hipError_t prior_impl(const PriorArgs& a, hipStream_t s) {
  using T = typename Form<PREC>::T;
  using TI = typename Form<PREC>::TI;
  const int N = a.W * a.H;
  const int nchunks = (N + CHUNK - 1) / CHUNK;
  hipLaunchKernelGGL((k_prior_init<T, TI>), dim3(nchunks), dim3(CHUNK), 0, s, a);
  hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, a.chunk_counts, nchunks, a.scal);
  hipLaunchKernelGGL(k_write_list, dim3(nchunks), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_prior(int prec, const PriorArgs& a, hipStream_t s) {
  switch (prec) {
    case KF_F64: return prior_impl<KF_F64>(a, s);
    case KF_F32: return prior_impl<KF_F32>(a, s);
    case KF_BF16_F32: return prior_impl<KF_BF16_F32>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_resample_priors(int prec, const ResampleArgs& a, hipStream_t s) {
  const int blocks = (a.W * a.H + 255) / 256;
  if (prec == KF_F64)
    hipLaunchKernelGGL(k_resample_priors<double>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_resample_priors<float>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_read(int prec, const ReadArgs& a, hipStream_t s) {
  const int blocks = (a.N + 255) / 256;
  if (prec == KF_F64)
    hipLaunchKernelGGL(k_read<double>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_read<float>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_import(int prec, const ImportArgs& a, hipStream_t s) {
  const int blocks = (a.N + 255) / 256;
  if (prec == KF_F64)
    hipLaunchKernelGGL(k_import<double>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_import<float>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace kf

namespace kf {

namespace {
__global__ void k_zero_words(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
}  // namespace

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

// Clears a 4-byte aligned device range with a kernel (no memset node, so a
// stream that is being captured into a graph replays it correctly).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

}  // namespace kf
