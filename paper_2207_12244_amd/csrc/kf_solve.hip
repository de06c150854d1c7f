// Optimisation (Sec. II-C): n_gn Gauss-Newton iterations alternating between the
// log-depth map x and the scale tau = ln s, each depth step solved by Jacobi-
// preconditioned CG on the 5-point normal equations, all in ONE persistent
// launch per frame (per batch of keyframes in the batched form).
//
// Decomposition: the keyframe is cut into tiles_x x tiles_y tiles; a team of
// workgroups, member b owning tile b, keeps the CG vectors of its pixels in
// registers and a one-pixel ghost ring of the stencil operand in LDS for the
// whole solve. Workgroups never meet at a grid barrier. At each
// synchronisation point every member publishes its partial sums and its tile
// boundary as 64-bit words tagged with an epoch number (relaxed agent-scope
// atomic stores), then polls the words it needs: all partials of the team
// (summed in a fixed order, so every member gets bit-identical totals) and the
// boundaries of its four neighbours. Slots are double-buffered by epoch
// parity; no member can run two synchronisations ahead of another because each
// one waits for every partial.
//
// Per GN iteration: 1 synchronisation for the initial residual, then per PCG
// iteration 1 (pipelined variant: both inner products and the boundary of the
// next stencil operand) or 2 (textbook variant: p.q; then r.z with the z
// boundary from which every member rebuilds its ghost copy of p, the last r.z
// skipped in fixed-count mode), and 1 for the scale step (which also ships the
// x boundary). The fixed-count pipelined variant skips the initial-residual
// synchronisation: its scale step ships x two pixels deep (plus the diagonal
// neighbours' corner pixels), from which each member assembles the ghost
// values of the first stencil operand itself.
#include "kf_internal.h"

namespace kf {

namespace {

constexpr int GMAX = 2;      // ghost slots per thread: ghost ring <= GMAX * threads cells
constexpr int G2MAX = 1;     // second-ring slots per thread: second ring + 4 corners <= threads cells

__device__ inline void st_word(KF_GLOBAL uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_word(const KF_GLOBAL uint64_t* p) {
  return __hip_atomic_load(const_cast<KF_GLOBAL uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Compiler-only barrier (no instruction): the value counts as redefined here,
// so per-pixel addresses derived from it are recomputed inside the loop that
// holds the barrier instead of being hoisted and kept live in registers for the
// whole launch (that cut the register count per pixel from ~53 to ~16).
__device__ inline void refresh(int& v) { asm volatile("" : "+v"(v)); }

__device__ inline uint64_t tagged(uint32_t bits, uint32_t e) { return ((uint64_t)e << 32) | (uint64_t)bits; }

template <typename V> struct Wire;
template <> struct Wire<float> {
  static constexpr int N = 1;
  __device__ static void put(KF_GLOBAL uint64_t* w, float v, uint32_t e) { st_word(w, tagged(__float_as_uint(v), e)); }
  __device__ static float make(uint32_t lo, uint32_t) { return __uint_as_float(lo); }
};
// One-word transport of an FP64 partial: the top 48 bits of the double
// (rounded; relative precision 2^-37) and a 16-bit epoch. Used when a launch
// spans fewer than 30000 epochs, so a slot's previous content is never 2^16
// epochs old.
struct Packed48 {
  __device__ static uint64_t make_word(double v, uint32_t e) {
    const uint64_t b = (uint64_t)__double_as_longlong(v) + 0x8000ull;
    return ((uint64_t)(e & 0xffffu) << 48) | (b >> 16);
  }
  __device__ static bool ready(uint64_t w, uint32_t e) { return (uint32_t)(w >> 48) == (e & 0xffffu); }
  __device__ static double value(uint64_t w) {
    return __longlong_as_double((long long)((w & 0xffffffffffffull) << 16));
  }
};

template <> struct Wire<double> {
  static constexpr int N = 2;
  __device__ static void put(KF_GLOBAL uint64_t* w, double v, uint32_t e) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    st_word(w, tagged((uint32_t)bits, e));
    st_word(w + 1, tagged((uint32_t)(bits >> 32), e));
  }
  __device__ static double make(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  }
};

// Data-parallel-primitive move of both halves of a double (out-of-row lanes read 0).
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes in a fixed order: an inclusive scan inside each
// 16-lane row (shifts 1, 2, 4, 8), then the row totals are carried with the
// row broadcasts 15 and 31; lane 63 ends with the total (other lanes hold
// partial sums).
__device__ inline double wave_total_lane63(double v) {
  v += dpp_d<0x111, 0xf, true>(v);   // row_shr:1
  v += dpp_d<0x112, 0xf, true>(v);   // row_shr:2
  v += dpp_d<0x114, 0xf, true>(v);   // row_shr:4
  v += dpp_d<0x118, 0xf, true>(v);   // row_shr:8
  v += dpp_d<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// IRLS weight of a whitened residual: Huber min(1, c / |r|), or Tukey's
// biweight (1 - (r/c)^2)^2 inside c and 0 beyond.
template <typename T>
__device__ inline T huber_w(T r, T delta, bool tukey = false) {
  if (tukey) {
    const T t = r / delta, t2 = t * t;
    return t2 <= (T)1 ? ((T)1 - t2) * ((T)1 - t2) : (T)0;
  }
  const T a = fabs(r);
  return a <= delta ? (T)1 : delta / a;
}

// IRLS weight of the gradient edge between x_a and its right / lower neighbour x_b.
template <typename T>
__device__ inline T edge_weight(T xa, T xb, T g, T isd, T delta, bool tukey) {
  const T r = ((xb - xa) - g) * isd;
  return huber_w(r, delta, tukey) * isd * isd;
}

template <typename T, int NT>
struct Team {
  static constexpr int NW = NT / 64;
  static constexpr int PSLOTS = (NV_MAX * MAX_TEAM + NT - 1) / NT;   // partial slots polled per thread
  static constexpr int CPV = MAX_TEAM / 64;                            // 64-slot chunks per value, at most
  int B, b, tw, th, rw, perim, tile_w, tile_h;
  int nb_up, nb_dn, nb_lf, nb_rt;
  KF_GLOBAL uint64_t* parts;
  KF_GLOBAL uint64_t* halo;
  KF_GLOBAL int32_t* err;
  uint64_t limit;
  bool packed;      // one-word partials (Packed48) instead of two words
  double* s_wred;   // [NW][NV_MAX]
  double* s_pol;    // [NV_MAX][CPV] chunk partials (unused chunks stay 0)
  int* s_abort;
  // ghost slots of this thread
  int g_src[GMAX];  // neighbour workgroup or -1
  int g_off[GMAX];  // offset in its boundary list
  int g_li[GMAX];   // ring index
  // second-ring slots of this thread (two-deep x boundary, see publish_ring2):
  // neighbour (or diagonal neighbour) workgroup or -1, offset in its boundary
  // lists, destination index relative to the x ring
  int g2_src[G2MAX];
  int g2_off[G2MAX];
  int g2_li[G2MAX];

  // Replica r of member j's partial v: every member writes all replicas and
  // reads replica (own index mod PART_REPLICAS), so the team's polling loads
  // spread over several copies of the hot words. A one-word partial sits at a
  // one-word stride, so a wavefront's 64 polled slots span half the cache
  // lines of two-word slots (-2 % on the 640 x 480 solve).
  __device__ KF_GLOBAL uint64_t* part_slot(uint32_t e, int v, int j, int r) const {
    return parts + ((size_t)(((e & 1u) * NV_MAX + v) * PART_REPLICAS + r) * B + j) * (packed ? 1 : 2);
  }
  // Boundary lists of member blk: [0, perim) its first row / column per side,
  // [perim, 2 perim) its second row / column per side (publish_ring2).
  // (a slot is as many words as the value's transport, Wire<T>::N)
  __device__ KF_GLOBAL uint64_t* halo_slot(uint32_t e, int blk, int off) const {
    return halo + ((size_t)((e & 1u) * B + blk) * (2 * perim) + off) * Wire<T>::N;
  }

  // Publishes the boundary value of own pixel (lx, ly) for the neighbours that read it.
  __device__ void publish(uint32_t e, int lx, int ly, T val) const {
    if (ly == 0 && nb_up >= 0) Wire<T>::put(halo_slot(e, b, lx), val, e);
    if (ly == th - 1 && nb_dn >= 0) Wire<T>::put(halo_slot(e, b, tile_w + lx), val, e);
    if (lx == 0 && nb_lf >= 0) Wire<T>::put(halo_slot(e, b, 2 * tile_w + ly), val, e);
    if (lx == tw - 1 && nb_rt >= 0) Wire<T>::put(halo_slot(e, b, 2 * tile_w + tile_h + ly), val, e);
  }

  // Publishes the whole tile boundary from the ring that holds the own values
  // (after a barrier): thread s writes boundary slot s, so only the first
  // perimeter's worth of threads issue the stores.
  __device__ void publish_ring(uint32_t e, const T* ring) const {
    int s = threadIdx.x;
    refresh(s);
    for (; s < perim; s += NT) {
      int lx, ly, nb;
      if (s < tile_w) {
        lx = s; ly = 0; nb = nb_up;
      } else if (s < 2 * tile_w) {
        lx = s - tile_w; ly = th - 1; nb = nb_dn;
      } else if (s < 2 * tile_w + tile_h) {
        lx = 0; ly = s - 2 * tile_w; nb = nb_lf;
      } else {
        lx = tw - 1; ly = s - 2 * tile_w - tile_h; nb = nb_rt;
      }
      if (nb >= 0 && lx < tw && ly < th) Wire<T>::put(halo_slot(e, b, s), ring[(ly + 1) * rw + lx + 1], e);
    }
  }

  // Publishes the second row / column of each side (row 1 for the member
  // above, row th - 2 below, column 1 to the left, column tw - 2 to the right)
  // from the ring of own values: with the first ones and the diagonal
  // neighbours' corner pixels, a neighbour holds the tile's x two pixels deep.
  __device__ void publish_ring2(uint32_t e, const T* ring) const {
    int s = threadIdx.x;
    refresh(s);
    for (; s < perim; s += NT) {
      int lx, ly, nb;
      if (s < tile_w) {
        lx = s; ly = 1; nb = nb_up;
      } else if (s < 2 * tile_w) {
        lx = s - tile_w; ly = th - 2; nb = nb_dn;
      } else if (s < 2 * tile_w + tile_h) {
        lx = 1; ly = s - 2 * tile_w; nb = nb_lf;
      } else {
        lx = tw - 2; ly = s - 2 * tile_w - tile_h; nb = nb_rt;
      }
      if (nb >= 0 && lx >= 0 && ly >= 0 && lx < tw && ly < th)
        Wire<T>::put(halo_slot(e, b, perim + s), ring[(ly + 1) * rw + lx + 1], e);
    }
  }

  // Team-wide sums of nv per-thread partials and, if `ghosts`, the neighbours'
  // published boundary values for this thread's ghost slots (stored into
  // `ring` too when given). With `ring_pub` the own boundary is published from
  // `ring` (the caller wrote its own values there), otherwise the caller has
  // published it. Each wavefront reduces the 64 team partials it polled;
  // every wavefront then adds those chunk sums in the same fixed order, so all
  // threads of all workgroups hold bit-identical totals. All words a thread
  // waits for are loaded together each polling round. Returns false if the
  // team aborts.
  __device__ bool sync(uint32_t e, int nv, const double* vals, double* tot, T* gval, bool ghosts, T* ring = nullptr,
                       bool ring_pub = false) {
    return this->template sync<false>(e, nv, vals, tot, gval, ghosts, ring, ring_pub, [] {});
  }

  // As above; `pre()` runs in every thread after the workgroup has published
  // its partials and before it polls: work that needs no neighbour data (and
  // may read LDS written before the synchronisation) overlaps the wait. With
  // R2 the second-ring slots are polled too, into `ring` at g2_li (the caller
  // publishes its own second rows in `pre`).
  template <bool R2, typename F>
  __device__ bool sync(uint32_t e, int nv, const double* vals, double* tot, T* gval, bool ghosts, T* ring, bool ring_pub,
                       F&& pre) {
    int tid = threadIdx.x;
    refresh(tid);
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int m = 0; m < GMAX; ++m) {
      refresh(g_src[m]);
      refresh(g_off[m]);
      refresh(g_li[m]);
    }
    // the nv scans are independent, so their DPP chains interleave; lane 63
    // holds each total and stores it (no read-back through a scalar)
    double wsum[NV_MAX];
#pragma unroll
    for (int v = 0; v < NV_MAX; ++v) wsum[v] = v < nv ? wave_total_lane63(vals[v]) : 0.0;
    if (lane == 63) {
#pragma unroll
      for (int v = 0; v < NV_MAX; ++v)
        if (v < nv) s_wred[wave * NV_MAX + v] = wsum[v];
    }
    __syncthreads();
    if (tid < nv * PART_REPLICAS) {
      const int v = tid % nv, r = tid / nv;
      double p = 0.0;
      for (int w = 0; w < NW; ++w) p += s_wred[w * NV_MAX + v];
      if (packed) st_word(part_slot(e, v, b, r), Packed48::make_word(p, e));
      else Wire<double>::put(part_slot(e, v, b, r), p, e);
    }
    if (ring_pub) publish_ring(e, ring);
    pre();
    // poll set of this thread: slot s = (value v, member j) with the members of
    // each value padded to a multiple of 64 slots, so that every wavefront
    // polls slots of one value only and can reduce them itself
    const int Bp = (B + 63) & ~63;
    const int nslots = nv * Bp;
    bool p_ready[PSLOTS], g_ready[GMAX], g2_ready[G2MAX];
    uint64_t pw0[PSLOTS], pw1[PSLOTS], gw0[GMAX], gw1[GMAX], g2w0[G2MAX], g2w1[G2MAX];
    double pval[PSLOTS];   // decoded partials; padding slots keep 0
    const KF_GLOBAL uint64_t* p_addr[PSLOTS];
    const int cpv = Bp >> 6;   // chunks per value
#pragma unroll
    for (int q = 0; q < PSLOTS; ++q) {
      const int sl = tid + q * NT;
      const int v = (sl >> 6) / cpv, j = sl - v * Bp;
      pval[q] = 0.0;
      p_ready[q] = sl >= nslots || j >= B;
      p_addr[q] = part_slot(e, p_ready[q] ? 0 : v, p_ready[q] ? 0 : j, b % PART_REPLICAS);
    }
#pragma unroll
    for (int m = 0; m < GMAX; ++m) g_ready[m] = !(ghosts && g_src[m] >= 0);
#pragma unroll
    for (int m = 0; m < G2MAX; ++m) {
      g2_ready[m] = !(R2 && g2_src[m] >= 0);
      g2w0[m] = g2w1[m] = 0;
      if (R2) {
        refresh(g2_src[m]);
        refresh(g2_off[m]);
        refresh(g2_li[m]);
      }
    }
    unsigned spins = 0;
    uint64_t t0 = 0;
    bool ok = true;
    while (true) {
      bool all = true;
#pragma unroll
      for (int q = 0; q < PSLOTS; ++q) {
        if (!p_ready[q]) {
          const KF_GLOBAL uint64_t* w = p_addr[q];
          pw0[q] = ld_word(w);
          if (!packed) pw1[q] = ld_word(w + 1);
        }
      }
#pragma unroll
      for (int m = 0; m < GMAX; ++m) {
        if (!g_ready[m]) {
          const KF_GLOBAL uint64_t* w = halo_slot(e, g_src[m], g_off[m]);
          gw0[m] = ld_word(w);
          if (Wire<T>::N == 2) gw1[m] = ld_word(w + 1);
        }
      }
#pragma unroll
      for (int m = 0; m < G2MAX; ++m) {
        if (R2 && !g2_ready[m]) {
          const KF_GLOBAL uint64_t* w = halo_slot(e, g2_src[m], g2_off[m]);
          g2w0[m] = ld_word(w);
          if (Wire<T>::N == 2) g2w1[m] = ld_word(w + 1);
        }
      }
#pragma unroll
      for (int q = 0; q < PSLOTS; ++q) {
        if (!p_ready[q]) {
          if (packed ? Packed48::ready(pw0[q], e)
                     : ((uint32_t)(pw0[q] >> 32) == e && (uint32_t)(pw1[q] >> 32) == e)) {
            p_ready[q] = true;
            pval[q] = packed ? Packed48::value(pw0[q]) : Wire<double>::make((uint32_t)pw0[q], (uint32_t)pw1[q]);
          } else {
            all = false;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < GMAX; ++m) {
        if (!g_ready[m]) {
          if ((uint32_t)(gw0[m] >> 32) == e && (Wire<T>::N == 1 || (uint32_t)(gw1[m] >> 32) == e)) {
            g_ready[m] = true;
            gval[m] = Wire<T>::make((uint32_t)gw0[m], (uint32_t)gw1[m]);
            if (ring) ring[g_li[m]] = gval[m];
          } else {
            all = false;
          }
        }
      }
#pragma unroll
      for (int m = 0; m < G2MAX; ++m) {
        if (R2 && !g2_ready[m]) {
          if ((uint32_t)(g2w0[m] >> 32) == e && (Wire<T>::N == 1 || (uint32_t)(g2w1[m] >> 32) == e)) {
            g2_ready[m] = true;
            ring[g2_li[m]] = Wire<T>::make((uint32_t)g2w0[m], (uint32_t)g2w1[m]);
          } else {
            all = false;
          }
        }
      }
      if (all) break;
      if ((++spins & 63u) == 0u) {
        const uint64_t now = wall_clock64();
        if (t0 == 0) t0 = now;
        if (now - t0 > limit ||
            (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT)) {
          ok = false;
          break;
        }
      }
    }
    if (!ok) {
      *s_abort = 1;
      __hip_atomic_fetch_or(err, ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // each wavefront sums its 64 polled slots (one value, fixed order) into a
    // chunk partial; the chunk index is wavefront-uniform
#pragma unroll
    for (int q = 0; q < PSLOTS; ++q) {
      const int chunk = (q * NT + tid) >> 6;
      if (chunk * 64 < nslots) {
        const double cs = wave_total_lane63(pval[q]);
        const int v = chunk / cpv;
        if (lane == 63) s_pol[v * CPV + chunk - v * cpv] = cs;
      }
    }
    __syncthreads();
    if (*s_abort) return false;
    // every wavefront forms the totals from the chunk partials (fixed order,
    // so all threads of all workgroups hold bit-identical totals); the
    // chunks past cpv hold zeros, so all CPV loads issue together
    for (int v = 0; v < nv; ++v) {
      double c[CPV];
#pragma unroll
      for (int k = 0; k < CPV; ++k) c[k] = s_pol[v * CPV + k];
      double acc = c[0];
#pragma unroll
      for (int k = 1; k < CPV; ++k) acc += c[k];
      tot[v] = acc;
    }
    return true;
  }
};

// LDS of one member: [NW][NV_MAX] wave partials, [NV_MAX][CPV] team chunk
// partials, abort flag, then three rings of (tile_h + 2) x (tile_w + 2):
// x and two stencil operands, then the second ring of x (2 tile_w + 2 tile_h:
// top, bottom, left, right; its corners sit in the corner cells of the x ring),
// then 12 x (2 tile_w + 2 tile_h) static row inputs of the ghost cells.
template <typename T, int NT>
struct MemberLds {
  T* xs;
  T* ps;
  T* ms0;
  T* x2;
  T* gdat;
};

// Tile coordinates of cell g of the second ring of x: [0, tw) the row above
// the ghost row, then the row below, the column left of the ghost column, the
// column right of it, then the four ghost-ring corners (-1, -1), (tw, -1),
// (-1, th), (tw, th).
__device__ inline void ring2_cell(int g, int tw, int th, int& cx, int& cy) {
  if (g < tw) {
    cx = g; cy = -2;
  } else if (g < 2 * tw) {
    cx = g - tw; cy = th + 1;
  } else if (g < 2 * tw + th) {
    cx = -2; cy = g - 2 * tw;
  } else if (g < 2 * tw + 2 * th) {
    cx = tw + 1; cy = g - 2 * tw - th;
  } else {
    const int k = g - 2 * tw - 2 * th;
    cx = (k & 1) ? tw : -1;
    cy = (k & 2) ? th : -1;
  }
}

// Sets up member b (tile b) of the team of `a`: tile geometry, neighbours,
// exchange words, LDS carve-up (cleared) and this thread's ghost slots (top
// row, bottom row, left column, right column). Ends with a workgroup barrier.
template <typename T, int NT>
__device__ __forceinline__ void team_init(Team<T, NT>& tm, MemberLds<T, NT>& lds, const SolveArgs& a, const int b,
                                          unsigned char* smem) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int W = a.W, H = a.H;
  tm.B = a.tiles_x * a.tiles_y;
  tm.b = b;
  const int bx = b % a.tiles_x, by = b / a.tiles_x;
  const int ox = bx * a.tile_w, oy = by * a.tile_h;
  tm.tile_w = a.tile_w;
  tm.tile_h = a.tile_h;
  tm.tw = min(a.tile_w, W - ox);
  tm.th = min(a.tile_h, H - oy);
  tm.rw = tm.tw + 2;
  tm.perim = a.perim;
  tm.nb_up = by > 0 ? b - a.tiles_x : -1;
  tm.nb_dn = by < a.tiles_y - 1 ? b + a.tiles_x : -1;
  tm.nb_lf = bx > 0 ? b - 1 : -1;
  tm.nb_rt = bx < a.tiles_x - 1 ? b + 1 : -1;
  tm.parts = gp(a.parts);
  tm.halo = gp(a.halo);
  tm.err = &gp(a.scal)->err;
  tm.limit = a.timeout_ticks;
  tm.packed = a.packed != 0;
  double* dsm = reinterpret_cast<double*>(smem);
  tm.s_wred = dsm;
  tm.s_pol = tm.s_wred + NW * NV_MAX;
  tm.s_abort = reinterpret_cast<int*>(tm.s_pol + NV_MAX * Team<T, NT>::CPV);
  const int ring_max = (a.tile_h + 2) * (a.tile_w + 2);
  lds.xs = reinterpret_cast<T*>(dsm + NW * NV_MAX + NV_MAX * Team<T, NT>::CPV + 2);
  lds.ps = lds.xs + ring_max;
  lds.ms0 = lds.ps + ring_max;
  lds.x2 = lds.ms0 + ring_max;
  lds.gdat = lds.x2 + a.perim;
  for (int i = tid; i < 3 * ring_max + a.perim; i += NT) lds.xs[i] = (T)0;
  if (tid < NV_MAX * Team<T, NT>::CPV) tm.s_pol[tid] = 0.0;
  if (tid == 0) *tm.s_abort = 0;
  const int tw = tm.tw, th = tm.th, rw = tm.rw;
  const int nghost = 2 * tw + 2 * th;
#pragma unroll
  for (int m = 0; m < GMAX; ++m) {
    const int g = tid + m * NT;
    tm.g_src[m] = -1;
    tm.g_off[m] = 0;
    tm.g_li[m] = 0;
    if (g < nghost) {
      if (g < tw) {
        tm.g_src[m] = tm.nb_up; tm.g_off[m] = a.tile_w + g; tm.g_li[m] = g + 1;
      } else if (g < 2 * tw) {
        const int lx = g - tw;
        tm.g_src[m] = tm.nb_dn; tm.g_off[m] = lx; tm.g_li[m] = (th + 1) * rw + lx + 1;
      } else if (g < 2 * tw + th) {
        const int ly = g - 2 * tw;
        tm.g_src[m] = tm.nb_lf; tm.g_off[m] = 2 * a.tile_w + a.tile_h + ly; tm.g_li[m] = (ly + 1) * rw;
      } else {
        const int ly = g - 2 * tw - th;
        tm.g_src[m] = tm.nb_rt; tm.g_off[m] = 2 * a.tile_w + ly; tm.g_li[m] = (ly + 1) * rw + tw + 1;
      }
    }
  }
  // second-ring slots: the neighbours' second rows / columns (published by
  // publish_ring2) where that pixel is inside the image, and the diagonal
  // neighbours' corner pixels from their first-row lists
  const int x2b = 3 * ring_max;   // index of the second ring relative to xs
  const int ncell = 2 * tw + 2 * th;
#pragma unroll
  for (int m = 0; m < G2MAX; ++m) {
    const int g = tid + m * NT;
    int src = -1, off = 0, li = 0;
    if (a.ghost_z && g < ncell + 4) {
      if (g < tw) {
        src = tm.nb_up; off = a.perim + a.tile_w + g; li = x2b + g;
      } else if (g < 2 * tw) {
        src = (tm.nb_dn >= 0 && oy + th + 1 < H) ? tm.nb_dn : -1; off = a.perim + (g - tw); li = x2b + g;
      } else if (g < 2 * tw + th) {
        src = tm.nb_lf; off = a.perim + 2 * a.tile_w + a.tile_h + (g - 2 * tw); li = x2b + g;
      } else if (g < ncell) {
        src = (tm.nb_rt >= 0 && ox + tw + 1 < W) ? tm.nb_rt : -1; off = a.perim + 2 * a.tile_w + (g - 2 * tw - th);
        li = x2b + g;
      } else {
        const int k = g - ncell;
        const bool up = !(k & 2), left = !(k & 1);
        const int nbv = up ? tm.nb_up : tm.nb_dn, nbh = left ? tm.nb_lf : tm.nb_rt;
        src = (nbv >= 0 && nbh >= 0) ? b + (up ? -a.tiles_x : a.tiles_x) + (left ? -1 : 1) : -1;
        off = (up ? a.tile_w : 0) + (left ? a.tile_w - 1 : 0);
        li = (up ? 0 : (th + 1) * rw) + (left ? 0 : tw + 1);
      }
    }
    tm.g2_src[m] = src;
    tm.g2_off[m] = off;
    tm.g2_li[m] = li;
  }
  __syncthreads();
}

// One member (tile b) of the team that solves keyframe `a`; every thread of
// the workgroup calls it. LDS: `smem` as sized by smem_for for this team.
// VAR: instantiation that handles the Sec. III variants and the keyframe rule;
// the plain form (variant FULL, no rule) runs the one without those branches
// (they cost it ~1 % per solve).
template <typename T, int NT, int PPT, bool PIPE, bool VAR>
__device__ __forceinline__ void solve_member(const SolveArgs& a, const int b, unsigned char* smem) {
  const int tid = threadIdx.x;
  const int W = a.W, H = a.H, N = W * H;

  Team<T, NT> tm;
  MemberLds<T, NT> lds;
  team_init(tm, lds, a, b, smem);
  const int ox = (b % a.tiles_x) * a.tile_w, oy = (b / a.tiles_x) * a.tile_h;
  KF_GLOBAL DevScalars* scal = gp(a.scal);
  T* xs = lds.xs;
  T* ps = lds.ps;
  T* ms0 = lds.ms0;

  const int tw = tm.tw, th = tm.th, rw = tm.rw;
  const int npx = tw * th;
  const T delta = (T)a.huber_delta;

  const KF_GLOBAL T* pr = gp(static_cast<const T*>(a.prior));
  const KF_GLOBAL T* mu_g = pr;
  const KF_GLOBAL T* isn_g = pr + (size_t)N;
  const KF_GLOBAL T* gx_g = pr + 2 * (size_t)N;
  const KF_GLOBAL T* isgx_g = pr + 3 * (size_t)N;
  const KF_GLOBAL T* gy_g = pr + 4 * (size_t)N;
  const KF_GLOBAL T* isgy_g = pr + 5 * (size_t)N;
  KF_GLOBAL T* x_g = gp(static_cast<T*>(a.x));
  const KF_GLOBAL T* rho_g = gp(static_cast<const T*>(a.rho));
  const KF_GLOBAL T* var_g = gp(static_cast<const T*>(a.var));

  // per-pixel registers; pixel j of this thread is k = tid + j NT of the tile
  int lxy[PPT];   // (ly << 16) | lx, or -1 when the thread has no j-th pixel
  T xr[PPT], rr[PPT], pv[PPT], dg[PPT], idg[PPT], cR[PPT], cL[PPT], cD[PPT], cU[PPT];
  const T r_floor = (T)a.r_floor;
#define KF_LX(j) (lxy[j] & 0xffff)
#define KF_LY(j) (lxy[j] >> 16)
#define KF_LI(j) ((KF_LY(j) + 1) * rw + KF_LX(j) + 1)
#define KF_GI(j) ((oy + KF_LY(j)) * W + ox + KF_LX(j))
  // Table III drops the gradient terms; Table II solves a scale-ambiguous
  // log-depth y = x - tau from the semi-dense and gradient terms (tau held at
  // 0 inside the GN loop) and fits the scale afterwards
  const bool nopair = VAR && a.variant == KF_VARIANT_NO_PAIRWISE;
  const bool postfit = VAR && a.variant == KF_VARIANT_SCALE_POSTFIT;
  const bool tukey = VAR && a.robust == KF_ROBUST_TUKEY;
  double tau = scal->tau;
  const T x_shift = postfit ? (T)tau : (T)0;
  // keyframe rule (Sec. II): a frame that moved the camera too far from the
  // keyframe, or whose semi-dense update found too few inliers, is not fused
  int new_kf = 0;
  if (VAR && a.lambda_trans > 0.0 && scal->frame_trans[a.buf] > a.lambda_trans) new_kf |= KF_NEW_KEYFRAME_TRANSLATION;
  if (VAR && a.lambda_inliers > 0 && scal->n_updated[a.buf] < a.lambda_inliers) new_kf |= KF_NEW_KEYFRAME_INLIERS;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int k = tid + j * NT;
    lxy[j] = k < npx ? (((k / tw) << 16) | (k % tw)) : -1;
    xr[j] = rr[j] = pv[j] = dg[j] = idg[j] = cR[j] = cL[j] = cD[j] = cU[j] = (T)0;
    if (lxy[j] >= 0) {
      xr[j] = x_g[KF_GI(j)] - x_shift;
      xs[KF_LI(j)] = xr[j];
    }
  }
  // ghost x straight from the state (consistent at launch)
#pragma unroll
  for (int m = 0; m < GMAX; ++m) {
    if (tm.g_src[m] >= 0) {
      const int li_g = tm.g_li[m];
      const int gy_ = li_g / rw - 1, gx_ = li_g % rw - 1;
      xs[li_g] = x_g[(oy + gy_) * W + ox + gx_] - x_shift;
    }
  }
  // and its second ring (slots only where that pixel is inside the image)
#pragma unroll
  for (int m = 0; m < G2MAX; ++m) {
    if (tm.g2_src[m] >= 0) {
      int cx, cy;
      ring2_cell(tid + m * NT, tw, th, cx, cy);
      xs[tm.g2_li[m]] = x_g[(oy + cy) * W + ox + cx] - x_shift;
    }
  }
  if (postfit && !new_kf) tau = 0.0;
  __syncthreads();

  // epoch base of this launch: written by the previous launch's workgroup 0
  // after its team finished, so every workgroup here reads the same value
  const uint32_t e0 = scal->epoch;
  uint32_t e = e0;
  const bool tol_mode = a.cg_rtol > 0.0;
  const int limit = tol_mode ? a.cg_max : a.n_cg;
  int cg_total = 0;
  double relres = 0.0;
  double n_valid = 0.0;
  double vals[NV_MAX], tot[NV_MAX];
  T gval[GMAX];

  // semi-dense measurement in log space (Sec. II-B last step): z = -ln rho,
  // R = max(v / rho^2, R_floor); returns 1/sqrt(R), 0 when the pixel has none
  auto semi = [&](int gi, T& z) -> T {
    const T v = var_g[gi];
    if (!(v > (T)0)) {
      z = (T)0;
      return (T)0;
    }
    const T rho = rho_g[gi];
    z = -log(rho);
    T R = v / (rho * rho);
    R = R > r_floor ? R : r_floor;
    return (T)1 / sqrt(R);
  };

  // The static inputs of one row of the 5-point normal equations at pixel
  // i = (u, v): network log-depth and its inverse sigma, the semi-dense
  // measurement, and per gradient edge (right, left, lower, upper) the prior
  // gradient and its inverse sigma (zeros for an edge that leaves the image).
  struct RowData {
    T mu, isn, zs, isr, gR, sR, gL, sL, gD, sD, gU, sU;
  };
  auto row_data = [&](int i, int u, int v) -> RowData {
    RowData r;
    r.mu = mu_g[i];
    r.isn = isn_g[i];
    r.isr = semi(i, r.zs);
    r.gR = r.sR = r.gL = r.sL = r.gD = r.sD = r.gU = r.sU = (T)0;
    if (u < W - 1) {
      r.gR = gx_g[i]; r.sR = isgx_g[i];
    }
    if (u > 0) {
      r.gL = gx_g[i - 1]; r.sL = isgx_g[i - 1];
    }
    if (v < H - 1) {
      r.gD = gy_g[i]; r.sD = isgy_g[i];
    }
    if (v > 0) {
      r.gU = gy_g[i - W]; r.sU = isgy_g[i - W];
    }
    return r;
  };

  // The row (Sec. II-C) at log-depth xi with its right / left / lower / upper
  // neighbours' values: IRLS weights of the unary terms, couplings of the
  // gradient edges (none for an edge that leaves the image, none at all
  // without `edges`), diagonal and right-hand side. Own pixels and ghost
  // pixels share it, so a ghost row repeats its owner's arithmetic.
  struct Row {
    T wn, ws, bb, cr, cl, cd, cu, d;
  };
  auto row_at = [&](const RowData& r, int u, int v, T xi, T xR, T xL, T xD, T xU, bool edges) -> Row {
    Row q;
    q.wn = postfit ? (T)0 : huber_w((xi - r.mu) * r.isn, delta, tukey) * r.isn * r.isn;
    q.ws = (T)0;
    if (r.isr > (T)0) q.ws = huber_w((xi - (T)tau - r.zs) * r.isr, delta, tukey) * r.isr * r.isr;
    T bb = q.wn * r.mu + q.ws * ((T)tau + r.zs);
    T cr = 0, cl = 0, cd = 0, cu = 0;
    if (edges) {
      if (u < W - 1) {
        cr = edge_weight(xi, xR, r.gR, r.sR, delta, tukey);
        bb -= cr * r.gR;
      }
      if (u > 0) {
        cl = edge_weight(xL, xi, r.gL, r.sL, delta, tukey);
        bb += cl * r.gL;
      }
      if (v < H - 1) {
        cd = edge_weight(xi, xD, r.gD, r.sD, delta, tukey);
        bb -= cd * r.gD;
      }
      if (v > 0) {
        cu = edge_weight(xU, xi, r.gU, r.sU, delta, tukey);
        bb += cu * r.gU;
      }
    }
    q.bb = bb;
    q.cr = cr; q.cl = cl; q.cd = cd; q.cu = cu;
    q.d = q.wn + q.ws + cr + cl + cd + cu;
    return q;
  };

  // Fixed-count pipelined CG with tiles at least 2 x 2: the first stencil
  // operand's ghost values are assembled locally (x is known two pixels deep
  // around the tile), which saves the initial-residual synchronisation of
  // every GN iteration. gz_c0: this thread's first ghost cell; the cells start
  // at the first wavefront whose threads hold one pixel fewer than PPT.
  const bool ghost_z = PIPE && !tol_mode && a.ghost_z != 0;
  T* x2 = lds.x2;
  T* gdat = lds.gdat;   // [12][perim]: the ghost cells' RowData, filled once per launch
  const int perim = a.perim;
  int gz_c0;
  {
    const int full = npx - (PPT - 1) * NT;   // threads [0, full) hold PPT pixels
    int t0 = full <= 0 ? 0 : ((full + 63) / 64) * 64;
    t0 = t0 < NT ? t0 : 0;
    gz_c0 = tid - t0;
    if (gz_c0 < 0) gz_c0 += NT;
  }
  // ghost cell c of the first ring: tile coordinates and the neighbour that owns it (-1: none)
  auto ghost_cell = [&](int c, int& gx, int& gy) -> int {
    if (c < tw) {
      gx = c; gy = -1; return tm.nb_up;
    } else if (c < 2 * tw) {
      gx = c - tw; gy = th; return tm.nb_dn;
    } else if (c < 2 * tw + th) {
      gx = -1; gy = c - 2 * tw; return tm.nb_lf;
    }
    gx = tw; gy = c - 2 * tw - th; return tm.nb_rt;
  };
  if (ghost_z && !nopair) {
    // the static part of this thread's ghost rows, read once; the same thread
    // reads it back in every GN iteration (no barrier needed)
#pragma unroll
    for (int m = 0; m < GMAX; ++m) {
      const int c = gz_c0 + m * NT;
      if (c >= 2 * tw + 2 * th) continue;
      int gx, gy;
      if (ghost_cell(c, gx, gy) < 0) continue;
      const int u = ox + gx, v = oy + gy;
      const RowData r = row_data(v * W + u, u, v);
      const T vals12[12] = {r.mu, r.isn, r.zs, r.isr, r.gR, r.sR, r.gL, r.sL, r.gD, r.sD, r.gU, r.sU};
#pragma unroll
      for (int k = 0; k < 12; ++k) gdat[k * perim + c] = vals12[k];
    }
  }

  for (int gn = 0; gn < (new_kf ? 0 : a.n_gn); ++gn) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) refresh(lxy[j]);
    // ---- IRLS weights and 5-point normal equations at (x, tau) (Sec. II-C);
    //      r = b - A x, z = r / diag, p = z
    double rz = 0.0, r2 = 0.0, b2 = 0.0;
    if (ghost_z && !nopair) {
      // z of the ghost ring assembled here from the two-deep x boundary (the
      // same row arithmetic as its owner's), instead of a synchronisation that
      // ships it; cells spread over the threads with the fewest own pixels
      // (the cell index is redefined here, so the compiler forms the cells'
      // addresses inside the GN loop instead of keeping them live all launch)
      int gc0 = gz_c0;
      refresh(gc0);
#pragma unroll
      for (int m = 0; m < GMAX; ++m) {
        const int c = gc0 + m * NT;
        if (c >= 2 * tw + 2 * th) continue;
        int gx, gy;
        if (ghost_cell(c, gx, gy) < 0) continue;
        const int lg = (gy + 1) * rw + gx + 1;
        const T xg = xs[lg];
        const T xR = gx == tw ? x2[2 * tw + th + gy] : xs[lg + 1];
        const T xL = gx == -1 ? x2[2 * tw + gy] : xs[lg - 1];
        const T xD = gy == th ? x2[tw + gx] : xs[lg + rw];
        const T xU = gy == -1 ? x2[gx] : xs[lg - rw];
        const int u = ox + gx, v = oy + gy;
        RowData r;
        r.mu = gdat[c]; r.isn = gdat[perim + c]; r.zs = gdat[2 * perim + c]; r.isr = gdat[3 * perim + c];
        r.gR = gdat[4 * perim + c]; r.sR = gdat[5 * perim + c]; r.gL = gdat[6 * perim + c];
        r.sL = gdat[7 * perim + c]; r.gD = gdat[8 * perim + c]; r.sD = gdat[9 * perim + c];
        r.gU = gdat[10 * perim + c]; r.sU = gdat[11 * perim + c];
        const Row q = row_at(r, u, v, xg, xR, xL, xD, xU, true);
        const T ig = q.d > (T)0 ? (T)1 / q.d : (T)0;
        const T ax = q.d * xg - q.cr * xR - q.cl * xL - q.cd * xD - q.cu * xU;
        ps[lg] = (q.bb - ax) * ig;
      }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (lxy[j] < 0) continue;
      const int u = ox + KF_LX(j), v = oy + KF_LY(j);
      const int i = KF_GI(j), l = KF_LI(j);
      const T xi = xr[j];
      const T xR = xs[l + 1], xL = xs[l - 1], xD = xs[l + rw], xU = xs[l - rw];
      const Row q = row_at(row_data(i, u, v), u, v, xi, xR, xL, xD, xU, !nopair);
      if (nopair) {
        // per-pixel weighted mean of the network and semi-dense log-depths
        if (q.wn + q.ws > (T)0) xr[j] = q.bb / (q.wn + q.ws);
        continue;
      }
      dg[j] = q.d;
      idg[j] = q.d > (T)0 ? (T)1 / q.d : (T)0;   // d = 0 only without network and gradient terms
      cR[j] = q.cr; cL[j] = q.cl; cD[j] = q.cd; cU[j] = q.cu;
      const T ax = q.d * xi - q.cr * xR - q.cl * xL - q.cd * xD - q.cu * xU;
      const T r = q.bb - ax;
      rr[j] = r;
      const T z = r * idg[j];
      pv[j] = z;
      ps[l] = z;
      rz += (double)r * (double)z;
      r2 += (double)r * (double)r;
      b2 += (double)q.bb * (double)q.bb;
    }
    int it = 0;
    T qv[PPT];
    if (!nopair) {
    double rz_t = 0.0, bnorm = 0.0;
    if (ghost_z) {
      __syncthreads();
    } else {
      vals[0] = rz; vals[1] = r2; vals[2] = b2;
      if (!tm.sync(e++, tol_mode ? 3 : 1, vals, tot, gval, true, ps, true)) return;
      rz_t = tot[0];
      bnorm = tol_mode ? sqrt(tot[2]) : 0.0;
    }
    bool converged = false;
    if (tol_mode) {
      relres = bnorm > 0.0 ? sqrt(tot[1]) / bnorm : 0.0;
      converged = sqrt(tot[1]) <= a.cg_rtol * bnorm;
    }

    if (PIPE) {
      // Pipelined Jacobi PCG (Ghysels and Vanroose): the same iterates as the
      // textbook recurrences in exact arithmetic, with the two inner products
      // of an iteration reduced together and overlapped with the stencil
      // product n = A m, so each iteration needs ONE team synchronisation
      // (partials gamma = r.u, delta = w.u plus the boundary of m).
      // ps holds u_0 = z_0 (own + ghost ring).
      T uv[PPT], wv[PPT], mv[PPT], zv[PPT], sv[PPT];
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        uv[j] = pv[j];
        wv[j] = mv[j] = zv[j] = sv[j] = qv[j] = (T)0;
        if (lxy[j] < 0) continue;
        const int l = KF_LI(j);
        const T w = dg[j] * uv[j] - cR[j] * ps[l + 1] - cL[j] * ps[l - 1] - cD[j] * ps[l + rw] - cU[j] * ps[l - rw];
        wv[j] = w;
        mv[j] = w * idg[j];
        ms0[l] = mv[j];
      }
      // alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}); with
      // den_i = gamma_i / alpha_i the last term is beta_i^2 den_{i-1}, so only
      // one division (by den_i) waits for the team totals: 1 / gamma_i is
      // formed beside the vector updates for the next iteration's beta
      double rgamma_prev = 1.0, den_prev = 1.0;
      for (int i = 0; i < limit && !converged; ++i) {
        T* mring = (i & 1) ? ps : ms0;
        T* mnext = (i & 1) ? ms0 : ps;
#pragma unroll
        for (int j = 0; j < PPT; ++j) refresh(lxy[j]);
        double ga = 0.0, de = 0.0;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          if (lxy[j] < 0) continue;
          ga += (double)rr[j] * (double)uv[j];
          de += (double)wv[j] * (double)uv[j];
        }
        vals[0] = ga; vals[1] = de;
        // the stencil product of the tile's interior pixels needs no ghost
        // value: it is formed while the team's words are in flight (for up to
        // 4 pixels per thread; with more, the extra registers cost more than
        // the overlap gains)
        constexpr bool OVERLAP = PPT <= 4;
        T nint[PPT];
        auto interior = [&] {
#pragma unroll
          for (int j = 0; j < PPT; ++j) {
            nint[j] = (T)0;
            if (!OVERLAP || lxy[j] < 0) continue;
            const int lx = KF_LX(j), ly = KF_LY(j);
            if (lx == 0 || ly == 0 || lx == tw - 1 || ly == th - 1) continue;
            const int l = KF_LI(j);
            nint[j] = dg[j] * mv[j] - cR[j] * mring[l + 1] - cL[j] * mring[l - 1] - cD[j] * mring[l + rw] -
                      cU[j] * mring[l - rw];
          }
        };
        // the neighbours' m lands directly in the ghost ring of mring
        if (!tm.template sync<false>(e++, 2, vals, tot, gval, true, mring, true, interior)) return;
        if (tot[0] == 0.0) break;
        double beta = 0.0, den = tot[1];
        if (i > 0) {
          beta = tot[0] * rgamma_prev;
          den = tot[1] - beta * beta * den_prev;
        }
        const double alpha = tot[0] / den;
        rgamma_prev = 1.0 / tot[0];
        den_prev = den;
        const T al = (T)alpha, be = (T)beta;
        const bool last = i == limit - 1;
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
          if (lxy[j] < 0) continue;
          pv[j] = i > 0 ? fma(be, pv[j], uv[j]) : uv[j];
          xr[j] = fma(al, pv[j], xr[j]);
          if (last) continue;
          const int l = KF_LI(j);
          const int lx = KF_LX(j), ly = KF_LY(j);
          T n = nint[j];
          if (!OVERLAP || lx == 0 || ly == 0 || lx == tw - 1 || ly == th - 1)
            n = dg[j] * mv[j] - cR[j] * mring[l + 1] - cL[j] * mring[l - 1] - cD[j] * mring[l + rw] -
                cU[j] * mring[l - rw];
          zv[j] = i > 0 ? fma(be, zv[j], n) : n;
          qv[j] = i > 0 ? fma(be, qv[j], mv[j]) : mv[j];
          sv[j] = i > 0 ? fma(be, sv[j], wv[j]) : wv[j];
          rr[j] = fma(-al, sv[j], rr[j]);
          uv[j] = fma(-al, qv[j], uv[j]);
          wv[j] = fma(-al, zv[j], wv[j]);
          mv[j] = wv[j] * idg[j];
          mnext[l] = mv[j];
        }
        ++it;
      }
    }
    while (!PIPE && !converged && it < limit && rz_t != 0.0) {
      // q = A p (5-point stencil; ghost ring holds the neighbours' p)
#pragma unroll
      for (int j = 0; j < PPT; ++j) refresh(lxy[j]);
      double pq = 0.0;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        qv[j] = (T)0;
        if (lxy[j] < 0) continue;
        const int l = KF_LI(j);
        const T q = dg[j] * pv[j] - cR[j] * ps[l + 1] - cL[j] * ps[l - 1] - cD[j] * ps[l + rw] - cU[j] * ps[l - rw];
        qv[j] = q;
        pq += (double)pv[j] * (double)q;
      }
      vals[0] = pq;
      if (!tm.sync(e++, 1, vals, tot, gval, false)) return;
      const double alpha = rz_t / tot[0];
      const T al = (T)alpha;
      double rzn = 0.0, rrn = 0.0;
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        if (lxy[j] < 0) continue;
        xr[j] += al * pv[j];
        rr[j] -= al * qv[j];
        const T z = rr[j] * idg[j];
        qv[j] = z;   // reuse as z
        rzn += (double)rr[j] * (double)z;
        rrn += (double)rr[j] * (double)rr[j];
      }
      ++it;
      if (!tol_mode && it == limit) break;
#pragma unroll
      for (int j = 0; j < PPT; ++j)
        if (lxy[j] >= 0) tm.publish(e, KF_LX(j), KF_LY(j), qv[j]);
      vals[0] = rzn; vals[1] = rrn;
      // ghost z arrives in gval: the ghost copy of p needs beta first
      if (!tm.sync(e++, tol_mode ? 2 : 1, vals, tot, gval, true)) return;
      if (tol_mode) {
        relres = bnorm > 0.0 ? sqrt(tot[1]) / bnorm : 0.0;
        if (sqrt(tot[1]) <= a.cg_rtol * bnorm) {
          converged = true;
          break;
        }
      }
      const T be = (T)(tot[0] / rz_t);
      rz_t = tot[0];
#pragma unroll
      for (int j = 0; j < PPT; ++j) {
        if (lxy[j] < 0) continue;
        pv[j] = fma(be, pv[j], qv[j]);
        ps[KF_LI(j)] = pv[j];
      }
#pragma unroll
      for (int m = 0; m < GMAX; ++m)
        if (tm.g_src[m] >= 0) ps[tm.g_li[m]] = fma(be, ps[tm.g_li[m]], gval[m]);
      __syncthreads();
    }
    }   // !nopair
    cg_total += it;

    // ---- scale step: semi weights at (x_new, tau), tau = sum w (x - z) / sum w (R13)
#pragma unroll
    for (int j = 0; j < PPT; ++j) refresh(lxy[j]);
    double num = 0.0, den = 0.0, cnt = 0.0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      if (lxy[j] < 0) continue;
      T zs;
      const T isr = semi(KF_GI(j), zs);
      if (isr > (T)0) {
        const T w = huber_w((xr[j] - (T)tau - zs) * isr, delta, tukey) * isr * isr;
        num += (double)w * (double)(xr[j] - zs);
        den += (double)w;
        cnt += 1.0;
      }
      xs[KF_LI(j)] = xr[j];
    }
    vals[0] = num; vals[1] = den; vals[2] = cnt;
    // the neighbours' x lands directly in the ghost ring of xs (with
    // ghost_z also its second ring and corners); the count of pixels with a
    // semi-dense measurement does not change over the GN iterations, so only
    // the first scale step reduces it
    const int nv_scale = gn == 0 ? 3 : 2;
    if constexpr (PIPE) {
      const uint32_t es = e;
      auto pub2 = [&] {
        if (ghost_z) tm.publish_ring2(es, xs);
      };
      if (!tm.template sync<true>(e++, nv_scale, vals, tot, gval, true, xs, true, pub2)) return;
    } else {
      if (!tm.sync(e++, nv_scale, vals, tot, gval, true, xs, true)) return;
    }
    if (!postfit && tot[1] > 0.0) tau = tot[0] / tot[1];
    if (gn == 0) n_valid = tot[2];
  }
  if (postfit && !new_kf) {
    // least-squares fit of the log-scale to the network: tau = mean(mu - y)
    double dev = 0.0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      refresh(lxy[j]);
      if (lxy[j] >= 0) dev += (double)mu_g[KF_GI(j)] - (double)xr[j];
    }
    vals[0] = dev;
    if (!tm.sync(e++, 1, vals, tot, gval, false)) return;
    tau = tot[0] / (double)N;
#pragma unroll
    for (int j = 0; j < PPT; ++j) xr[j] += (T)tau;
  }

#pragma unroll
  for (int j = 0; j < PPT; ++j)
    if (lxy[j] >= 0 && !new_kf) x_g[KF_GI(j)] = xr[j];
#undef KF_LX
#undef KF_LY
#undef KF_LI
#undef KF_GI
  if (b == 0 && tid == 0) {
    // every member has read e0 before its first publish, and workgroup 0
    // passed the last synchronisation, so no member still needs the old base
    // a launch that made no synchronisation (new keyframe) keeps the base:
    // then every exchange slot's last write stays within one launch span of
    // its next poll, whatever runs of such launches occur, which the 16-bit
    // tags of one-word partials rely on
    scal->epoch = e0 + (e != e0 ? a.epoch_span : 0u);
    scal->tau = tau;
    scal->cg_iterations = cg_total;
    scal->cg_rel_residual = relres;
    if (!new_kf) scal->n_valid = (int32_t)n_valid;
    scal->team_syncs = (int32_t)(e - e0);
    scal->new_keyframe = new_kf;
  }
}

template <typename T, int NT, int PPT, bool PIPE, bool VAR>
__global__ __launch_bounds__(NT) void k_solve(SolveArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  solve_member<T, NT, PPT, PIPE, VAR>(a, blockIdx.x, smem);
}

// Batched form: workgroup g works through its queue of (keyframe, member)
// entries in order. Queues list teams in one global order, so the lowest
// unfinished team always has every member at it and the launch cannot
// deadlock, provided all workgroups are co-resident. FP32 512-thread
// workgroups of up to 4 pixels per thread are held to 128 registers so that two
// of them share a compute unit (one computes while the other's team
// synchronises).
template <typename T, int NT, int PPT, bool PIPE, bool VAR>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && NT == 512 && NT * PPT <= 2048 ? 4 : 1)))
void k_solve_batch(const SolveArgs* __restrict__ tab,
                                                    const int32_t* __restrict__ queue,
                                                    const int32_t* __restrict__ qoff) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int q1 = qoff[blockIdx.x + 1];
  for (int q = qoff[blockIdx.x]; q < q1; ++q) {
    const int32_t ent = queue[q];
    const SolveArgs a = tab[ent >> 8];
    __syncthreads();   // the previous member's last LDS reads are done
    solve_member<T, NT, PPT, PIPE, VAR>(a, ent & 255, smem);
  }
}

// Synchronisation probe: the team of `a` makes `rounds` exchanges of the kind
// a pipelined PCG iteration makes (nv partial sums and the tile boundary of a
// stencil operand, through the same Team::sync) with no arithmetic between
// them, so launch time / rounds is the cost of one team synchronisation at
// this layout.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_sync_probe(SolveArgs a, int rounds, int nv) {
  extern __shared__ __align__(16) unsigned char smem[];
  Team<T, NT> tm;
  MemberLds<T, NT> lds;
  team_init(tm, lds, a, blockIdx.x, smem);
  KF_GLOBAL DevScalars* scal = gp(a.scal);
  const uint32_t e0 = scal->epoch;
  uint32_t e = e0;
  double vals[NV_MAX], tot[NV_MAX];
  T gval[GMAX];
#pragma unroll
  for (int v = 0; v < NV_MAX; ++v) vals[v] = (double)threadIdx.x;
  for (int r = 0; r < rounds; ++r) {
    T* ring = (r & 1) ? lds.ps : lds.ms0;
    if (!tm.sync(e++, nv, vals, tot, gval, true, ring, true)) return;
    vals[0] = tot[0] * 0x1p-100;   // the next round depends on this one's totals
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal->epoch = e0 + a.epoch_span;
    scal->team_syncs = (int32_t)(e - e0);
  }
}

}  // namespace

namespace {

// (threads, pixels per thread) combinations whose registers fit without
// scratch spills (the ppt_max table of the host side follows these)
#define KF_SOLVE_COMBOS                                                              \
  KF_PPT(256, 1) KF_PPT(256, 2) KF_PPT(256, 3) KF_PPT(256, 4) KF_PPT(256, 6)          \
  KF_PPT(512, 1) KF_PPT(512, 2) KF_PPT(512, 3) KF_PPT(512, 4)                         \
  KF_PPT(1024, 1)                                                                     \
  if constexpr (sizeof(T) == 4) {                                                     \
    KF_PPT(256, 8) KF_PPT(512, 6) KF_PPT(512, 8) KF_PPT(512, 10) KF_PPT(1024, 2)      \
    KF_PPT(1024, 3)                                                                   \
  }

size_t smem_for(size_t elt, const Tiling& t) {
  const size_t ring = (size_t)(t.tile_h + 2) * (t.tile_w + 2);
  const size_t ring2 = 2 * (size_t)t.tile_w + 2 * (size_t)t.tile_h;
  return sizeof(double) * ((size_t)(t.threads / 64) * NV_MAX + NV_MAX * (MAX_TEAM / 64) + 2) + (3 * ring + 13 * ring2) * elt;
}

template <typename T, bool PIPE, bool VAR>
const void* solve_fn_p(const Tiling& t) {
#define KF_PPT(nt, n) if (t.threads == nt && t.ppt == n) return reinterpret_cast<const void*>(&k_solve<T, nt, n, PIPE, VAR>);
  KF_SOLVE_COMBOS
#undef KF_PPT
  return nullptr;
}

// kind: bit 0 pipelined CG, bit 1 the instantiation with the variants and the keyframe rule
template <typename T>
const void* solve_fn(const Tiling& t, int kind) {
  switch (kind & 3) {
    case 0: return solve_fn_p<T, false, false>(t);
    case 1: return solve_fn_p<T, true, false>(t);
    case 2: return solve_fn_p<T, false, true>(t);
    default: return solve_fn_p<T, true, true>(t);
  }
}

template <typename T, bool PIPE, bool VAR>
const void* batch_fn_p(int threads, int ppt) {
#define KF_PPT(nt, n) if (threads == nt && ppt == n) return reinterpret_cast<const void*>(&k_solve_batch<T, nt, n, PIPE, VAR>);
  KF_SOLVE_COMBOS
#undef KF_PPT
  return nullptr;
}

template <typename T>
const void* batch_fn_t(int threads, int ppt, int kind) {
  switch (kind & 3) {
    case 0: return batch_fn_p<T, false, false>(threads, ppt);
    case 1: return batch_fn_p<T, true, false>(threads, ppt);
    case 2: return batch_fn_p<T, false, true>(threads, ppt);
    default: return batch_fn_p<T, true, true>(threads, ppt);
  }
}

const void* batch_fn(int prec, int threads, int ppt, int kind) {
  return prec == KF_F64 ? batch_fn_t<double>(threads, ppt, kind) : batch_fn_t<float>(threads, ppt, kind);
}

template <typename T>
hipError_t solve_t(const Tiling& t, const SolveArgs& a, bool cooperative, int kind, hipStream_t s) {
  const size_t sm = smem_for(sizeof(T), t);
  void* args[] = {const_cast<SolveArgs*>(&a)};
  const void* fn = solve_fn<T>(t, kind);
  if (!fn) return hipErrorInvalidValue;
  if (sm > 48 * 1024) {
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (err != hipSuccess) return err;
  }
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(t.blocks), dim3(t.threads), args, (unsigned)sm, s);
  return hipLaunchKernel(fn, dim3(t.blocks), dim3(t.threads), args, (unsigned)sm, s);
}

}  // namespace

size_t solve_smem_bytes(int prec, const Tiling& t) { return smem_for(prec == KF_F64 ? 8 : 4, t); }

// Workgroups of kernel fn the device holds at once with `smem` bytes of LDS
// each; 0 (and the runtime's error state cleared) if a query fails.
int coresident_of(const void* fn, int threads, size_t smem, int device) {
  int per_cu = 0, cus = 0;
  hipError_t e = hipSuccess;
  if (smem > 48 * 1024) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, smem);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per_cu * cus;
}

int solve_max_coresident(int prec, const Tiling& t, int kind, int device) {
  const void* fn = prec == KF_F64 ? solve_fn<double>(t, kind) : solve_fn<float>(t, kind);
  if (!fn) return 0;
  return coresident_of(fn, t.threads, solve_smem_bytes(prec, t), device);
}

hipError_t launch_solve(int prec, const Tiling& t, const SolveArgs& a, bool cooperative, int kind, hipStream_t s) {
  if (prec == KF_F64) return solve_t<double>(t, a, cooperative, kind, s);
  return solve_t<float>(t, a, cooperative, kind, s);
}

hipError_t launch_sync_probe(int prec, const Tiling& t, const SolveArgs& a, int rounds, int nv, hipStream_t s) {
  const void* fn = nullptr;
  if (prec == KF_F64) {
    fn = t.threads == 256 ? reinterpret_cast<const void*>(&k_sync_probe<double, 256>)
         : t.threads == 512 ? reinterpret_cast<const void*>(&k_sync_probe<double, 512>)
                            : reinterpret_cast<const void*>(&k_sync_probe<double, 1024>);
  } else {
    fn = t.threads == 256 ? reinterpret_cast<const void*>(&k_sync_probe<float, 256>)
         : t.threads == 512 ? reinterpret_cast<const void*>(&k_sync_probe<float, 512>)
                            : reinterpret_cast<const void*>(&k_sync_probe<float, 1024>);
  }
  const size_t sm = solve_smem_bytes(prec, t);
  if (sm > 48 * 1024) {
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (err != hipSuccess) return err;
  }
  void* args[] = {const_cast<SolveArgs*>(&a), &rounds, &nv};
  return hipLaunchKernel(fn, dim3(t.blocks), dim3(t.threads), args, (unsigned)sm, s);
}

bool solve_batch_supported(int prec, int threads, int ppt) { return batch_fn(prec, threads, ppt, 1) != nullptr; }

int solve_batch_coresident(int prec, int threads, int ppt, int kind, size_t smem, int device) {
  const void* fn = batch_fn(prec, threads, ppt, kind);
  if (!fn) return 0;
  return coresident_of(fn, threads, smem, device);
}

hipError_t launch_solve_batch(int prec, int threads, int ppt, int kind, const SolveArgs* tab,
                              const int32_t* queue, const int32_t* qoff, int grid, size_t smem, hipStream_t s) {
  const void* fn = batch_fn(prec, threads, ppt, kind);
  if (!fn || grid < 1) return hipErrorInvalidValue;
  void* args[] = {const_cast<SolveArgs**>(&tab), const_cast<int32_t**>(&queue), const_cast<int32_t**>(&qoff)};
  return hipLaunchKernel(fn, dim3(grid), dim3(threads), args, (unsigned)smem, s);
}

}  // namespace kf
