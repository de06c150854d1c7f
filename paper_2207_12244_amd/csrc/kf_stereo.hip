// Semi-dense estimation (Sec. II-B): epipolar SSD search, interpolation between
// two steps, variance of eq. (semi), inverse-depth Gaussian filter.
//
// Work mapping: a group of G lanes of one wavefront (lanes_per_pixel) handles
// one textured keyframe pixel; lane l of the group evaluates S = N_s / G
// samples: k = l S, ..., l S + S - 1 for the 5-point line pattern (consecutive
// samples share four of their five points when the step is 1 px) and k = l,
// l + G, ... for the 5 x 5 patch. The keyframe pattern (5 or 25 values) is
// evaluated once per pixel and handed to every lane of the group by cross-lane
// broadcasts when the group has a lane per point, otherwise by every lane;
// the argmin over the N_s SSDs is a butterfly of cross-lane shuffles inside
// the group with ties resolved to the smaller k. No LDS, no barriers.
#include <type_traits>

#include "kf_internal.h"

namespace kf {

namespace {

constexpr int ST_THREADS = 256;
constexpr int ST_WAVES = ST_THREADS / 64;

// Lanes of a wavefront that share one textured pixel: N_s / 16, i.e. 16
// samples per lane, for both patterns. The per-pixel work (geometry, argmin,
// sub-pixel step, filter, and for the 25-point patch below 25 lanes the
// keyframe pattern itself) is repeated by every lane of the group, so smaller
// groups do less of it per pixel; 16 samples per lane is where the lane's own
// sample registers still fit. Measured per 640 x 480 frame with a grid of 8
// workgroups per compute unit: SQ5X5 at N_s = 32 / 64 / 128 takes 63 / 93 /
// 138 us (f32) with 2 / 4 / 8 lanes, against 134 / 141 / 156 us with 32 lanes
// and 229 us with 4 lanes at N_s = 128; LINE5 at N_s = 32 and 64 is slower
// with half or twice its group. With the resident grid (bf16 form, N_s =
// 128): 103 us with 8 lanes, 120 / 118 us with 16 / 4. The argmin is a
// lexicographic (SSD, k) minimum, so the split only changes which lane
// evaluates a sample.
constexpr int lanes_per_pixel(int, int ns) {
  return ns / 16 < 1 ? 1 : (ns / 16 > 64 ? 64 : ns / 16);
}

template <typename T>
struct PixelGeom {
  T A0, A1, A2;      // H (u, v, 1)
  T cx, cy;          // segment centre in image 1
  T lx, ly;          // unit direction of the segment (image 1)
  T h;               // step between samples (>= 1 px)
  T l0x, l0y;        // keyframe epipolar direction (LINE5)
  bool use_x;        // solve rho from the x coordinate
  bool ok;
};

// Two consecutive uint8 taps at byte address p of the staged frame from the
// two aligned dwords that hold them (rows are padded by >= 8 bytes, so the
// second dword is in bounds) and one byte-align.
template <typename T>
__device__ inline void tap_pair(const KF_GLOBAL uint8_t* p, T& t0, T& t1) {
  const uintptr_t a = (uintptr_t)p;
  const KF_GLOBAL uint32_t* w = (const KF_GLOBAL uint32_t*)(a & ~(uintptr_t)3);
  const uint32_t v = __builtin_amdgcn_alignbyte(w[1], w[0], (uint32_t)(a & 3u));
  t0 = (T)(v & 0xffu);
  t1 = (T)((v >> 8) & 0xffu);
}

// Bilinear intensity of the staged new frame (uint8, row stride `st`) at
// (u, v), 0 <= u <= W-1, 0 <= v <= H-1.
template <typename T>
__device__ inline T bilin_u8(const KF_GLOBAL uint8_t* img, int st, int W, int H, T u, T v) {
  T fu = floor(u), fv = floor(v);
  fu = fu < (T)(W - 2) ? fu : (T)(W - 2);
  fv = fv < (T)(H - 2) ? fv : (T)(H - 2);
  fu = fu > (T)0 ? fu : (T)0;
  fv = fv > (T)0 ? fv : (T)0;
  const T f = u - fu, g = v - fv;
  const size_t i = (size_t)(int)fv * st + (int)fu;
  T i00, i10, i01, i11;
  tap_pair<T>(img + i, i00, i10);
  tap_pair<T>(img + i + st, i01, i11);
  const T top = i00 + f * (i10 - i00);
  const T bot = i01 + f * (i11 - i01);
  return top + g * (bot - top);
}

// Six consecutive uint8 taps starting at byte address p of the staged frame
// (rows are padded, so reading up to 8 bytes past a row's last pixel is in
// bounds): three aligned dword loads and two byte-aligns.
template <typename T>
__device__ inline void taps6(const KF_GLOBAL uint8_t* p, T* t) {
  const uintptr_t a = (uintptr_t)p;
  const KF_GLOBAL uint32_t* w = (const KF_GLOBAL uint32_t*)(a & ~(uintptr_t)3);
  const uint32_t sh = (uint32_t)(a & 3u);
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
  const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w1, sh);
  t[0] = (T)(lo & 0xffu);
  t[1] = (T)((lo >> 8) & 0xffu);
  t[2] = (T)((lo >> 16) & 0xffu);
  t[3] = (T)(lo >> 24);
  t[4] = (T)(hi & 0xffu);
  t[5] = (T)((hi >> 8) & 0xffu);
}

// Five consecutive bf16 elements of the keyframe image from element index e
// on, as floats, from the three aligned dwords that hold them: one dword load
// per two elements instead of one load each. The image is followed by more
// workspace, so the dword that holds its last element is in bounds.
__device__ inline void row5_bf16(const KF_GLOBAL bf16* img, size_t e, float* t) {
  const KF_GLOBAL uint32_t* w = (const KF_GLOBAL uint32_t*)(img + (e & ~(size_t)1));
  const uint32_t sh = (uint32_t)(e & 1) * 2u;
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
  const uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh);
  const uint32_t mid = __builtin_amdgcn_alignbyte(w2, w1, sh);
  const uint32_t hi = __builtin_amdgcn_alignbyte(w2, w2, sh);   // low half: element e + 4
  t[0] = __uint_as_float(lo << 16);
  t[1] = __uint_as_float(lo & 0xffff0000u);
  t[2] = __uint_as_float(mid << 16);
  t[3] = __uint_as_float(mid & 0xffff0000u);
  t[4] = __uint_as_float(hi << 16);
}

// Same for the resident keyframe image (storage type TI).
template <typename T, typename TI>
__device__ inline T bilin_kf(const KF_GLOBAL TI* img, int W, int H, T u, T v) {
  T fu = floor(u), fv = floor(v);
  fu = fu < (T)(W - 2) ? fu : (T)(W - 2);
  fv = fv < (T)(H - 2) ? fv : (T)(H - 2);
  fu = fu > (T)0 ? fu : (T)0;
  fv = fv > (T)0 ? fv : (T)0;
  const T f = u - fu, g = v - fv;
  const size_t i = (size_t)(int)fv * W + (int)fu;
  const T i00 = img_value(img[i]), i10 = img_value(img[i + 1]);
  const T i01 = img_value(img[i + W]), i11 = img_value(img[i + W + 1]);
  const T top = i00 + f * (i10 - i00);
  const T bot = i01 + f * (i11 - i01);
  return top + g * (bot - top);
}

template <typename T>
__device__ inline bool inside(T u, T v, int W, int H) {
  return u >= (T)0 && u <= (T)(W - 1) && v >= (T)0 && v <= (T)(H - 1);
}

// Epipolar geometry of one pixel (identical in every lane of its group).
// The image of the ray is a straight line: p(rho) - p(rho') =
// (rho - rho') (b_xy A_z - A_xy b_z) / (Z(rho) Z(rho')), with Z(rho) = A_z + rho b_z.
// Once the filter is confident the interval projects to a segment far shorter
// than a pixel, and the difference of its two nearly equal endpoints would keep
// few digits in FP32 (samples tens of pixels from the centre would sit a tenth
// of a pixel off the line); so the float forms take the direction as
// b_xy A_z - A_xy b_z normalised and the length from the same identity. FP64
// takes the endpoint difference itself.
template <typename T, int PAT, int NS>
__device__ inline PixelGeom<T> pixel_geometry(const StereoArgs& a, T u, T v, T rho, T var, bool has) {
  const FrameConst& c = a.fc;
  PixelGeom<T> g;
  const T H0 = (T)c.Hm[0], H1 = (T)c.Hm[1], H2 = (T)c.Hm[2];
  const T H3 = (T)c.Hm[3], H4 = (T)c.Hm[4], H5 = (T)c.Hm[5];
  const T H6 = (T)c.Hm[6], H7 = (T)c.Hm[7], H8 = (T)c.Hm[8];
  const T b0 = (T)c.b[0], b1 = (T)c.b[1], b2 = (T)c.b[2];
  const T rmin = (T)c.rho_min, rmax = (T)c.rho_max;
  g.A0 = H0 * u + H1 * v + H2;
  g.A1 = H3 * u + H4 * v + H5;
  g.A2 = H6 * u + H7 * v + H8;
  // search interval in inverse depth: rho +- 2 sigma clamped, or the whole range
  T lo = rmin, hi = rmax;
  if (has) {
    const T sd = sqrt(var);
    lo = rho - (T)2 * sd;
    lo = lo > rmin ? lo : rmin;
    hi = rho + (T)2 * sd;
    hi = hi < rmax ? hi : rmax;
  }
  g.ok = hi > lo;
  const T dlo = g.A2 + lo * b2, dhi = g.A2 + hi * b2;
  g.ok = g.ok && dlo > (T)0 && dhi > (T)0;
  const T plx = (g.A0 + lo * b0) / dlo, ply = (g.A1 + lo * b1) / dlo;
  const T phx = (g.A0 + hi * b0) / dhi, phy = (g.A1 + hi * b1) / dhi;
  T L, lx, ly;
  if constexpr (sizeof(T) == 8) {
    const T dx = phx - plx, dy = phy - ply;
    L = sqrt(dx * dx + dy * dy);
    lx = dx / L;
    ly = dy / L;
  } else {
    const T Dx = b0 * g.A2 - g.A0 * b2, Dy = b1 * g.A2 - g.A1 * b2;
    const T nD = sqrt(Dx * Dx + Dy * Dy);
    L = nD * ((hi - lo) / (dlo * dhi));
    lx = Dx / nD;
    ly = Dy / nD;
  }
  g.ok = g.ok && isfinite((double)L) && L >= (T)1e-6;
  g.lx = g.ok ? lx : (T)1;
  g.ly = g.ok ? ly : (T)0;
  const T hs = L / (T)(NS - 1);
  g.h = g.ok ? (hs > (T)1 ? hs : (T)1) : (T)1;
  g.cx = g.ok ? (plx + phx) / (T)2 : u;
  g.cy = g.ok ? (ply + phy) / (T)2 : v;
  g.use_x = fabs((double)g.lx) >= fabs((double)g.ly);
  g.l0x = (T)0;
  g.l0y = (T)0;
  if (PAT == KF_PAT_LINE5) {
    // keyframe epipolar line through the pixel and the epipole K c1
    const T ex = (T)c.e0[0], ey = (T)c.e0[1], ez = (T)c.e0[2];
    const T ddx = ez * u - ex, ddy = ez * v - ey;
    const T n0 = sqrt(ddx * ddx + ddy * ddy);
    const bool ok0 = n0 > (T)0 && isfinite((double)n0);
    T l0x = ok0 ? ddx / n0 : (T)0, l0y = ok0 ? ddy / n0 : (T)0;
    // orient it so that a step along it moves the projection along +l1
    const T rc = (lo + hi) / (T)2;
    const T q0d = g.A2 + rc * b2;
    const T q0x = (g.A0 + rc * b0) / q0d, q0y = (g.A1 + rc * b1) / q0d;
    const T u1 = u + l0x, v1 = v + l0y;
    const T B0 = H0 * u1 + H1 * v1 + H2 + rc * b0;
    const T B1 = H3 * u1 + H4 * v1 + H5 + rc * b1;
    const T B2 = H6 * u1 + H7 * v1 + H8 + rc * b2;
    const T q1x = B0 / B2, q1y = B1 / B2;
    if ((q1x - q0x) * g.lx + (q1y - q0y) * g.ly < (T)0) {
      l0x = -l0x;
      l0y = -l0y;
    }
    g.ok = g.ok && ok0 && isfinite((double)l0x) && isfinite((double)l0y);
    g.l0x = l0x;
    g.l0y = l0y;
  }
  return g;
}

// Position of sample k in image 1.
template <typename T, int NS>
__device__ inline void sample_xy(const PixelGeom<T>& g, int k, T& px, T& py) {
  const T off = (T)k - (T)((NS - 1) * 0.5);
  px = g.cx + off * g.h * g.lx;
  py = g.cy + off * g.h * g.ly;
}

// Inverse depth at image-1 position (px, py) of the pixel's ray, as the
// quotient num / den of the coordinate the geometry solves from.
template <typename T>
__device__ inline void depth_ratio(const PixelGeom<T>& g, const FrameConst& c, T px, T py, T& num, T& den) {
  const T pm = g.use_x ? px : py;
  const T Am = g.use_x ? g.A0 : g.A1;
  const T bm = g.use_x ? (T)c.b[0] : (T)c.b[1];
  num = pm * g.A2 - Am;
  den = bm - pm * (T)c.b[2];
}

// Position and inverse depth of sample k.
template <typename T, int NS>
__device__ inline void sample_pos(const PixelGeom<T>& g, const FrameConst& c, int k, T& px, T& py, T& rk) {
  sample_xy<T, NS>(g, k, px, py);
  T num, den;
  depth_ratio<T>(g, c, px, py, num, den);
  rk = num / den;
}

// Whether the inverse depth at (px, py) is finite and inside [rho_min,
// rho_max]. FP64 tests the quotient itself; the float forms test the signs of
// the differences from the bounds times the denominator (the same test in
// exact arithmetic, without the division).
template <typename T>
__device__ inline bool depth_in_range(const PixelGeom<T>& g, const FrameConst& c, T px, T py, T rmin, T rmax) {
  T num, den;
  depth_ratio<T>(g, c, px, py, num, den);
  if constexpr (sizeof(T) == 8) {
    const T rk = num / den;
    return isfinite(rk) & (rk >= rmin) & (rk <= rmax);
  } else {
    // rk - rmin and rmax - rk have the signs of (num - rmin den) den and
    // (rmax den - num) den; each fused difference keeps its exact sign
    const T lo = fma(-rmin, den, num) * den, hi = fma(rmax, den, -num) * den;
    return (den != (T)0) & (fmin(lo, hi) >= (T)0);
  }
}

// Photometric residual of pattern point j at sample position (px, py).
template <typename T, int PAT>
__device__ inline T point_residual(const StereoArgs& a, const PixelGeom<T>& g, T px, T py, int j, T pat_j) {
  T tu, tv;
  if (PAT == KF_PAT_LINE5) {
    const T jj = (T)(j - 2);
    tu = px + jj * g.lx;
    tv = py + jj * g.ly;
  } else {
    tu = px + (T)(j % 5 - 2);
    tv = py + (T)(j / 5 - 2);
  }
  return bilin_u8<T>(gp(a.i1s), a.i1_stride, a.W, a.H, tu, tv) - pat_j;
}

// Keyframe pattern value of point j at pixel (u, v), rounded to the patch storage type.
// Textured pixels lie >= 2 px inside the image, so every point is in bounds.
template <typename T, typename TI, int PAT>
__device__ inline T kf_point(const KF_GLOBAL TI* i0, int W, int H, T u, T v, const PixelGeom<T>& g, int j) {
  if constexpr (PAT == KF_PAT_LINE5) {
    const T jj = (T)(j - 2);
    return round_to_img<TI, T>(bilin_kf<T, TI>(i0, W, H, u + jj * g.l0x, v + jj * g.l0y));
  } else {   // a stored element, already in the storage type
    const int iu = (int)u + (j % 5 - 2), iv = (int)v + (j / 5 - 2);
    return img_value(i0[(size_t)iv * W + iu]);
  }
}

template <typename T>
__device__ inline T shfl_xor_t(T v, int m) { return __shfl_xor(v, m, 64); }

// Value of v in lane `src` (wave-uniform) for every lane.
__device__ inline float readlane_t(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double readlane_t(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ inline T shfl_t(T v, int src) { return __shfl(v, src, 64); }

// One textured pixel (entry `idx` of the search list of keyframe `a`) for the
// lane group of this thread. Every lane of the wavefront calls it together
// (cross-lane operations inside); `active` masks groups without an entry.
// Returns true if the group's lane 0 wrote a new filter estimate.
template <typename T, typename TI, int PAT, int NS>
__device__ inline bool stereo_pixel(const StereoArgs& a, int idx, bool active, int lane) {
  constexpr int G = lanes_per_pixel(PAT, NS);
  constexpr int S = NS / G;                // samples per lane
  constexpr int P = PAT == KF_PAT_LINE5 ? 5 : 25;
  constexpr T INF = (T)INFINITY;
  const int grp = lane / G;
  const int gl = lane % G;
  const KF_GLOBAL TI* i0 = gp(static_cast<const TI*>(a.i0));
  const KF_GLOBAL T* rho_s = gp(static_cast<const T*>(a.rho));
  const KF_GLOBAL T* var_s = gp(static_cast<const T*>(a.var));
  KF_GLOBAL T* rho_o = gp(static_cast<T*>(a.rho_out));
  KF_GLOBAL T* var_o = gp(static_cast<T*>(a.var_out));
  const int W = a.W, H = a.H;
  const int st = a.i1_stride;
  bool updated = false;
  const int pix = active ? gp(a.list)[idx] : 0;
  const T u = (T)(pix % W), v = (T)(pix / W);
  const T rho0 = rho_s[pix], var0 = var_s[pix];
  const bool has = var0 > (T)0;
  PixelGeom<T> g = pixel_geometry<T, PAT, NS>(a, u, v, rho0, var0, has);
  g.ok = g.ok && active;

  // keyframe pattern I0(a_j) (in the form's patch storage type): with at least
  // P lanes per pixel, lane j evaluates point j and every lane receives all P
  // values by a cross-lane broadcast (a scalar readlane when one pixel fills
  // the wavefront); with fewer lanes every lane evaluates all points.
  T mine = (T)0;
  T pat[P];
  if (G >= P) {
    if (gl < P && active) mine = kf_point<T, TI, PAT>(i0, W, H, u, v, g, gl);
#pragma unroll
    for (int j = 0; j < P; ++j) pat[j] = (G == 64) ? readlane_t(mine, j) : shfl_t(mine, grp * G + j);
  } else {
    // no branch around the loads, so that all P are in flight together: a
    // group without a pixel reads the pattern at (2, 2) (in bounds, unused)
    const T uu = active ? u : (T)2, vv = active ? v : (T)2;
    if constexpr (PAT == KF_PAT_SQ5X5 && std::is_same<TI, bf16>::value) {
#pragma unroll
      for (int r = 0; r < 5; ++r) row5_bf16(i0, (size_t)((int)vv + r - 2) * W + ((int)uu - 2), &pat[5 * r]);
    } else {
#pragma unroll
      for (int j = 0; j < P; ++j) pat[j] = kf_point<T, TI, PAT>(i0, W, H, uu, vv, g, j);
    }
  }

  // SSD of this lane's samples. LINE5 lanes take S consecutive samples
  // (k = gl S + s): with a 1-px step, point j + 1 of sample k is point j of
  // sample k + 1, so the lane evaluates S + 4 bilinear points instead of 5 S.
  // SQ5X5 lanes take every G-th sample.
  constexpr bool CONSEC = PAT == KF_PAT_LINE5;
  const T rho_lo = (T)a.fc.rho_min, rho_hi = (T)a.fc.rho_max;
  T ssd[S];
  T best = INF;
  int bestk = 0x7fffffff;
  const bool shared_pts = CONSEC && g.ok && g.h == (T)1;
  T bv[S + 4];
  bool bin[S + 4];
  if (CONSEC) {
    T qx, qy, qr;
    sample_pos<T, NS>(g, a.fc, gl * S, qx, qy, qr);
#pragma unroll
    for (int t = 0; t < S + 4; ++t) {
      const T tu = qx + (T)(t - 2) * g.lx, tv = qy + (T)(t - 2) * g.ly;
      bin[t] = shared_pts && inside<T>(tu, tv, W, H);
      bv[t] = bin[t] ? bilin_u8<T>(gp(a.i1s), st, W, H, tu, tv) : (T)0;
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int k = CONSEC ? gl * S + s : gl + G * s;
    T px, py;
    sample_xy<T, NS>(g, k, px, py);
    bool ok = g.ok & depth_in_range<T>(g, a.fc, px, py, rho_lo, rho_hi);
    T acc = (T)0;
    if (PAT == KF_PAT_LINE5 && shared_pts) {
#pragma unroll
      for (int j = 0; j < 5; ++j) ok = ok && bin[s + j];
      if (ok) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const T e = bv[s + j] - pat[j];
          acc += e * e;
        }
      }
    } else if (PAT == KF_PAT_LINE5) {
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const T jj = (T)(j - 2);
        ok = ok && inside<T>(px + jj * g.lx, py + jj * g.ly, W, H);
      }
      if (ok) {
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const T e = point_residual<T, PAT>(a, g, px, py, j, pat[j]);
          acc += e * e;
        }
      }
    } else {
      ok = ok && px - (T)2 >= (T)0 && px + (T)2 <= (T)(W - 1) && py - (T)2 >= (T)0 &&
           py + (T)2 <= (T)(H - 1);
      if (ok) {
        // 6 x 6 tap window shared by the 25 points (translation-only warp)
        const T fpx = floor(px), fpy = floor(py);
        const T f = px - fpx, gg = py - fpy;
        const T fm = (T)1 - f, gm = (T)1 - gg;
        const int c0 = (int)fpx - 2, r0 = (int)fpy - 2;
        T hprev[5];
        const KF_GLOBAL uint8_t* base = gp(a.i1s) + (size_t)r0 * st + c0;
#pragma unroll
        for (int n = 0; n < 6; ++n) {
          // rows and the 6th column may reach one pad row / byte (weight 0 there)
          T t[6];
          taps6<T>(base + (size_t)n * st, t);
          T hrow[5];
          // FP64 interpolates as a + w (b - a), like the oracle; the float
          // forms weight both ends, (1 - w) a + w b, which takes one
          // instruction less per point (the tap difference would be an
          // integer subtraction and a conversion) and rounds differently
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            if constexpr (sizeof(T) == 8) hrow[m] = t[m] + f * (t[m + 1] - t[m]);
            else hrow[m] = fma(f, t[m + 1], fm * t[m]);
          }
          if (n > 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) {
              T e;
              if constexpr (sizeof(T) == 8) e = hprev[m] + gg * (hrow[m] - hprev[m]) - pat[(n - 1) * 5 + m];
              else e = fma(gg, hrow[m], fma(gm, hprev[m], -pat[(n - 1) * 5 + m]));
              acc += e * e;
            }
          }
#pragma unroll
          for (int m = 0; m < 5; ++m) hprev[m] = hrow[m];
        }
      }
    }
    ssd[s] = ok ? acc : INF;
    if (ssd[s] < best) {          // s increases with k: keeps the first minimum
      best = ssd[s];
      bestk = k;
    }
  }
  // argmin across the group: smaller SSD, ties -> smaller k
#pragma unroll
  for (int m = 1; m < G; m <<= 1) {
    const T ob = shfl_xor_t(best, m);
    const int ok_ = __shfl_xor(bestk, m, 64);
    if (ob < best || (ob == best && ok_ < bestk)) {
      best = ob;
      bestk = ok_;
    }
  }
  const bool any_valid = g.ok && best < INF;
  const int kstar = bestk;
  // SSD of the two neighbours k* - 1 and k* + 1
  T s_m = INF, s_p = INF;
  {
    const int km = any_valid ? kstar - 1 : -1;
    const int kp = any_valid ? kstar + 1 : NS;
    const int base = grp * G;
    T vm = INF, vp = INF;
    // every lane reads its own slot value for the owner's sample index
    const int slot_m = km >= 0 ? (CONSEC ? km % S : km / G) : 0;
    const int slot_p = kp < NS ? (CONSEC ? kp % S : kp / G) : 0;
    T mine_m = ssd[0], mine_p = ssd[0];
#pragma unroll
    for (int s = 1; s < S; ++s) {
      if (slot_m == s) mine_m = ssd[s];
      if (slot_p == s) mine_p = ssd[s];
    }
    vm = shfl_t(mine_m, base + (km >= 0 ? (CONSEC ? km / S : km % G) : 0));
    vp = shfl_t(mine_p, base + (kp < NS ? (CONSEC ? kp / S : kp % G) : 0));
    s_m = km >= 0 ? vm : INF;
    s_p = kp < NS ? vp : INF;
  }
  const bool has_nb = any_valid && (s_m < INF || s_p < INF);
  const int nstar = (s_m <= s_p) ? kstar - 1 : kstar + 1;

  // residual vectors at k* and n*: lane j of the group computes point j
  T pxk = 0, pyk = 0, rk_k = 0, pxn = 0, pyn = 0, rk_n = 0;
  if (has_nb) {
    sample_pos<T, NS>(g, a.fc, kstar, pxk, pyk, rk_k);
    sample_pos<T, NS>(g, a.fc, nstar, pxn, pyn, rk_n);
  }
  T sum_kd = 0, sum_dd = 0;
  if (has_nb) {
    for (int j = gl; j < P; j += G) {
      const T pj = G >= P ? mine : kf_point<T, TI, PAT>(i0, W, H, u, v, g, j);
      const T ek = point_residual<T, PAT>(a, g, pxk, pyk, j, pj);
      const T en = point_residual<T, PAT>(a, g, pxn, pyn, j, pj);
      const T de = en - ek;
      sum_kd += ek * de;
      sum_dd += de * de;
    }
  }
#pragma unroll
  for (int m = 1; m < G; m <<= 1) {
    sum_kd += shfl_xor_t(sum_kd, m);
    sum_dd += shfl_xor_t(sum_dd, m);
  }
  if (gl == 0 && active) {
    gp(a.match)[pix] = (g.ok && best < INF) ? kstar : -1;
    if (has_nb && sum_dd > (T)0) {
      T lam = -sum_kd / sum_dd;
      lam = lam < (T)0 ? (T)0 : (lam > (T)1 ? (T)1 : lam);
      const T d_a = (T)1 / rk_k, d_b = (T)1 / rk_n;
      const T dd = d_b - d_a;
      const T dstar = d_a + lam * dd;
      const T sp = (T)a.fc.sigma_photo;
      const T var_d = sp * sp * dd * dd / sum_dd;       // eq. (semi) with J = de / dd
      const T ro = (T)1 / dstar;
      const T d2 = dstar * dstar;
      const T vo = var_d / (d2 * d2);
      if (isfinite((double)var_d) && var_d > (T)0 && isfinite((double)dstar) && dstar > (T)0 &&
          isfinite((double)vo) && vo > (T)0) {
        if (has) {   // Gaussian product with the current estimate
          rho_o[pix] = (vo * rho0 + var0 * ro) / (var0 + vo);
          var_o[pix] = var0 * vo / (var0 + vo);
        } else {
          rho_o[pix] = ro;
          var_o[pix] = vo;
        }
        updated = true;
      }
    }
    if (!updated && a.rho_out != a.rho) {   // double-buffered state: carry the estimate over
      rho_o[pix] = rho0;
      var_o[pix] = var0;
    }
  }
  return updated;
}

template <typename T, typename TI, int PAT, int NS>
__global__ __launch_bounds__(ST_THREADS) void k_stereo(StereoArgs a) {
  constexpr int G = lanes_per_pixel(PAT, NS);
  constexpr int GPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane / G;
  const int count = gp(a.scal_ro)->mask_count;
  const int groups_per_block = ST_WAVES * GPW;
  const int ngroups = gridDim.x * groups_per_block;
  const int wave_first = blockIdx.x * groups_per_block + wave * GPW;
  const int my_group = wave_first + grp;
  // rounds with at least one pixel for this wavefront (wave-uniform)
  const int rounds = count > wave_first ? (count - wave_first + ngroups - 1) / ngroups : 0;
  int updated_here = 0;
  for (int r = 0; r < rounds; ++r) {      // wave-uniform trip count (cross-lane operations inside)
    const int idx = my_group + r * ngroups;
    const bool active = idx < count;
    if (stereo_pixel<T, TI, PAT, NS>(a, active ? idx : 0, active, lane)) ++updated_here;
  }
  // one atomic per wavefront
  for (int m = 32; m > 0; m >>= 1) updated_here += __shfl_xor(updated_here, m, 64);
  if (lane == 0 && updated_here) atomicAdd(&gp(a.scal)->n_updated[a.buf], updated_here);
}

// Prefix sums of n per-keyframe counts in LDS (pref[0] = 0, pref[n] = total).
template <typename F>
__device__ inline void block_prefix(int n, F count, int* pref) {
  if (threadIdx.x == 0) {
    int acc = 0;
    pref[0] = 0;
    for (int c = 0; c < n; ++c) {
      acc += count(c);
      pref[c + 1] = acc;
    }
  }
  __syncthreads();
}

// Keyframe c with pref[c] <= item < pref[c + 1].
__device__ inline int find_keyframe(const int* pref, int n, int item) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pref[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Batched form: the textured pixels of n keyframes form one item space of
// wavefront-sized slots (each keyframe's list padded to whole wavefronts), so
// a wavefront always works on one keyframe and reads its arguments as
// wave-uniform (scalar) values.
template <typename T, typename TI, int PAT, int NS>
__global__ __launch_bounds__(ST_THREADS) void k_stereo_batch(const StereoArgs* __restrict__ tab,
                                                             const int32_t* __restrict__ n_dev) {
  constexpr int G = lanes_per_pixel(PAT, NS);
  constexpr int GPW = 64 / G;
  __shared__ int pref[KF_BATCH_MAX + 1];
  __shared__ int upd[KF_BATCH_MAX];
  const int n = *n_dev;
  for (int c = threadIdx.x; c < n; c += blockDim.x) upd[c] = 0;
  block_prefix(n, [&](int c) { return (gp(tab[c].scal_ro)->mask_count + GPW - 1) / GPW; }, pref);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane / G;
  const int total = pref[n];
  const int nwaves = gridDim.x * ST_WAVES;
  const int my_wave = blockIdx.x * ST_WAVES + wave;
  const int rounds = total > my_wave ? (total - my_wave + nwaves - 1) / nwaves : 0;
  for (int r = 0; r < rounds; ++r) {
    const int witem = my_wave + r * nwaves;
    const bool wactive = witem < total;
    const int c = __builtin_amdgcn_readfirstlane(wactive ? find_keyframe(pref, n, witem) : 0);
    const StereoArgs a = tab[c];
    const int idx = (witem - pref[c]) * GPW + grp;
    const bool active = wactive && idx < gp(a.scal_ro)->mask_count;
    if (stereo_pixel<T, TI, PAT, NS>(a, active ? idx : 0, active, lane)) atomicAdd(&upd[c], 1);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    if (upd[c]) atomicAdd(&gp(tab[c].scal)->n_updated[tab[c].buf], upd[c]);
}

// Copies the caller's frame into rows of `st` bytes, zero padded, plus one zero row.
// Per-frame counters of filter-state buffer `buf`: the update counter starts at
// zero and the frame's camera-centre distance from the keyframe is recorded
// (keyframe rule). A launch of its own: written from inside the staging kernel,
// these stores cost the next frame's stereo ~10 % of its overlap with a running
// solve (measured, frame pipelining at 640 x 480).
__global__ void k_frame_begin(DevScalars* scal, int buf, double trans) {
  scal->n_updated[buf] = 0;
  scal->frame_trans[buf] = trans;
}

// Stages the new frame with padded rows.
__global__ void k_stage_frame(const uint8_t* src, uint8_t* dst, int W, int H, int st) {
  const int total = (H + 1) * st;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int r = i / st, c = i - r * st;
    dst[i] = (r < H && c < W) ? src[(size_t)r * W + c] : (uint8_t)0;
  }
}

// Batched staging: row y of the grid stages active keyframe y's frame (as
// k_stage_frame does) and resets its update counter.
__global__ void k_stage_batch(const StereoArgs* __restrict__ tab, const int32_t* __restrict__ n_dev) {
  if ((int)blockIdx.y >= *n_dev) return;
  const StereoArgs& a = tab[blockIdx.y];
  const int st = a.i1_stride, W = a.W, H = a.H;
  const int total = (H + 1) * st;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int r = i / st, col = i - r * st;
    gp(a.i1s)[i] = (r < H && col < W) ? gp(a.i1)[(size_t)r * W + col] : (uint8_t)0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    gp(a.scal)->n_updated[a.buf] = 0;
    gp(a.scal)->frame_trans[a.buf] = a.fc.trans;
  }
}

// Workgroups of kernel `k` one compute unit holds at once (its registers and
// LDS decide), queried once per instantiation; 8 if the query fails.
template <typename K>
int resident_per_cu(K k) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, ST_THREADS, 0) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    n = 8;
  }
  return n;
}

// Grid of a stereo launch: beside a running solve (frame pipelining) one
// workgroup per compute unit, else as many as the device holds at once. The
// stereo is bound by instruction issue and memory latency, so a single
// generation of workgroups that stride over the pixel list until it is done
// beats a grid of several generations, whose last one leaves most SIMDs
// idle: 640 x 480, SQ5X5, N_s = 128 (3 resident workgroups per compute unit)
// takes 103 us per frame against 115 us with 6 per unit and 136 us with 8.
// Beside a solve, whose team waits on its slowest workgroup and so on every
// SIMD the stereo's waves share, one per unit keeps the stereo hidden and
// the solve undisturbed (640 x 480 pipelined, 8 / 4 / 2 / 1 / 0.5 per unit:
// 452 / 464 / 470 / 472 / 465 Mpixel/s; at 0.25 the stereo outlasts the solve).
template <auto K>
int stereo_grid(int cus, bool beside_solve) {
  static const int per_cu = resident_per_cu(K);   // one query per kernel instantiation
  return beside_solve ? cus : cus * per_cu;
}

template <typename T, typename TI, int PAT>
hipError_t stereo_batch_ns(int ns, const StereoArgs* tab, const int32_t* n, int cus, hipStream_t s) {
  switch (ns) {
#define KF_NS(v)                                                                                        \
  case v: {                                                                                             \
    constexpr auto k = k_stereo_batch<T, TI, PAT, v>;                                                   \
    hipLaunchKernelGGL(k, dim3(stereo_grid<k>(cus, false)), dim3(ST_THREADS), 0, s, tab, n);            \
    break;                                                                                              \
  }
    KF_NS(4) KF_NS(8) KF_NS(16) KF_NS(32) KF_NS(64) KF_NS(128) KF_NS(256) KF_NS(512) KF_NS(1024)
#undef KF_NS
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t stereo_batch_prec(int pattern, int ns, const StereoArgs* tab, const int32_t* n, int cus, hipStream_t s) {
  using T = typename Form<PREC>::T;
  using TI = typename Form<PREC>::TI;
  if (pattern == KF_PAT_LINE5) return stereo_batch_ns<T, TI, KF_PAT_LINE5>(ns, tab, n, cus, s);
  return stereo_batch_ns<T, TI, KF_PAT_SQ5X5>(ns, tab, n, cus, s);
}

template <typename T, typename TI, int PAT>
hipError_t stereo_ns(int ns, const StereoArgs& a, int cus, bool beside_solve, hipStream_t s) {
  switch (ns) {
#define KF_NS(v)                                                                                        \
  case v: {                                                                                             \
    constexpr auto k = k_stereo<T, TI, PAT, v>;                                                         \
    hipLaunchKernelGGL(k, dim3(stereo_grid<k>(cus, beside_solve)), dim3(ST_THREADS), 0, s, a);          \
    break;                                                                                              \
  }
    KF_NS(4) KF_NS(8) KF_NS(16) KF_NS(32) KF_NS(64) KF_NS(128) KF_NS(256) KF_NS(512) KF_NS(1024)
#undef KF_NS
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t stereo_prec(int pattern, int ns, const StereoArgs& a, int cus, bool beside_solve, hipStream_t s) {
  using T = typename Form<PREC>::T;
  using TI = typename Form<PREC>::TI;
  if (pattern == KF_PAT_LINE5) return stereo_ns<T, TI, KF_PAT_LINE5>(ns, a, cus, beside_solve, s);
  return stereo_ns<T, TI, KF_PAT_SQ5X5>(ns, a, cus, beside_solve, s);
}

}  // namespace

int device_cus(int device) {
  int cus = 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  return cus;
}

hipError_t launch_stereo_batch(int prec, int pattern, int ns, const StereoArgs* tab, const int32_t* n, int nmax,
                               int cus, hipStream_t s) {
  hipLaunchKernelGGL(k_stage_batch, dim3(64, nmax), dim3(256), 0, s, tab, n);
  switch (prec) {
    case KF_F64: return stereo_batch_prec<KF_F64>(pattern, ns, tab, n, cus, s);
    case KF_F32: return stereo_batch_prec<KF_F32>(pattern, ns, tab, n, cus, s);
    case KF_BF16_F32: return stereo_batch_prec<KF_BF16_F32>(pattern, ns, tab, n, cus, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stereo(int prec, int pattern, int ns, const StereoArgs& a, int cus, bool beside_solve,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_frame_begin, dim3(1), dim3(1), 0, s, a.scal, a.buf, a.fc.trans);
  {
    const int total = (a.H + 1) * a.i1_stride;
    int nb = (total + 255) / 256;
    nb = nb < 2048 ? nb : 2048;
    hipLaunchKernelGGL(k_stage_frame, dim3(nb), dim3(256), 0, s, a.i1, a.i1s, a.W, a.H, a.i1_stride);
  }
  switch (prec) {
    case KF_F64: return stereo_prec<KF_F64>(pattern, ns, a, cus, beside_solve, s);
    case KF_F32: return stereo_prec<KF_F32>(pattern, ns, a, cus, beside_solve, s);
    case KF_BF16_F32: return stereo_prec<KF_BF16_F32>(pattern, ns, a, cus, beside_solve, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace kf
