// fd_device.hpp -- device helpers shared by the gfx950 kernels of libfusedir.
//
// Camera records are 16 floats: fx, fy, cx, cy, R[9] (row-major), t[3].
// Maps are V x H x W of float or binary16.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fd {

constexpr int kWave = 64;

// Texel (x, y) of one map as float; outside the image reads 0 (zero
// border).  The load itself is unconditional (at a clamped address), so a
// run of them can be issued back to back.
template <typename T>
__device__ __forceinline__ float tex_load_nb(const T* __restrict__ m, int W, int H, int x,
                                             int y) {
  const bool in = (unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H;
  const int xc = min(max(x, 0), W - 1), yc = min(max(y, 0), H - 1);
  float v;
  if constexpr (sizeof(T) == 2)
    v = __half2float(((const __half*)m)[(size_t)yc * W + xc]);
  else
    v = ((const float*)m)[(size_t)yc * W + xc];
  return in ? v : 0.0f;
}

// binary64 reciprocal and reciprocal square root of finite positive x:
// the hardware estimate refined by two Newton steps (error within an ulp or
// two of the rounded result; the search compares such values only against
// each other, never bit for bit with another implementation).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = __builtin_fma(-h * y, y, 0.5);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-h * y, y, 0.5);
  return __builtin_fma(y, e, y);
}

// Projection, eligibility and the Eq. (4) ranking score, in binary64.
// The calibrated pinhole model of Sec. 3.1: X_c = R p + t, pixel
// u = (f_x X/Z + c_x, f_y Y/Z + c_y).  Every discrete choice of the view
// selection (in front, inside the image, visible, centre confidence above
// zero, the ranking) is taken on binary64 values computed from the binary32
// and binary16 inputs (which convert exactly), so each choice is the exact
// mathematical one up to binary64 rounding.  project64 evaluates, one
// rounding per operation in the order written (the library is built without
// floating-point contraction; binary64 division is IEEE):
//   X = ((R0 px + R1 py) + R2 pz) + t0   (likewise Y, Z)
//   front: Z > z_near;  u = fx (X / Z) + cx,  v = fy (Y / Z) + cy
//   inside: 0 <= u <= W-1 and 0 <= v <= H-1
// The projection u is also the centre of the fusion patch (Sec. 3.1.3).
struct Proj {
  double X, Y, Z, u, v;
};

__device__ __forceinline__ bool project64(const float* __restrict__ cam, double px, double py,
                                          double pz, int W, int H, double z_near, Proj& o) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  o.X = (double)R[0] * px + (double)R[1] * py + (double)R[2] * pz + (double)t[0];
  o.Y = (double)R[3] * px + (double)R[4] * py + (double)R[5] * pz + (double)t[1];
  o.Z = (double)R[6] * px + (double)R[7] * py + (double)R[8] * pz + (double)t[2];
  if (!(o.Z > z_near)) return false;
  o.u = (double)cam[0] * (o.X / o.Z) + (double)cam[2];
  o.v = (double)cam[1] * (o.Y / o.Z) + (double)cam[3];
  return o.u >= 0.0 && o.u <= (double)(W - 1) && o.v >= 0.0 && o.v <= (double)(H - 1);
}

// The same projection from the per-call binary64 camera table (kCam64
// values per view: u = row0 . (p, 1) / Z, v = row1 . (p, 1) / Z with
// Z = row2 . (p, 1)), for the loops over every view of a point: nine fma
// and one reciprocal instead of the camera's own rows and two divisions.
// It agrees with project64 up to binary64 rounding (a few ulp of u).
struct ProjT {
  double Z, u, v;
};

__device__ __forceinline__ bool project_tab(const double* __restrict__ c, double px, double py,
                                            double pz, int W, int H, double z_near, ProjT& o) {
  o.Z = __builtin_fma(c[8], px, __builtin_fma(c[9], py, __builtin_fma(c[10], pz, c[11])));
  const double nu = __builtin_fma(c[0], px, __builtin_fma(c[1], py, __builtin_fma(c[2], pz, c[3])));
  const double nv = __builtin_fma(c[4], px, __builtin_fma(c[5], py, __builtin_fma(c[6], pz, c[7])));
  const bool front = o.Z > z_near;
  const double iz = rcp64(front ? o.Z : 1.0);
  o.u = nu * iz;
  o.v = nv * iz;
  return front && o.u >= 0.0 && o.u <= (double)(W - 1) && o.v >= 0.0 && o.v <= (double)(H - 1);
}

// Texel at a 32-bit offset from a view's base pointer (the base is the same
// for the whole wave, so the load takes a scalar base and a vector offset).
template <typename T>
__device__ __forceinline__ float ld_texel(const T* __restrict__ base, uint32_t off) {
  // a 32-bit byte offset (a plane holds at most 2^30 texels, so it cannot
  // wrap) lets the load use the scalar-base addressing form
  const char* b = (const char*)base + (uint32_t)(off * (uint32_t)sizeof(T));
  if constexpr (sizeof(T) == 2)
    return __half2float(*(const __half*)b);
  else
    return *(const float*)b;
}

// Visibility of Sec. 3.1.1 (the score V_i^v): the camera-space depth of the
// point agrees with the rendered depth at the nearest texel of its
// projection, (floor(u + 1/2), floor(v + 1/2)), within tau (binary64).
// No depth maps: every eligible view is visible.  A +inf (background) or
// NaN depth never is.  `ok` (the view is eligible) guards the texel read:
// an eligible projection lies inside the image.
template <typename T, typename PR>
__device__ __forceinline__ bool visible_at(const T* __restrict__ db, int W, bool ok,
                                           const PR& pr, double tau) {
  if (db == nullptr) return ok;
  const double u = ok ? pr.u : 0.0, v = ok ? pr.v : 0.0;
  const uint32_t xn = (uint32_t)floor(u + 0.5), yn = (uint32_t)floor(v + 0.5);
  const double D = (double)ld_texel<T>(db, yn * (uint32_t)W + xn);
  return ok && fabs(pr.Z - D) <= tau;
}

// Bilinear centre confidence of an eligible projection (Eq. 4's ranking
// score), split so that a caller can skip the texels of a view no lane of
// its wave sees:
//   x0 = floor(u), fx = u - x0 (likewise y)
//   C = (1-fx)(1-fy) C00 + fx (1-fy) C10 + (1-fx) fy C01 + fx fy C11
// with texels outside the image read as 0; an eligible projection lies
// inside the image, so only the +1 neighbours need that check.
struct ConfTexels {
  float c00, c10, c01, c11;
  double fx, fy;
  bool xin, yin;
};

// The two binary16 texels (x, x + 1) of a row, from one 8-byte load of the
// aligned texel pair that holds x and the next pair: `row` is the row's
// offset in texels, x & ~1 <= W - 4, W even and the map 4-byte aligned (so
// the load stays in the row and is dword aligned).
__device__ __forceinline__ void ld_pair_h(const void* __restrict__ base, uint32_t row,
                                          uint32_t x, float& lo, float& hi) {
  const uint32_t a = x & ~1u;
  const uint2 w = *(const uint2*)((const char*)base + (uint32_t)((row + a) * 2u));
  const uint32_t p = __builtin_amdgcn_alignbit(w.y, w.x, (x & 1u) * 16u);
  lo = __half2float(__ushort_as_half((unsigned short)(p & 0xffffu)));
  hi = __half2float(__ushort_as_half((unsigned short)(p >> 16)));
}

// pair loads apply: the scene allows them (binary16, even width, 4-byte
// aligned maps) and the pair at x & ~1 and the next one lie inside the row
template <typename T>
__device__ __forceinline__ bool pair_ok(bool pairs, int W, uint32_t x) {
  return sizeof(T) == 2 && pairs && (x & ~1u) + 3u < (uint32_t)W;
}

template <typename T, typename PR>
__device__ __forceinline__ ConfTexels conf_texels(const T* __restrict__ cb, int W, int H,
                                                     bool ok, const PR& pr, bool pairs) {
  ConfTexels t;
  const double u = ok ? pr.u : 0.0, v = ok ? pr.v : 0.0;
  const double x0 = floor(u), y0 = floor(v);
  t.fx = u - x0;
  t.fy = v - y0;
  const uint32_t ix = (uint32_t)x0, iy = (uint32_t)y0;
  const uint32_t o00 = iy * (uint32_t)W + ix;
  t.xin = ix + 1u < (uint32_t)W;
  t.yin = iy + 1u < (uint32_t)H;
  const uint32_t dx = t.xin ? 1u : 0u, dy = t.yin ? (uint32_t)W : 0u;
  if (pair_ok<T>(pairs, W, ix)) {  // x + 1 is inside the row here
    ld_pair_h(cb, iy * (uint32_t)W, ix, t.c00, t.c10);
    ld_pair_h(cb, iy * (uint32_t)W + dy, ix, t.c01, t.c11);
  } else {
    t.c00 = ld_texel<T>(cb, o00);
    t.c10 = ld_texel<T>(cb, o00 + dx);
    t.c01 = ld_texel<T>(cb, o00 + dy);
    t.c11 = ld_texel<T>(cb, o00 + dx + dy);
  }
  return t;
}

__device__ __forceinline__ double conf_combine(const ConfTexels& t) {
  const double c10 = t.xin ? (double)t.c10 : 0.0;
  const double c01 = t.yin ? (double)t.c01 : 0.0;
  const double c11 = (t.xin && t.yin) ? (double)t.c11 : 0.0;
  return (1.0 - t.fx) * (1.0 - t.fy) * (double)t.c00 + t.fx * (1.0 - t.fy) * c10 +
         (1.0 - t.fx) * t.fy * c01 + t.fx * t.fy * c11;
}

// sin x and cos x in binary32 for |x| <= 1024 (the doubled angle of a map
// texel): Cody-Waite reduction by pi/2 with the constant split in three
// parts (each step one fma), then the minimax polynomials on [-pi/4, pi/4]
// of Moshier's Cephes library (sinf, cosf).  Error within 1.5 ulp of 1
// (checked over every binary16 angle in [0, pi] and 2e5 random binary32
// angles against binary64 sin/cos).
__device__ __forceinline__ void sincos_reduced(float x, float* s, float* c) {
  const float k = rintf(x * 0.636619772367581343f);
  float r = __builtin_fmaf(-k, 1.5703125f, x);
  r = __builtin_fmaf(-k, 4.838267923332751e-4f, r);
  r = __builtin_fmaf(-k, 2.5632829192545614e-12f, r);
  const float r2 = r * r;
  const float ps = __builtin_fmaf(__builtin_fmaf(-1.9515295891e-4f, r2, 8.3321608736e-3f), r2,
                                  -1.6666654611e-1f);
  const float pc = __builtin_fmaf(__builtin_fmaf(2.443315711809948e-5f, r2, -1.388731625493765e-3f),
                                  r2, 4.166664568298827e-2f);
  const float sp = __builtin_fmaf(r * r2, ps, r);
  const float cp = __builtin_fmaf(r2 * r2, pc, __builtin_fmaf(-0.5f, r2, 1.0f));
  const int q = (int)k & 3;
  const float sv = (q & 1) ? cp : sp, cv = (q & 1) ? sp : cp;
  *s = (q & 2) ? -sv : sv;
  *c = ((q + 1) & 2) ? -cv : cv;
}

// Logical block index such that the blocks of one XCD cover a contiguous
// range of tiles:
// the dispatcher deals workgroups to the 8 XCDs round-robin, so remap
// blockIdx so that neighbouring (spatially sorted) tiles share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t nblocks) {
  const int64_t b = blockIdx.x;
  const int64_t per = nblocks / 8, rem = nblocks % 8;
  const int64_t xcd = b % 8, k = b / 8;
  // XCD x owns logical blocks [start(x), start(x) + per + (x < rem))
  const int64_t start = xcd * per + (xcd < rem ? xcd : rem);
  return start + k;
}

// The index of this thread's wave within the grid, in XCD-aware block order,
// read from lane 0 so that the compiler keeps it (and whatever is indexed by
// it) in scalar registers: it is the same on every lane of the wave.
__device__ __forceinline__ int64_t wave_tile(int64_t nblocks) {
  const int64_t t = xcd_tile(nblocks) * (blockDim.x / kWave) + (threadIdx.x / kWave);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)t >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lanes of a wave are split into groups of `k` consecutive lanes; returns the
// sum of v over the caller's group, added in lane order (slot 0 first) so
// every lane of the group gets the same bits.
template <typename V>
__device__ __forceinline__ V group_sum(V v, int group_base, int k) {
  V s = __shfl(v, group_base, kWave);
  for (int j = 1; j < k; ++j) s += __shfl(v, group_base + j, kWave);
  return s;
}

// group_sum with the group size known at compile time (KT > 0): the K
// shuffles are issued back to back and waited for once.
template <int KT, typename V>
__device__ __forceinline__ V group_sum_t(V v, int group_base, int k) {
  if constexpr (KT > 0) {
    V x[KT];
#pragma unroll
    for (int j = 0; j < KT; ++j) x[j] = __shfl(v, group_base + j, kWave);
    V s = x[0];
#pragma unroll
    for (int j = 1; j < KT; ++j) s += x[j];
    return s;
  } else {
    return group_sum<V>(v, group_base, k);
  }
}

}  // namespace fd
