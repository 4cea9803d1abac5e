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

// Projection and eligibility, in binary32 with the fixed operation order
// every implementation of the method shares (view selection is a discrete
// decision and must come out the same everywhere):
//   X = fma(R0, px, fma(R1, py, fma(R2, pz, t0)))  (likewise Y, Z)
//   front: Z > z_near;  iz = 1 / Z,  u = fma(fx, X * iz, cx), v = fma(fy, Y * iz, cy)
//   inside: 0 <= u <= W-1 and 0 <= v <= H-1
// The reciprocal is IEEE (the library is built without fast-math).
struct Proj {
  float X, Y, Z, u, v;
};

__device__ __forceinline__ bool project32(const float* __restrict__ cam,
                                          float px, float py, float pz, int W,
                                          int H, float z_near, Proj& o) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  o.X = __builtin_fmaf(R[0], px, __builtin_fmaf(R[1], py, __builtin_fmaf(R[2], pz, t[0])));
  o.Y = __builtin_fmaf(R[3], px, __builtin_fmaf(R[4], py, __builtin_fmaf(R[5], pz, t[1])));
  o.Z = __builtin_fmaf(R[6], px, __builtin_fmaf(R[7], py, __builtin_fmaf(R[8], pz, t[2])));
  if (!(o.Z > z_near)) return false;
  const float iz = 1.0f / o.Z;
  o.u = __builtin_fmaf(cam[0], o.X * iz, cam[2]);
  o.v = __builtin_fmaf(cam[1], o.Y * iz, cam[3]);
  return o.u >= 0.0f && o.u <= (float)(W - 1) && o.v >= 0.0f &&
         o.v <= (float)(H - 1);
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

// View eligibility and centre confidence for Eq. (4), split so that a caller
// can skip the confidence loads of a view no lane of its wave sees.
// visible_at: eligible (ok) and, with depth maps, visible (the rule of
// visible32, nearest texel of the projection).  conf_texels + conf_combine:
// the bilinear confidence of an eligible projection in the fixed order
//   x0 = floor(u), fx = u - x0, gx = 1 - fx (likewise y)
//   w00 = gx*gy, w10 = fx*gy, w01 = gx*fy, w11 = fx*fy
//   C = fma(w11, C11, fma(w01, C01, fma(w10, C10, w00*C00)))
// with texels outside the image read as 0; an eligible projection lies inside
// the image, so only the +1 neighbours need that check.  Texels are read at
// 32-bit offsets from the view's base pointer.
template <typename T>
__device__ __forceinline__ bool visible_at(const T* __restrict__ db, int W, bool ok,
                                           const Proj& pr, float tau) {
  if (db == nullptr) return ok;
  const float u = ok ? pr.u : 0.0f, v = ok ? pr.v : 0.0f;
  const uint32_t xn = (uint32_t)floorf(u + 0.5f), yn = (uint32_t)floorf(v + 0.5f);
  const float D = ld_texel<T>(db, yn * (uint32_t)W + xn);
  return ok && fabsf(pr.Z - D) <= tau;
}

struct ConfTexels {
  float c00, c10, c01, c11, fx, fy;
  bool xin, yin;
};

template <typename T>
__device__ __forceinline__ ConfTexels conf_texels(const T* __restrict__ cb, int W, int H,
                                                     bool ok, const Proj& pr) {
  ConfTexels t;
  const float u = ok ? pr.u : 0.0f, v = ok ? pr.v : 0.0f;
  const float x0 = floorf(u), y0 = floorf(v);
  t.fx = u - x0;
  t.fy = v - y0;
  const uint32_t ix = (uint32_t)x0, iy = (uint32_t)y0;
  const uint32_t o00 = iy * (uint32_t)W + ix;
  t.xin = ix + 1u < (uint32_t)W;
  t.yin = iy + 1u < (uint32_t)H;
  const uint32_t dx = t.xin ? 1u : 0u, dy = t.yin ? (uint32_t)W : 0u;
  t.c00 = ld_texel<T>(cb, o00);
  t.c10 = ld_texel<T>(cb, o00 + dx);
  t.c01 = ld_texel<T>(cb, o00 + dy);
  t.c11 = ld_texel<T>(cb, o00 + dx + dy);
  return t;
}

__device__ __forceinline__ float conf_combine(const ConfTexels& t) {
  const float c10 = t.xin ? t.c10 : 0.0f;
  const float c01 = t.yin ? t.c01 : 0.0f;
  const float c11 = (t.xin && t.yin) ? t.c11 : 0.0f;
  const float gx = 1.0f - t.fx, gy = 1.0f - t.fy;
  const float w00 = gx * gy, w10 = t.fx * gy, w01 = gx * t.fy, w11 = t.fx * t.fy;
  return __builtin_fmaf(w11, c11, __builtin_fmaf(w01, c01, __builtin_fmaf(w10, c10, w00 * t.c00)));
}

// Visibility of Sec. 3.1.1 (the score V_i^v), decided in binary32: the
// camera-space depth of the point agrees with the rendered depth at the
// nearest texel of its projection,
//   ix = (int)floor(u + 0.5f), iy = (int)floor(v + 0.5f),  |Z - D(ix, iy)| <= tau.
// No depth maps: always visible.  A +inf (background) or NaN depth never is.
template <typename T>
__device__ __forceinline__ bool visible32(const void* depth, size_t plane, int view, int W,
                                          int H, const Proj& pr, float tau) {
  if (depth == nullptr) return true;
  const int ix = (int)floorf(pr.u + 0.5f), iy = (int)floorf(pr.v + 0.5f);
  const float D = tex_load_nb<T>((const T*)depth + plane * view, W, H, ix, iy);
  return fabsf(pr.Z - D) <= tau;
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

// Lanes of a wave are split into groups of `k` consecutive lanes; returns the
// sum of v over the caller's group, added in lane order (slot 0 first) so
// every lane of the group gets the same bits.
__device__ __forceinline__ float group_sum(float v, int group_base, int k) {
  float s = __shfl(v, group_base, kWave);
  for (int j = 1; j < k; ++j) s += __shfl(v, group_base + j, kWave);
  return s;
}

// group_sum with the group size known at compile time (KT > 0): the K
// shuffles are issued back to back and waited for once.
template <int KT>
__device__ __forceinline__ float group_sum_t(float v, int group_base, int k) {
  if constexpr (KT > 0) {
    float x[KT];
#pragma unroll
    for (int j = 0; j < KT; ++j) x[j] = __shfl(v, group_base + j, kWave);
    float s = x[0];
#pragma unroll
    for (int j = 1; j < KT; ++j) s += x[j];
    return s;
  } else {
    return group_sum(v, group_base, k);
  }
}

}  // namespace fd
