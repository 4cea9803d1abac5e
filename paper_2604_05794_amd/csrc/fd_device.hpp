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

// Texel of one map as float; outside the image reads 0 (zero border).
template <typename T>
__device__ __forceinline__ float tex_load(const T* __restrict__ m, int W, int H,
                                          int x, int y);

template <>
__device__ __forceinline__ float tex_load<float>(const float* __restrict__ m,
                                                 int W, int H, int x, int y) {
  if ((unsigned)x >= (unsigned)W || (unsigned)y >= (unsigned)H) return 0.0f;
  return m[(size_t)y * W + x];
}

template <>
__device__ __forceinline__ float tex_load<__half>(const __half* __restrict__ m,
                                                  int W, int H, int x, int y) {
  if ((unsigned)x >= (unsigned)W || (unsigned)y >= (unsigned)H) return 0.0f;
  return __half2float(m[(size_t)y * W + x]);
}

// Same value as tex_load, but the load itself is unconditional (at a clamped
// address), so a run of them can be issued back to back.
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

// Bilinear confidence at the projection, same fixed order:
//   x0 = floor(u), fx = u - x0, gx = 1 - fx (likewise y)
//   w00 = gx*gy, w10 = fx*gy, w01 = gx*fy, w11 = fx*fy
//   C = fma(w11, C11, fma(w01, C01, fma(w10, C10, w00*C00)))
template <typename T>
__device__ __forceinline__ float centre_conf32(const T* __restrict__ cm, int W,
                                               int H, float u, float v) {
  float x0 = floorf(u), y0 = floorf(v);
  float fx = u - x0, fy = v - y0;
  float gx = 1.0f - fx, gy = 1.0f - fy;
  int ix = (int)x0, iy = (int)y0;
  float c00 = tex_load_nb<T>(cm, W, H, ix, iy);
  float c10 = tex_load_nb<T>(cm, W, H, ix + 1, iy);
  float c01 = tex_load_nb<T>(cm, W, H, ix, iy + 1);
  float c11 = tex_load_nb<T>(cm, W, H, ix + 1, iy + 1);
  float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  return __builtin_fmaf(w11, c11, __builtin_fmaf(w01, c01, __builtin_fmaf(w10, c10, w00 * c00)));
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

// Centre confidence of a projection for Eq. (4), or 0 when the view is not
// eligible (ok false) or, with depth maps, the point is hidden in it.  Same
// value and operation order as centre_conf32 and visible32; since an eligible
// projection lies inside the image, only the +1 neighbours need the zero
// border check.  cb / db: this view's confidence and depth planes (db NULL:
// no visibility test).  *seen (optional): eligible and visible.
template <typename T>
__device__ __forceinline__ float eligible_conf32(const T* __restrict__ cb,
                                                 const T* __restrict__ db, int W, int H,
                                                 bool ok, const Proj& pr, float tau,
                                                 bool* seen = nullptr) {
  const float u = ok ? pr.u : 0.0f, v = ok ? pr.v : 0.0f;
  const float x0 = floorf(u), y0 = floorf(v);
  const float fx = u - x0, fy = v - y0;
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  const uint32_t ix = (uint32_t)x0, iy = (uint32_t)y0;
  const uint32_t o00 = iy * (uint32_t)W + ix;
  const bool xin = ix + 1u < (uint32_t)W, yin = iy + 1u < (uint32_t)H;
  const uint32_t dx = xin ? 1u : 0u, dy = yin ? (uint32_t)W : 0u;
  float c00 = ld_texel<T>(cb, o00);
  float c10 = ld_texel<T>(cb, o00 + dx);
  float c01 = ld_texel<T>(cb, o00 + dy);
  float c11 = ld_texel<T>(cb, o00 + dx + dy);
  bool vis = true;
  if (db != nullptr) {
    const uint32_t xn = (uint32_t)floorf(u + 0.5f), yn = (uint32_t)floorf(v + 0.5f);
    const float D = ld_texel<T>(db, yn * (uint32_t)W + xn);
    vis = fabsf(pr.Z - D) <= tau;
  }
  c10 = xin ? c10 : 0.0f;
  c01 = yin ? c01 : 0.0f;
  c11 = (xin && yin) ? c11 : 0.0f;
  const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  const float c =
      __builtin_fmaf(w11, c11, __builtin_fmaf(w01, c01, __builtin_fmaf(w10, c10, w00 * c00)));
  if (seen) *seen = ok && vis;  // eligible and visible, whatever the confidence
  return (ok && vis) ? c : 0.0f;
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
