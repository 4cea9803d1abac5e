// fd_features.hpp -- per-point device code of the proposal-network input
// (the most frontal views of a point and what each of them observes).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/fusedir.h"
#include "fd_device.hpp"
#include "fd_kernels.hpp"
#include "fd_search.hpp"

namespace fd {

constexpr int kSlots = FD_FEATURE_SLOTS;
constexpr float kInvPi = 0.318309886183790671538f;

__device__ __forceinline__ uint16_t feat_bf16(float x) {
  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Frontal ranking key of a view (the "most frontal" views of the proposal
// features), in binary64 (the ranking is a discrete decision):
//   c = -R^T t  (c_k = -((R_k t0 + R_{3+k} t1) + R_{6+k} t2))
//   a = c - p, b = p - o
//   score = ((a_x b_x + a_y b_y) + a_z b_z) / sqrt((a_x^2 + a_y^2) + a_z^2)
// i.e. the cosine between the point->camera direction and the outward
// direction p - o, times |p - o| (common to every view of the point).
// vdir (optional) receives the unit point->camera direction a / |a|.
__device__ __forceinline__ double frontal_score64(const float* cam, double px, double py,
                                                  double pz, const float* o, float* vdir) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  const double t0 = t[0], t1 = t[1], t2 = t[2];
  const double cx = -((double)R[0] * t0 + (double)R[3] * t1 + (double)R[6] * t2);
  const double cy = -((double)R[1] * t0 + (double)R[4] * t1 + (double)R[7] * t2);
  const double cz = -((double)R[2] * t0 + (double)R[5] * t1 + (double)R[8] * t2);
  const double ax = cx - px, ay = cy - py, az = cz - pz;
  const double bx = px - (double)o[0], by = py - (double)o[1], bz = pz - (double)o[2];
  const double la = sqrt(ax * ax + ay * ay + az * az);
  if (vdir) {
    vdir[0] = (float)(ax / la);
    vdir[1] = (float)(ay / la);
    vdir[2] = (float)(az / la);
  }
  return (ax * bx + ay * by + az * bz) / la;
}

// The frontal key in the loop over every view of a point, from the camera
// centre in the binary64 table and b = p - o computed once per point:
// (a . b) / |a| with a reciprocal square root (agrees with frontal_score64
// up to binary64 rounding).
__device__ __forceinline__ double frontal_key(const double* __restrict__ c64, double px,
                                              double py, double pz, double bx, double by,
                                              double bz) {
  const double ax = c64[12] - px, ay = c64[13] - py, az = c64[14] - pz;
  const double dot = __builtin_fma(ax, bx, __builtin_fma(ay, by, az * bz));
  const double la2 = __builtin_fma(ax, ax, __builtin_fma(ay, ay, az * az));
  return dot * rsq64(la2);
}

// Stable insertion of view v with frontal score cs into the descending list
// (sc, id) of kSlots entries (empty entries hold -inf): equal scores keep the
// lower view index first; a view that does not beat the last entry is
// skipped.  The score of an eligible view is finite (the point lies more
// than z_near in front of the camera, so its distance to the centre is not
// zero for any z_near > 0), so it always beats an empty entry.
__device__ __forceinline__ void frontal_insert(double (&sc)[kSlots], int (&id)[kSlots],
                                               double cs, int cv) {
  if (!(cs > sc[kSlots - 1])) return;
  bool ins = false;
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    const bool take = ins || (cs > sc[k]);
    const double ts = sc[k];
    const int tv = id[k];
    sc[k] = take ? cs : ts;
    id[k] = take ? cv : tv;
    cs = take ? ts : cs;
    cv = take ? tv : cv;
    ins = ins || take;
  }
}

// Per slot of the frontal list: the observed orientation as
// (q_x, q_y) = |m| (cos 2psi, sin 2psi) (m the bilinear confidence-weighted
// doubled-angle vector, psi the angle of the plane it back-projects to, in a
// frame tied to the line of sight), the bilinear confidence C, the unit
// point->camera direction and 1; empty slots are 0.  Written as 112
// bfloat16 to feats row `row`.  The sample position is the binary64
// projection; the values are formed in binary32 (the hardware sine and
// cosine of the texel angles err by ~1e-6, far below the 2^-9 relative
// rounding of bfloat16).
template <typename T>
__device__ __forceinline__ void write_feature_row(const SceneDev& s, double z_near, double px,
                                                  double py, double pz, const int (&id)[kSlots],
                                                  int64_t row, uint16_t* __restrict__ feats) {
  const T* th = (const T*)s.theta;
  const T* cf = (const T*)s.conf;
  const size_t plane = (size_t)s.W * s.H;
  // the row in two halves of kSlots / 2 slots (7 x 16 bytes each), so that
  // only half of it is held in registers at a time
  constexpr int kHalf = kSlots / 2;
  static_assert((7 * kHalf * 2) % 16 == 0, "half rows are whole 16-byte chunks");
  uint4* dst = (uint4*)(feats + (size_t)row * (7 * kSlots));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
  uint16_t out[7 * kHalf];
#pragma unroll
  for (int kk = 0; kk < kHalf; ++kk) {
    const int k = h * kHalf + kk;
    float f[7] = {0, 0, 0, 0, 0, 0, 0};
    if (id[k] >= 0) {
      const int v = id[k];
      const float* cam = s.cams + 16 * v;
      Proj pr;
      project64(cam, px, py, pz, s.W, s.H, z_near, pr);
      const double x0 = floor(pr.u), y0 = floor(pr.v);
      const float fx = (float)(pr.u - x0), fy = (float)(pr.v - y0);
      const int ix = (int)x0, iy = (int)y0;
      const float pX = (float)pr.X, pY = (float)pr.Y, pZ = (float)pr.Z;
      float cb = 0.0f, mx = 0.0f, my = 0.0f;
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const float w = (a ? fx : 1.0f - fx) * (b ? fy : 1.0f - fy);
          const float t = tex_load_nb<T>(th + plane * v, s.W, s.H, ix + a, iy + b);
          const float c = tex_load_nb<T>(cf + plane * v, s.W, s.H, ix + a, iy + b);
          const float wc = w * c;
          cb += wc;
          mx += wc * __builtin_amdgcn_cosf(t * kInvPi);
          my += wc * __builtin_amdgcn_sinf(t * kInvPi);
        }
      float vd[3];
      frontal_score64(cam, px, py, pz, s.hc, vd);
      // The observed image line back-projects to a plane through the camera
      // centre containing the line of sight vd; its direction across vd,
      // tt = n x vd, is given by the angle psi in the frame
      // e1 = normalize(z x vd), e2 = vd x e1, carried as |m| (cos 2psi, sin 2psi).
      float qx = 0.0f, qy = 0.0f;
      const float mag = sqrtf(mx * mx + my * my);
      if (mag > 0.0f) {
        const float ch = mx / mag, sh = my / mag;  // cos, sin of 2 theta
        const float ox = sqrtf(fmaxf(0.5f * (1.0f + ch), 0.0f));
        const float oy = copysignf(sqrtf(fmaxf(0.5f * (1.0f - ch), 0.0f)), sh);
        const float dlx = ox / cam[0], dly = oy / cam[1];
        const float ncx = -pZ * dly, ncy = pZ * dlx, ncz = pX * dly - pY * dlx;
        const float* R = cam + 4;
        const float nwx = R[0] * ncx + R[3] * ncy + R[6] * ncz;
        const float nwy = R[1] * ncx + R[4] * ncy + R[7] * ncz;
        const float nwz = R[2] * ncx + R[5] * ncy + R[8] * ncz;
        const float tx = nwy * vd[2] - nwz * vd[1];
        const float ty = nwz * vd[0] - nwx * vd[2];
        const float tz = nwx * vd[1] - nwy * vd[0];
        const bool vert = fabsf(vd[2]) > 1.0f - 1e-6f;
        const float ux = vert ? 1.0f : 0.0f, uz = vert ? 0.0f : 1.0f;
        // e1 = up x vd, up = (ux, 0, uz)
        float e1x = -uz * vd[1], e1y = uz * vd[0] - ux * vd[2], e1z = ux * vd[1];
        const float il = 1.0f / sqrtf(e1x * e1x + e1y * e1y + e1z * e1z);
        e1x *= il;
        e1y *= il;
        e1z *= il;
        const float e2x = vd[1] * e1z - vd[2] * e1y;
        const float e2y = vd[2] * e1x - vd[0] * e1z;
        const float e2z = vd[0] * e1y - vd[1] * e1x;
        const float t1 = tx * e1x + ty * e1y + tz * e1z;
        const float t2 = tx * e2x + ty * e2y + tz * e2z;
        const float tn = t1 * t1 + t2 * t2;
        if (tn > 0.0f) {
          qx = mag * (t1 * t1 - t2 * t2) / tn;
          qy = mag * 2.0f * t1 * t2 / tn;
        }
      }
      f[0] = qx;
      f[1] = qy;
      f[2] = cb;
      f[3] = vd[0];
      f[4] = vd[1];
      f[5] = vd[2];
      f[6] = 1.0f;
    }
#pragma unroll
    for (int e = 0; e < 7; ++e) out[7 * kk + e] = feat_bf16(f[e]);
  }
  const uint4* src = (const uint4*)out;
#pragma unroll
  for (int e = 0; e < (7 * kHalf * 2) / 16; ++e) dst[h * ((7 * kHalf * 2) / 16) + e] = src[e];
  }
}

// One lane per point: the kSlots most frontal eligible views, then their
// feature row (processing-order index j when by_j, else the point index,
// plus row_base).
template <typename T>
__device__ __forceinline__ void features_point(const SceneDev& s, double z_near, int64_t j,
                                               int by_j, int64_t row_base,
                                               uint16_t* __restrict__ feats) {
  const uint32_t i = s.perm ? s.perm[j] : (uint32_t)j;
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  double sc[kSlots];
  int id[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    sc[k] = -INFINITY;
    id[k] = -1;
  }
  const size_t plane = (size_t)s.W * s.H;
  const T* depth = (const T*)s.depth;
  const double bx = px - (double)s.hc[0], by = py - (double)s.hc[1], bz = pz - (double)s.hc[2];
  for (int v = 0; v < s.V; ++v) {
    ProjT pr;
    const bool ok = project_tab(s.cam64 + kCam64 * v, px, py, pz, s.W, s.H, z_near, pr);
    if (!visible_at<T>(depth ? depth + plane * v : nullptr, s.W, ok, pr, (double)s.vis_tau))
      continue;
    frontal_insert(sc, id, frontal_key(s.cam64 + kCam64 * v, px, py, pz, bx, by, bz), v);
  }
  write_feature_row<T>(s, z_near, px, py, pz, id, row_base + (by_j ? j : (int64_t)i), feats);
}

// Eq. (4) view selection and the proposal features in one pass over the
// views (one projection per view): writes views / kcount like topk_point
// and feature row row_base + j.
template <typename T, int KS>
__device__ __forceinline__ void topk_features_point(const SceneDev& s, const SearchDev& q,
                                                    int64_t j, int64_t row_base,
                                                    uint16_t* __restrict__ feats) {
  const uint32_t i = s.perm[j];
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  double ck[KS];
  int vk[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    ck[k] = -1.0;
    vk[k] = 0;
  }
  double sc[kSlots];
  int id[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    sc[k] = -INFINITY;
    id[k] = -1;
  }
  const T* conf = (const T*)s.conf;
  const T* depth = (const T*)s.depth;
  const size_t plane = (size_t)s.W * s.H;
  const double tau = (double)s.vis_tau;
  const double bx = px - (double)s.hc[0], by = py - (double)s.hc[1], bz = pz - (double)s.hc[2];
  // views in groups of two (four as in topk_point would hold more registers
  // next to the frontal list): a view no lane of the wave sees skips its
  // confidence texels and both insertions
  constexpr int kGroup = 2;
  for (int v0 = 0; v0 < s.V; v0 += kGroup) {
    ProjT pr[kGroup];
    bool seen[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int v = min(v0 + u, s.V - 1);
      const bool ok = project_tab(s.cam64 + kCam64 * v, px, py, pz, s.W, s.H, q.z_near, pr[u]);
      seen[u] = visible_at<T>(depth ? depth + plane * v : nullptr, s.W, ok, pr[u], tau) &&
                v0 + u < s.V;
    }
    ConfTexels tx[kGroup];
    bool any[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      any[u] = __ballot(seen[u]) != 0;  // wave-uniform
      if (any[u]) tx[u] = conf_texels<T>(conf + plane * (v0 + u), s.W, s.H, seen[u], pr[u]);
    }
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      if (!any[u]) continue;
      const int v = v0 + u;
      const double c = seen[u] ? conf_combine(tx[u]) : 0.0;
      if (c > 0.0) topk_insert<KS>(ck, vk, c, v);
      // frontal slots: eligible and visible views, whatever their confidence
      if (seen[u])
        frontal_insert(sc, id, frontal_key(s.cam64 + kCam64 * v, px, py, pz, bx, by, bz), v);
    }
  }
  int keff = 0;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    if (k < q.K && ck[k] > 0.0) keff = k + 1;
    s.views[FD_TOPK_SLOTS * j + k] = (uint16_t)vk[k];
  }
  s.kcount[j] = (uint8_t)keff;
  write_feature_row<T>(s, q.z_near, px, py, pz, id, row_base + j, feats);
}

}  // namespace fd
