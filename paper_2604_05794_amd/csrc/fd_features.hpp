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
// Scenes with at most this many views take the three-pass form
// (vis_topk_masked, then frontal_row_masked), their visibility bits passed
// between the two through the feature row.
constexpr int kMaskViews = 128;
constexpr float kInvPi = 0.318309886183790671538f;

typedef float feat_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 feat_bf16x2_t __attribute__((ext_vector_type(2)));

// (a, b) rounded to bfloat16 (nearest even; the packed conversion
// instruction), a in the low half.
__device__ __forceinline__ uint32_t feat_bf16x2(float a, float b) {
  const feat_bf16x2_t v = __builtin_convertvector((feat_f32x2){a, b}, feat_bf16x2_t);
  return __builtin_bit_cast(uint32_t, v);
}

// Frontal ranking key of a view (the "most frontal" views of the proposal
// features), in binary64 (the ranking is a discrete decision): with the
// camera centre c = -R^T t from the binary64 table, a = c - p and
// b = p - o (o the head centre, b formed once per point),
//   key = (a . b) / |a|,
// the cosine between the point->camera direction and the outward direction
// p - o, times |p - o| (common to every view of the point); the reciprocal
// square root is the refined hardware estimate.
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
// bfloat16 to feats row `row`.  These are values, not decisions (the slot
// views are chosen in binary64 beforehand), and they are rounded to
// bfloat16 (relative step 2^-8), so apart from the sample position
// (binary64) they are formed in binary32 with the hardware reciprocal,
// square root and sine / cosine (errors ~1e-6 relative).
// One slot of the row, without branches (the slot's view is v; a slot
// that is empty passes valid = false, reads view 0 and yields zeros), so
// that the loads of neighbouring slots can be in flight together.  tab is
// the scene's camera table (kCam64 slots per view; global memory or a copy
// in LDS).  PAIRS: the scene allows texel-pair loads (binary16).
template <typename T, bool PAIRS>
__device__ __forceinline__ void feature_slot(const SceneDev& s, const double* __restrict__ tab,
                                             double px, double py, double pz, int v, bool valid,
                                             float (&f)[7]) {
  const T* th = (const T*)s.theta;
  const T* cf = (const T*)s.conf;
  const size_t plane = (size_t)s.W * s.H;
  // the binary32 record, two values per binary64 slot (read as the slots'
  // own type and split by value, so the accesses match how it was stored)
  const double* rec = tab + kCam64 * v + kCam32Off;
  float cr[16];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float2 pr2 = __builtin_bit_cast(float2, rec[e]);
    cr[2 * e] = pr2.x;
    cr[2 * e + 1] = pr2.y;
  }
  const float4 q0 = make_float4(cr[0], cr[1], cr[2], cr[3]);
  const float4 q1 = make_float4(cr[4], cr[5], cr[6], cr[7]);
  const float4 q2 = make_float4(cr[8], cr[9], cr[10], cr[11]);
  const float4 q3 = make_float4(cr[12], cr[13], cr[14], cr[15]);
  // fx fy cx cy | R0 R1 R2 R3 | R4 R5 R6 R7 | R8 t0 t1 t2
  // the sample position in binary64 from the same record (binary32 would
  // move the bilinear weights by ~5e-5 and flip the bfloat16 rounding of
  // many more values)
  const double dX = __builtin_fma((double)q1.x, px, __builtin_fma((double)q1.y, py,
                                  __builtin_fma((double)q1.z, pz, (double)q3.y)));
  const double dY = __builtin_fma((double)q1.w, px, __builtin_fma((double)q2.x, py,
                                  __builtin_fma((double)q2.y, pz, (double)q3.z)));
  const double dZ = __builtin_fma((double)q2.z, px, __builtin_fma((double)q2.w, py,
                                  __builtin_fma((double)q3.x, pz, (double)q3.w)));
  // a slot's view sees the point: dZ > z_near > 0
  const double idz = rcp64(valid ? dZ : 1.0);
  const double su = valid ? __builtin_fma((double)q0.x, dX * idz, (double)q0.z) : 0.0;
  const double sv = valid ? __builtin_fma((double)q0.y, dY * idz, (double)q0.w) : 0.0;
  const float pX = (float)dX, pY = (float)dY, pZ = (float)dZ;
  // the visible projection lies in [0, W-1] x [0, H-1] (up to the last bit
  // of this binary64 evaluation; the clamp keeps the weights continuous)
  const int ix = min(max((int)floor(su), 0), s.W - 1), iy = min(max((int)floor(sv), 0), s.H - 1);
  const float fx = (float)(su - (double)ix), fy = (float)(sv - (double)iy);
  const bool yin = iy + 1 < s.H;
  // the 2 x 2 texels (zero outside the image)
  float tq[2][2], cq[2][2];
  if constexpr (PAIRS) {
    // one 8-byte load per row and map: the texel pair at a = min(ix & ~1,
    // W - 4) and the next pair (W even, W >= 4, rows 4-byte aligned)
    const uint32_t a = min((uint32_t)ix & ~1u, (uint32_t)s.W - 4u);
    const uint32_t d = (uint32_t)ix - a;  // 0..3
    const uint32_t r0 = (uint32_t)iy * (uint32_t)s.W;
    const uint32_t r1 = r0 + (yin ? (uint32_t)s.W : 0u);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t off = ((b ? r1 : r0) + a) * 2u;
      const uint2 wt = *(const uint2*)((const char*)(th + plane * v) + off);
      const uint2 wc = *(const uint2*)((const char*)(cf + plane * v) + off);
      const uint64_t pt = ((uint64_t)wt.y << 32) | wt.x, pc = ((uint64_t)wc.y << 32) | wc.x;
      const bool row_in = b == 0 || yin;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint32_t k = d + (uint32_t)e;  // 4: texel W, outside
        const bool in = row_in && k < 4u;
        const uint32_t sh = 16u * (k & 3u);
        tq[b][e] = in ? __half2float(__ushort_as_half((unsigned short)(pt >> sh))) : 0.0f;
        cq[b][e] = in ? __half2float(__ushort_as_half((unsigned short)(pc >> sh))) : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        tq[b][e] = tex_load_nb<T>(th + plane * v, s.W, s.H, ix + e, iy + b);
        cq[b][e] = tex_load_nb<T>(cf + plane * v, s.W, s.H, ix + e, iy + b);
      }
  }
  float cb = 0.0f, mx = 0.0f, my = 0.0f;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float w = (e ? fx : 1.0f - fx) * (b ? fy : 1.0f - fy);
      const float wc = w * cq[b][e];
      cb += wc;
      mx = __builtin_fmaf(wc, __builtin_amdgcn_cosf(tq[b][e] * kInvPi), mx);
      my = __builtin_fmaf(wc, __builtin_amdgcn_sinf(tq[b][e] * kInvPi), my);
    }
  // unit point -> camera direction vd: centre c = -R^T t
  const float qx0 = (float)px, qy0 = (float)py, qz0 = (float)pz;
  const float ccx = -__builtin_fmaf(q1.x, q3.y, __builtin_fmaf(q1.w, q3.z, q2.z * q3.w));
  const float ccy = -__builtin_fmaf(q1.y, q3.y, __builtin_fmaf(q2.x, q3.z, q2.w * q3.w));
  const float ccz = -__builtin_fmaf(q1.z, q3.y, __builtin_fmaf(q2.y, q3.z, q3.x * q3.w));
  float vd[3] = {ccx - qx0, ccy - qy0, ccz - qz0};
  {
    const float il = __builtin_amdgcn_rsqf(
        __builtin_fmaf(vd[0], vd[0], __builtin_fmaf(vd[1], vd[1], vd[2] * vd[2])));
    vd[0] *= il;
    vd[1] *= il;
    vd[2] *= il;
  }
  // The observed image line back-projects to a plane through the camera
  // centre containing the line of sight vd; its direction across vd,
  // tt = n x vd, is given by the angle psi in the frame
  // e1 = normalize(z x vd), e2 = vd x e1, carried as |m| (cos 2psi, sin 2psi).
  float qx = 0.0f, qy = 0.0f;
  const float m2 = __builtin_fmaf(mx, mx, my * my);
  if (m2 > 0.0f) {
    const float imag = __builtin_amdgcn_rsqf(m2);
    const float mag = m2 * imag;
    const float ch = mx * imag, sh = my * imag;  // cos, sin of 2 theta
    const float ox = __builtin_amdgcn_sqrtf(fmaxf(0.5f * (1.0f + ch), 0.0f));
    const float oy = copysignf(__builtin_amdgcn_sqrtf(fmaxf(0.5f * (1.0f - ch), 0.0f)), sh);
    const float dlx = ox * __builtin_amdgcn_rcpf(q0.x), dly = oy * __builtin_amdgcn_rcpf(q0.y);
    const float ncx = -pZ * dly, ncy = pZ * dlx, ncz = pX * dly - pY * dlx;
    const float nwx = __builtin_fmaf(q1.x, ncx, __builtin_fmaf(q1.w, ncy, q2.z * ncz));
    const float nwy = __builtin_fmaf(q1.y, ncx, __builtin_fmaf(q2.x, ncy, q2.w * ncz));
    const float nwz = __builtin_fmaf(q1.z, ncx, __builtin_fmaf(q2.y, ncy, q3.x * ncz));
    const float tx = nwy * vd[2] - nwz * vd[1];
    const float ty = nwz * vd[0] - nwx * vd[2];
    const float tz = nwx * vd[1] - nwy * vd[0];
    const bool vert = fabsf(vd[2]) > 1.0f - 1e-6f;
    const float ux = vert ? 1.0f : 0.0f, uz = vert ? 0.0f : 1.0f;
    // e1 = up x vd, up = (ux, 0, uz)
    float e1x = -uz * vd[1], e1y = uz * vd[0] - ux * vd[2], e1z = ux * vd[1];
    const float il = __builtin_amdgcn_rsqf(
        __builtin_fmaf(e1x, e1x, __builtin_fmaf(e1y, e1y, e1z * e1z)));
    e1x *= il;
    e1y *= il;
    e1z *= il;
    const float e2x = vd[1] * e1z - vd[2] * e1y;
    const float e2y = vd[2] * e1x - vd[0] * e1z;
    const float e2z = vd[0] * e1y - vd[1] * e1x;
    const float t1 = __builtin_fmaf(tx, e1x, __builtin_fmaf(ty, e1y, tz * e1z));
    const float t2 = __builtin_fmaf(tx, e2x, __builtin_fmaf(ty, e2y, tz * e2z));
    const float tn = __builtin_fmaf(t1, t1, t2 * t2);
    if (tn > 0.0f) {
      const float r = mag * __builtin_amdgcn_rcpf(tn);
      qx = r * __builtin_fmaf(t1, t1, -t2 * t2);
      qy = r * 2.0f * t1 * t2;
    }
  }
  f[0] = valid ? qx : 0.0f;
  f[1] = valid ? qy : 0.0f;
  f[2] = valid ? cb : 0.0f;
  f[3] = valid ? vd[0] : 0.0f;
  f[4] = valid ? vd[1] : 0.0f;
  f[5] = valid ? vd[2] : 0.0f;
  f[6] = valid ? 1.0f : 0.0f;
}

// Per slot of the frontal list: the observed orientation as
// (q_x, q_y) = |m| (cos 2psi, sin 2psi) (m the bilinear confidence-weighted
// doubled-angle vector, psi the angle of the plane it back-projects to, in a
// frame tied to the line of sight), the bilinear confidence C, the unit
// point->camera direction and 1; empty slots are 0.  Written as 112
// bfloat16 to feats row `row`.  These are values, not decisions (the slot
// views are chosen in binary64 beforehand), and they are rounded to
// bfloat16 (relative step 2^-8), so apart from the sample position
// (binary64) they are formed in binary32 with the hardware reciprocal,
// square root and sine / cosine (errors ~1e-6 relative).
template <typename T, bool PAIRS>
__device__ __forceinline__ void write_feature_row_t(const SceneDev& s,
                                                    const double* __restrict__ tab, double px,
                                                    double py, double pz,
                                                    const int (&id)[kSlots], int64_t row,
                                                    uint16_t* __restrict__ feats) {
  // slots in pairs, whose 14 values convert to 7 packed bfloat16 pairs and
  // are stored at once (rows are 224 bytes, so every pair starts on a
  // 4-byte boundary); one pair is processed per pass, the views of the
  // next pair moved to the front of the list
  static_assert(kSlots % 2 == 0, "slots are converted in pairs");
  uint32_t* dst = (uint32_t*)(feats + (size_t)row * (7 * kSlots));
  int idr[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) idr[k] = id[k];
#pragma unroll 1
  for (int kp = 0; kp < kSlots; kp += 2) {
    float f0[7], f1[7];
    feature_slot<T, PAIRS>(s, tab, px, py, pz, max(idr[0], 0), idr[0] >= 0, f0);
    feature_slot<T, PAIRS>(s, tab, px, py, pz, max(idr[1], 0), idr[1] >= 0, f1);
    float f2[14];
#pragma unroll
    for (int e = 0; e < 7; ++e) {
      f2[e] = f0[e];
      f2[7 + e] = f1[e];
    }
#pragma unroll
    for (int e = 0; e < 7; ++e) dst[7 * (kp / 2) + e] = feat_bf16x2(f2[2 * e], f2[2 * e + 1]);
#pragma unroll
    for (int k = 0; k + 2 < kSlots; ++k) idr[k] = idr[k + 2];
  }
}

template <typename T>
__device__ __forceinline__ void write_feature_row(const SceneDev& s, const double* __restrict__ tab,
                                                  double px, double py, double pz,
                                                  const int (&id)[kSlots], int64_t row,
                                                  uint16_t* __restrict__ feats) {
  if (sizeof(T) == 2 && s.pairs)
    write_feature_row_t<T, true>(s, tab, px, py, pz, id, row, feats);
  else
    write_feature_row_t<T, false>(s, tab, px, py, pz, id, row, feats);
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
  write_feature_row<T>(s, s.cam64, px, py, pz, id, row_base + (by_j ? j : (int64_t)i), feats);
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
      if (any[u]) tx[u] = conf_texels<T>(conf + plane * (v0 + u), s.W, s.H, seen[u], pr[u], s.pairs);
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
  write_feature_row<T>(s, s.cam64, px, py, pz, id, row_base + j, feats);
}

// Bitwise OR of m over the wave, in a scalar register.
__device__ __forceinline__ uint32_t wave_or32(uint32_t m) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) m |= (uint32_t)__shfl_xor((int)m, off, kWave);
  return __builtin_amdgcn_readfirstlane(m);
}

// For scenes of at most 32 MW views the view selection and the features
// run as two kernels, each holding less state.  The first
// (vis_topk_masked) makes the Eq. (4) selection (four views at a time, as
// topk_point) and keeps each view's visibility as a bit in MW registers,
// which it leaves in the first 4 MW bytes of the point's feature row; the
// second (frontal_row_masked) takes the bits back, ranks the visible views
// by frontality (projections and depth texels are not read again; the
// views are taken in increasing order, so the list is the same as the
// one-pass form's) and writes the row over them.  The gather loop of the
// first then runs at the occupancy its own registers allow.  ctab is the
// scene's camera table, read at wave-uniform addresses only (the caller may
// pass the global table, whose records then come through the scalar cache
// without taking vector registers, or a copy in LDS).
template <typename T, int KS, int MW>
__device__ __forceinline__ void vis_topk_masked(const SceneDev& s, const SearchDev& q,
                                                const double* __restrict__ ctab, int64_t j,
                                                int64_t row, uint16_t* __restrict__ feats) {
  static_assert(4 * MW <= 14 * kSlots, "the bits fit in the row");
  const uint32_t i = s.perm[j];
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  const T* conf = (const T*)s.conf;
  const T* depth = (const T*)s.depth;
  const size_t plane = (size_t)s.W * s.H;
  const double tau = (double)s.vis_tau;
  uint32_t mask[MW];
  {
    double ck[KS];
    int vk[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      ck[k] = -1.0;
      vk[k] = 0;
    }
    constexpr int kGroup = 4;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      uint32_t bits = 0;
      const int vend = min(s.V, 32 * (w + 1));
      for (int v0 = 32 * w; v0 < vend; v0 += kGroup) {
        ProjT pr[kGroup];
        bool seen[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          const int v = min(v0 + u, s.V - 1);
          const bool ok =
              project_tab(ctab + kCam64 * v, px, py, pz, s.W, s.H, q.z_near, pr[u]);
          seen[u] = visible_at<T>(depth ? depth + plane * v : nullptr, s.W, ok, pr[u], tau) &&
                    v0 + u < s.V;
          bits |= (seen[u] ? 1u : 0u) << (v0 + u - 32 * w);
        }
        ConfTexels tx[kGroup];
        bool any[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          any[u] = __ballot(seen[u]) != 0;  // wave-uniform
          if (any[u]) tx[u] = conf_texels<T>(conf + plane * (v0 + u), s.W, s.H, seen[u], pr[u], s.pairs);
        }
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          if (!any[u]) continue;
          const double c = seen[u] ? conf_combine(tx[u]) : 0.0;
          if (c > 0.0) topk_insert<KS>(ck, vk, c, v0 + u);
        }
      }
      mask[w] = bits;
    }
    int keff = 0;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      if (k < q.K && ck[k] > 0.0) keff = k + 1;
      s.views[FD_TOPK_SLOTS * j + k] = (uint16_t)vk[k];
    }
    s.kcount[j] = (uint8_t)keff;
  }
  uint32_t* bits_out = (uint32_t*)(feats + (size_t)row * (7 * kSlots));
#pragma unroll
  for (int w = 0; w < MW; ++w) bits_out[w] = mask[w];
}

template <typename T, int MW>
__device__ __forceinline__ void frontal_row_masked(const SceneDev& s,
                                                   const double* __restrict__ ctab, int64_t j,
                                                   int64_t row, uint16_t* __restrict__ feats) {
  const uint32_t i = s.perm[j];
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  uint32_t mask[MW];
  const uint32_t* bits_in = (const uint32_t*)(feats + (size_t)row * (7 * kSlots));
#pragma unroll
  for (int w = 0; w < MW; ++w) mask[w] = bits_in[w];
  double sc[kSlots];
  int id[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    sc[k] = -INFINITY;
    id[k] = -1;
  }
  const double bx = px - (double)s.hc[0], by = py - (double)s.hc[1], bz = pz - (double)s.hc[2];
#pragma unroll
  for (int w = 0; w < MW; ++w) {
    uint32_t um = wave_or32(mask[w]);  // views some lane of the wave sees
    while (um) {
      const int b = __builtin_ctz(um);
      um &= um - 1u;
      const int v = 32 * w + b;
      if ((mask[w] >> b) & 1u)
        frontal_insert(sc, id, frontal_key(ctab + kCam64 * v, px, py, pz, bx, by, bz), v);
    }
  }
  // the row reads its slots' camera records from the global table: their
  // views differ from lane to lane (per-lane reads of the LDS copy have
  // given results that varied from run to run)
  write_feature_row<T>(s, s.cam64, px, py, pz, id, row, feats);
}

}  // namespace fd
