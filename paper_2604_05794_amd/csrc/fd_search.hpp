// fd_search.hpp -- per-point device code of the direction search, shared by
// the single-scene kernels (fd_fuse.hip) and the batched ones
// (fd_batched.hip).  EfficientMonoHair, Sec. 3.1: Eq. (4) view selection,
// Eqs. (8)-(11) objective, Eq. (12) best candidate, pattern-search
// refinement.
//
// Precision.  View selection is decided in binary64 (fd_device.hpp).  The
// lattice stage of Eq. (12) scores its candidates in binary32 on binary32
// patch coefficients (the bulk of the work: the best lattice point is far
// from the runner-up in all but a vanishing fraction of points).  The
// refinement compares candidates whose costs differ by as little as the
// square of its last steps (~1e-6), which binary32 rounding of the cost
// itself (~1e-7) would decide at random in a few percent of points; it
// therefore scores each candidate by the change of the cost from the
// centre, formed from differences so that the rounding is relative to the
// change (view_delta).  The reported cost is
// the objective at the result evaluated in binary64 (on the binary32
// coefficients, whose rounding moves the cost smoothly with the direction).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fd_device.hpp"
#include "fd_kernels.hpp"

namespace fd {

// ---- Eq. (4): top-K views by centre confidence ------------------------------
// One lane per point (processing-order index j).  Stable insertion into a
// register list of KS >= K slots: a view enters ahead of a listed one only if
// strictly more confident, so equal confidences keep the lower view index
// first.  Slots 0..KS-1 of the point's view row are written.
template <int KS, typename S>
__device__ __forceinline__ void topk_insert(S (&sc)[KS], int (&id)[KS], S c, int v) {
  S cs = c;
  int cv = v;
  bool ins = false;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const bool take = ins || (cs > sc[k]);
    const S ts = sc[k];
    const int tv = id[k];
    sc[k] = take ? cs : ts;
    id[k] = take ? cv : tv;
    cs = take ? ts : cs;
    cv = take ? tv : cv;
    ins = take;
  }
}

template <typename T, int KS>
__device__ __forceinline__ void topk_point(const SceneDev& s, const SearchDev& q, int64_t j) {
  const uint32_t i = s.perm[j];
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  double sc[KS];
  int id[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    sc[k] = -1.0;
    id[k] = 0;
  }
  const T* conf = (const T*)s.conf;
  const T* depth = (const T*)s.depth;
  const size_t plane = (size_t)s.W * s.H;
  const double tau = (double)s.vis_tau;
  // Views in groups of kGroup.  Projections and depth texels of a group are
  // issued together; a view that no lane of the wave sees (all hidden, behind
  // or outside, common for the far side of a head) skips its confidence
  // texels and insertion.  The confidence loads of the seen views are issued
  // before any of them is used.
  constexpr int kGroup = 4;
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
      const double c = seen[u] ? conf_combine(tx[u]) : 0.0;
      if (c > 0.0) topk_insert<KS>(sc, id, c, v0 + u);
    }
  }
  int keff = 0;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    if (k < q.K && sc[k] > 0.0) keff = k + 1;
    s.views[FD_TOPK_SLOTS * j + k] = (uint16_t)id[k];
  }
  s.kcount[j] = (uint8_t)keff;
}

// ---- per-lane view state ------------------------------------------------------

template <int P>
struct ViewPatch {
  static constexpr int P2 = P * P;
  float a[P2], b[P2], c[P2];  // quadratic-form coefficients per patch sample
  float M[6];                  // image direction r = M d (rows of the projection Jacobian)
};

// Build the lane's view state: Jacobian rows and the P x P patch of Sec. 3.1.3
// centred on the projection (offsets (a, b) in {-h..h}^2 pixels from the
// sub-pixel centre, each a bilinear sample of the doubled-angle vector
// weighted by bilinear weight times confidence, zero outside the image).
// The projection and the Jacobian are taken in binary64 and rounded once;
// the texel angles go through an accurate sine/cosine (sincos_reduced), and
// the sample's normalisation through IEEE square root and division.
template <typename T, int P>
__device__ __forceinline__ void build_patch(const SceneDev& s, const SearchDev& q, int view,
                                            bool active, double px, double py, double pz,
                                            ViewPatch<P>& vp) {
  constexpr int P2 = P * P, HP = (P - 1) / 2;
#pragma unroll
  for (int k = 0; k < P2; ++k) vp.a[k] = vp.b[k] = vp.c[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) vp.M[k] = 0.0f;
  if (!active) return;
  const float* cam = s.cams + 16 * view;
  Proj pr;
  project64(cam, px, py, pz, s.W, s.H, q.z_near, pr);
  // r = J_pi d up to the positive factor 1/Z^2:
  //   r_x = fx (Z (R0 . d) - X (R2 . d)),  r_y = fy (Z (R1 . d) - Y (R2 . d))
  const float* R = cam + 4;
  const double f0 = cam[0], f1 = cam[1];
  vp.M[0] = (float)(f0 * (pr.Z * R[0] - pr.X * R[6]));
  vp.M[1] = (float)(f0 * (pr.Z * R[1] - pr.X * R[7]));
  vp.M[2] = (float)(f0 * (pr.Z * R[2] - pr.X * R[8]));
  vp.M[3] = (float)(f1 * (pr.Z * R[3] - pr.Y * R[6]));
  vp.M[4] = (float)(f1 * (pr.Z * R[4] - pr.Y * R[7]));
  vp.M[5] = (float)(f1 * (pr.Z * R[5] - pr.Y * R[8]));

  const size_t plane = (size_t)s.W * s.H;
  const T* th = (const T*)s.theta + plane * view;
  const T* cf = (const T*)s.conf + plane * view;
  const double x0 = floor(pr.u), y0 = floor(pr.v);
  const float fx = (float)(pr.u - x0), fy = (float)(pr.v - y0);
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  const int ix = (int)x0 - HP, iy = (int)y0 - HP;
  // texel rows of the (P+1)^2 footprint: C, C cos 2theta, C sin 2theta
  float rc[2][P + 1], rx[2][P + 1], ry[2][P + 1];
  // binary16 rows away from the right edge of an even-width, 4-byte aligned
  // map: one 16-byte load per map covers texels [ix & ~1, (ix & ~1) + 7]
  const bool wide_ok = sizeof(T) == 2 && P <= 5 && s.pairs;
  auto load_row = [&](int slot, int y) {
    float tv[P + 1], cv[P + 1];
    const int a0 = ix & ~1;
    if (wide_ok && ix >= 0 && a0 + 7 <= s.W - 1 && (unsigned)y < (unsigned)s.H) {
      const size_t off = (size_t)y * s.W + a0;
      const uint4 wt = *(const uint4*)((const uint16_t*)th + off);
      const uint4 wc = *(const uint4*)((const uint16_t*)cf + off);
      // shift the 8 halves right by one half for an odd start (funnel shift)
      const uint32_t sh = (ix & 1) ? 16u : 0u;
      const uint32_t t0 = __builtin_amdgcn_alignbit(wt.y, wt.x, sh);
      const uint32_t t1 = __builtin_amdgcn_alignbit(wt.z, wt.y, sh);
      const uint32_t t2 = __builtin_amdgcn_alignbit(wt.w, wt.z, sh);
      const uint32_t c0 = __builtin_amdgcn_alignbit(wc.y, wc.x, sh);
      const uint32_t c1 = __builtin_amdgcn_alignbit(wc.z, wc.y, sh);
      const uint32_t c2 = __builtin_amdgcn_alignbit(wc.w, wc.z, sh);
      const uint32_t tw[3] = {t0, t1, t2}, cw[3] = {c0, c1, c2};
#pragma unroll
      for (int a = 0; a <= P; ++a) {
        const uint32_t wtv = tw[a >> 1], wcv = cw[a >> 1];
        tv[a] = __half2float(__ushort_as_half((unsigned short)((a & 1) ? (wtv >> 16) : (wtv & 0xffffu))));
        cv[a] = __half2float(__ushort_as_half((unsigned short)((a & 1) ? (wcv >> 16) : (wcv & 0xffffu))));
      }
    } else {
#pragma unroll
      for (int a = 0; a <= P; ++a) {
        tv[a] = tex_load_nb<T>(th, s.W, s.H, ix + a, y);
        cv[a] = tex_load_nb<T>(cf, s.W, s.H, ix + a, y);
      }
    }
#pragma unroll
    for (int a = 0; a <= P; ++a) {
      float sn, cs;
      sincos_reduced(2.0f * tv[a], &sn, &cs);  // 2 theta is exact in binary32
      rc[slot][a] = cv[a];
      rx[slot][a] = cv[a] * cs;
      ry[slot][a] = cv[a] * sn;
    }
  };
  load_row(0, iy);
#pragma unroll
  for (int b = 0; b < P; ++b) {
    const int r0 = b & 1, r1 = (b + 1) & 1;
    load_row(r1, iy + b + 1);
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const float cb = w00 * rc[r0][a] + w10 * rc[r0][a + 1] + w01 * rc[r1][a] + w11 * rc[r1][a + 1];
      const float mx = w00 * rx[r0][a] + w10 * rx[r0][a + 1] + w01 * rx[r1][a] + w11 * rx[r1][a + 1];
      const float my = w00 * ry[r0][a] + w10 * ry[r0][a + 1] + w01 * ry[r1][a] + w11 * ry[r1][a + 1];
      const float n2 = mx * mx + my * my;
      const float al = 0.5f * cb * cb;
      const bool on = n2 > 0.0f;
      const float n = on ? sqrtf(n2) : 1.0f;
      const int k = b * P + a;
      vp.a[k] = on ? al : 0.0f;
      vp.b[k] = on ? al * mx / n : 0.0f;
      vp.c[k] = on ? 2.0f * al * my / n : 0.0f;  // the factor 2 of 2 rx ry folded in
    }
  }
}

// The patch in binary64 throughout (texel angles, bilinear weights,
// normalisation, Jacobian): the paper-literal candidate mode, which scores a
// handful of candidates per point and compares their costs directly.
template <int P>
struct ViewPatch64 {
  static constexpr int P2 = P * P;
  double a[P2], b[P2], c[P2];
  double M[6];
};

template <typename T, int P>
__device__ __forceinline__ void build_patch64(const SceneDev& s, const SearchDev& q, int view,
                                              bool active, double px, double py, double pz,
                                              ViewPatch64<P>& vp) {
  constexpr int P2 = P * P, HP = (P - 1) / 2;
#pragma unroll
  for (int k = 0; k < P2; ++k) vp.a[k] = vp.b[k] = vp.c[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) vp.M[k] = 0.0;
  if (!active) return;
  const float* cam = s.cams + 16 * view;
  Proj pr;
  project64(cam, px, py, pz, s.W, s.H, q.z_near, pr);
  const float* R = cam + 4;
  const double f0 = cam[0], f1 = cam[1];
  vp.M[0] = f0 * (pr.Z * R[0] - pr.X * R[6]);
  vp.M[1] = f0 * (pr.Z * R[1] - pr.X * R[7]);
  vp.M[2] = f0 * (pr.Z * R[2] - pr.X * R[8]);
  vp.M[3] = f1 * (pr.Z * R[3] - pr.Y * R[6]);
  vp.M[4] = f1 * (pr.Z * R[4] - pr.Y * R[7]);
  vp.M[5] = f1 * (pr.Z * R[5] - pr.Y * R[8]);
  const size_t plane = (size_t)s.W * s.H;
  const T* th = (const T*)s.theta + plane * view;
  const T* cf = (const T*)s.conf + plane * view;
  const double x0 = floor(pr.u), y0 = floor(pr.v);
  const double fx = pr.u - x0, fy = pr.v - y0;
  const int ix = (int)x0 - HP, iy = (int)y0 - HP;
  // One patch row per pass (the loop is not unrolled: each sample takes
  // four sine/cosine evaluations), appended at the end of the arrays after
  // the earlier rows move up by one row, so that every array index is a
  // constant and the patch stays in registers (indexing by the row made it
  // a private array in memory).
  for (int b = 0; b < P; ++b) {
    double ra[P], rb[P], rc[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      double cb = 0.0, mx = 0.0, my = 0.0;
#pragma unroll
      for (int jy = 0; jy < 2; ++jy)
#pragma unroll
        for (int jx = 0; jx < 2; ++jx) {
          const double w = (jx ? fx : 1.0 - fx) * (jy ? fy : 1.0 - fy);
          const double t = tex_load_nb<T>(th, s.W, s.H, ix + a + jx, iy + b + jy);
          const double c = tex_load_nb<T>(cf, s.W, s.H, ix + a + jx, iy + b + jy);
          double sn, cs;
          sincos(2.0 * t, &sn, &cs);
          cb += w * c;
          mx += w * c * cs;
          my += w * c * sn;
        }
      const double n = sqrt(mx * mx + my * my);
      const double al = 0.5 * cb * cb;
      ra[a] = n > 0.0 ? al : 0.0;
      rb[a] = n > 0.0 ? al * mx / n : 0.0;
      rc[a] = n > 0.0 ? 2.0 * al * my / n : 0.0;
    }
#pragma unroll
    for (int k = 0; k < P2 - P; ++k) {
      vp.a[k] = vp.a[k + P];
      vp.b[k] = vp.b[k + P];
      vp.c[k] = vp.c[k + P];
    }
#pragma unroll
    for (int a = 0; a < P; ++a) {
      vp.a[P2 - P + a] = ra[a];
      vp.b[P2 - P + a] = rb[a];
      vp.c[P2 - P + a] = rc[a];
    }
  }
}

template <int P>
__device__ __forceinline__ double eval_patch64(const ViewPatch64<P>& vp, double dx, double dy,
                                               double dz) {
  constexpr int P2 = P * P;
  const double rx = __builtin_fma(vp.M[0], dx, __builtin_fma(vp.M[1], dy, vp.M[2] * dz));
  const double ry = __builtin_fma(vp.M[3], dx, __builtin_fma(vp.M[4], dy, vp.M[5] * dz));
  const double xx = rx * rx;
  const double n2 = __builtin_fma(ry, ry, xx);
  const bool on = n2 > 0.0;
  const double inv = 1.0 / (on ? n2 : 1.0);
  const double c2 = __builtin_fma(-ry, ry, xx) * inv;
  const double s2 = (rx * ry) * inv;
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < P2; ++k)
    m = fmax(m, __builtin_fma(vp.b[k], c2, __builtin_fma(vp.c[k], s2, vp.a[k])));
  return (on && m > 0.0) ? sqrt(m) : 0.0;
}

// max_p C_p |cos(phi(d) - theta_p)| for this lane's view (0 if the tangent
// projects to a point or the lane has no view), binary32: the lattice stage.
// With r = M d, n2 = |r|^2:
// C^2 cos^2(phi - theta) = a + b (rx^2 - ry^2)/n2 + c (rx ry)/n2, c = 2 gamma.
// For n2 = 0 the reciprocal is +inf, every q is NaN, fmaxf keeps the other
// operand, and the maximum stays 0.
template <int P>
__device__ __forceinline__ float eval_view(const ViewPatch<P>& vp, float dx, float dy,
                                           float dz) {
  constexpr int P2 = P * P;
  const float rx = __builtin_fmaf(vp.M[0], dx, __builtin_fmaf(vp.M[1], dy, vp.M[2] * dz));
  const float ry = __builtin_fmaf(vp.M[3], dx, __builtin_fmaf(vp.M[4], dy, vp.M[5] * dz));
  const float xx = rx * rx;
  const float inv = __builtin_amdgcn_rcpf(__builtin_fmaf(ry, ry, xx));
  const float c2 = __builtin_fmaf(-ry, ry, xx) * inv;
  const float s2 = (rx * ry) * inv;
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k + 1 < P2; k += 2) {
    const float q0 = __builtin_fmaf(vp.b[k], c2, __builtin_fmaf(vp.c[k], s2, vp.a[k]));
    const float q1 = __builtin_fmaf(vp.b[k + 1], c2, __builtin_fmaf(vp.c[k + 1], s2, vp.a[k + 1]));
    m = __builtin_fmaxf(__builtin_fmaxf(m, q0), q1);
  }
  if (P2 & 1) {
    const float q0 = __builtin_fmaf(vp.b[P2 - 1], c2, __builtin_fmaf(vp.c[P2 - 1], s2, vp.a[P2 - 1]));
    m = __builtin_fmaxf(m, q0);
  }
  return __builtin_amdgcn_sqrtf(m);
}

// The same in binary64 (the refinement): the coefficients are widened
// exactly, every operation is binary64, and a tangent that projects to a
// point gives 0.
template <int P>
__device__ __forceinline__ double eval_view64(const ViewPatch<P>& vp, double dx, double dy,
                                              double dz) {
  constexpr int P2 = P * P;
  const double rx = __builtin_fma((double)vp.M[0], dx,
                                  __builtin_fma((double)vp.M[1], dy, (double)vp.M[2] * dz));
  const double ry = __builtin_fma((double)vp.M[3], dx,
                                  __builtin_fma((double)vp.M[4], dy, (double)vp.M[5] * dz));
  const double xx = rx * rx;
  const double n2 = __builtin_fma(ry, ry, xx);
  const bool on = n2 > 0.0;
  const double inv = rcp64(on ? n2 : 1.0);
  const double c2 = __builtin_fma(-ry, ry, xx) * inv;
  const double s2 = (rx * ry) * inv;
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < P2; ++k) {
    const double qk = __builtin_fma((double)vp.b[k], c2,
                                    __builtin_fma((double)vp.c[k], s2, (double)vp.a[k]));
    m = fmax(m, qk);
  }
  return (on && m > 0.0) ? m * rsq64(m) : 0.0;
}

// Marks the patch coefficients as rewritten at this point (an empty asm
// statement on their registers; their values do not change), so that the
// widening of eval_view64 stays at the evaluation instead of being
// scheduled early, where 3 P^2 binary64 values would hold twice the
// registers of the binary32 patch through the whole refinement.
template <int P>
__device__ __forceinline__ void pin_patch(ViewPatch<P>& vp) {
#pragma unroll
  for (int k = 0; k < P * P; ++k) asm volatile("" : "+v"(vp.a[k]), "+v"(vp.b[k]), "+v"(vp.c[k]));
}

// Waves per SIMD the search kernels are compiled for: patches up to 5 x 5
// fit three waves' register share (168) with a few spilled bytes, which
// measures faster than two waves; 7 x 7 patches keep the compiler's choice.
#ifndef FD_SEARCH_WAVES
#define FD_SEARCH_WAVES 3
#endif
constexpr int search_waves(int P) { return P <= 5 ? FD_SEARCH_WAVES : 1; }

// Lane groups: the K lanes of one point.  With K known at compile time
// (KT > 0) the groups lie inside the wave's 16-lane rows (16 / K groups per
// row, the rest of the row idle: for K = 5 the same 12 groups per wave as
// packing them end to end), so that a group's view sum can be formed with
// row shifts (group_lead_sum); otherwise the groups are packed end to end.
// Idle lanes belong to no point (lane_ok false) but take part in the
// cross-lane operations of the last group of their row or wave.
struct Group {
  int K, G, g, slot, base;
  bool lane_ok;
};

template <int KT>
__device__ __forceinline__ Group make_group(int K) {
  Group gr;
  const int lane = threadIdx.x & (kWave - 1);
  gr.K = K;
  if constexpr (KT > 0) {
    constexpr int R = 16 / KT;
    static_assert(4 * R == kWave / KT, "as many groups per wave as the host's 64 / K");
    const int row = lane >> 4, r = lane & 15;
    const int gi = r / KT;
    gr.G = 4 * R;
    gr.lane_ok = gi < R;
    const int gc = gr.lane_ok ? gi : R - 1;
    gr.g = row * R + gc;
    gr.slot = r - gc * KT;
    gr.base = row * 16 + gc * KT;
  } else {
    gr.G = kWave / K;
    gr.g = lane / K;
    gr.slot = lane - gr.g * K;
    gr.lane_ok = gr.g < gr.G;
    gr.base = (gr.lane_ok ? gr.g : gr.G - 1) * K;
  }
  return gr;
}

// The group's sum of v, added in slot order (slot 0 first), exact only in
// the group's slot-0 lane: with row-aligned groups (KT > 0) that lane reads
// slot j through a row shift by j, which never leaves the row; otherwise
// every lane gets the sum.  A decision taken on it is passed to the rest of
// the group with lead_value.
// v of lane + J within the 16-lane row (DPP row_shl:J; 0 past the row's end).
template <int J>
__device__ __forceinline__ float row_shl(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + J, 0xf, 0xf,
                                                    true));
}

template <int KT, int J>
__device__ __forceinline__ float lead_sum_from(float s, float v) {
  if constexpr (J < KT)
    return lead_sum_from<KT, J + 1>(s + row_shl<J>(v), v);
  else
    return s;
}

template <int KT>
__device__ __forceinline__ float group_lead_sum(float v, int base, int k) {
  if constexpr (KT > 0) {
    static_assert(KT <= 16, "a group fits in a row");
    return lead_sum_from<KT, 1>(v, v);
  } else {
    return group_sum<float>(v, base, k);
  }
}

// x of lane - J within the 16-lane row (DPP row_shr:J; 0 before the row's start).
template <int J>
__device__ __forceinline__ int row_shr(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x110 + J, 0xf, 0xf, true);
}

template <int KT, int J>
__device__ __forceinline__ int lead_from(int x, int slot, int acc) {
  if constexpr (J <= KT) {
    // the shift is formed by every lane and only then selected: the empty
    // asm statement keeps the compiler from moving it under the selection,
    // where the lanes it reads from would be switched off
    int y = row_shr<J>(x);
    asm volatile("" : "+v"(y));
    return lead_from<KT, J + 1>(x, slot, slot == J ? y : acc);
  } else {
    return acc;
  }
}

// The value x of the group's slot-0 lane, in every lane of the group: with
// row-aligned groups lane slot reads it through a row shift by slot (the
// row's idle lanes, slots up to KT, follow the last group's lead).
template <int KT>
__device__ __forceinline__ int lead_value(int x, int slot) {
  if constexpr (KT > 0)
    return lead_from<KT, 1>(x, slot, x);
  else
    return x;
}

// Change of this lane's view term L_v = sqrt(max_p q_p) from the centre d
// of a refinement iteration to the candidate d + du (du the exact stencil
// offset), computed from differences so that binary32 rounding is relative
// to the change rather than to L_v itself.  With z = rx + i ry the image
// direction at d and dz = M du, e^{2 i phi} moves by
//   e^{2 i phi_d} * 2 i Im(eps) / conj(1 + eps),  eps = dz / z,
// the quadratic form of sample p by b_p dc2 + c_p ds2, and its patch value
// relative to the centre's maximum Q0 is v_p = g_p + b_p dc2 + c_p ds2 with
// g_p = q_p(d) - Q0; then L(d + du) - L(d) = V / (sqrt(Q0 + V) + sqrt(Q0)),
// V = max_p v_p.  A view whose centre direction projects to a point
// (|z| = 0, L(d) = 0) takes the candidate's own quadratic form instead
// (g_p = a_p, Q0 = 0); a candidate that projects to a point has L = 0.
struct ViewCentre {
  float zx, zy, iz2;  // z and 1 / |z|^2
  float ec, es;       // cos 2 phi_d, sin 2 phi_d
  float q0, l0;       // max_p q_p(d) and its square root
  bool on;            // |z| > 0
};

template <int P>
__device__ __forceinline__ ViewCentre view_centre(const ViewPatch<P>& vp, float dx, float dy,
                                                  float dz, float (&g)[P * P]) {
  constexpr int P2 = P * P;
  ViewCentre c;
  const float rx = __builtin_fmaf(vp.M[0], dx, __builtin_fmaf(vp.M[1], dy, vp.M[2] * dz));
  const float ry = __builtin_fmaf(vp.M[3], dx, __builtin_fmaf(vp.M[4], dy, vp.M[5] * dz));
  const float xx = rx * rx;
  const float n2 = __builtin_fmaf(ry, ry, xx);
  c.on = n2 > 0.0f;
  const float i2 = c.on ? __builtin_amdgcn_rcpf(n2) : 0.0f;
  // off (rx = ry = 0): c2 = s2 = 0, so q_p = a_p and, with m = 0 below,
  // g_p = a_p as the off case requires
  const float c2 = __builtin_fmaf(-ry, ry, xx) * i2, s2 = (rx * ry) * i2;
  c.zx = rx;
  c.zy = ry;
  c.iz2 = i2;
  c.ec = c2;
  c.es = 2.0f * s2;
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < P2; ++k) {
    g[k] = __builtin_fmaf(vp.b[k], c2, __builtin_fmaf(vp.c[k], s2, vp.a[k]));
    m = __builtin_fmaxf(m, g[k]);
  }
  m = c.on ? m : 0.0f;
#pragma unroll
  for (int k = 0; k < P2; ++k) g[k] -= m;
  c.q0 = m;
  c.l0 = __builtin_amdgcn_sqrtf(m);
  return c;
}

// The stencil's image offsets relative to the centre: with e1, e2 the
// basis and z = M d, a candidate's dz = M du = (cos a - 1) z + sin a
// (cos j M e1 + sin j M e2), so eps = dz / z = (cos a - 1) + sin a (cos j
// A1 + sin j A2) + i sin a (cos j B1 + sin j B2) with A_k + i B_k =
// M e_k / z, formed once per iteration.
struct StencilFrame {
  float a1, a2, b1, b2;  // sin a times A_k and B_k
  float m1x, m1y, m2x, m2y;  // sin a times M e_k (off-centre views)
};

template <int P>
__device__ __forceinline__ StencilFrame stencil_frame(const ViewPatch<P>& vp, const ViewCentre& c,
                                                      float sa, float e1x, float e1y, float e1z,
                                                      float e2x, float e2y, float e2z) {
  StencilFrame f;
  const float p1x = __builtin_fmaf(vp.M[0], e1x, __builtin_fmaf(vp.M[1], e1y, vp.M[2] * e1z));
  const float p1y = __builtin_fmaf(vp.M[3], e1x, __builtin_fmaf(vp.M[4], e1y, vp.M[5] * e1z));
  const float p2x = __builtin_fmaf(vp.M[0], e2x, __builtin_fmaf(vp.M[1], e2y, vp.M[2] * e2z));
  const float p2y = __builtin_fmaf(vp.M[3], e2x, __builtin_fmaf(vp.M[4], e2y, vp.M[5] * e2z));
  f.m1x = sa * p1x;
  f.m1y = sa * p1y;
  f.m2x = sa * p2x;
  f.m2y = sa * p2y;
  const float si = sa * c.iz2;
  f.a1 = (p1x * c.zx + p1y * c.zy) * si;
  f.b1 = (p1y * c.zx - p1x * c.zy) * si;
  f.a2 = (p2x * c.zx + p2y * c.zy) * si;
  f.b2 = (p2y * c.zx - p2x * c.zy) * si;
  return f;
}

template <int P>
__device__ __forceinline__ float view_delta(const ViewPatch<P>& vp, const float (&g)[P * P],
                                            const ViewCentre& c, const StencilFrame& f,
                                            bool any_off, float cm1, float cj, float sj) {
  constexpr int P2 = P * P;
  // centred form: eps = er + i ei
  const float er = __builtin_fmaf(cj, f.a1, __builtin_fmaf(sj, f.a2, cm1));
  const float ei = __builtin_fmaf(cj, f.b1, sj * f.b2);
  const float opr = 1.0f + er;
  const float D = __builtin_fmaf(opr, opr, ei * ei);
  const float iD = __builtin_amdgcn_rcpf(D);
  const float dre = -2.0f * ei * ei * iD, dim = 2.0f * ei * opr * iD;
  float dc2 = c.ec * dre - c.es * dim;
  float ds2 = 0.5f * (c.ec * dim + c.es * dre);
  bool cand_on = D > 0.0f;
  if (any_off) {  // wave-uniform: some lane's centre direction projects to a point
    // (z = 0 there, so dz is the stencil part alone)
    const float Dx = __builtin_fmaf(cj, f.m1x, sj * f.m2x);
    const float Dy = __builtin_fmaf(cj, f.m1y, sj * f.m2y);
    const float xx = Dx * Dx, n2 = __builtin_fmaf(Dy, Dy, xx);
    const float inv = __builtin_amdgcn_rcpf(n2);
    dc2 = c.on ? dc2 : __builtin_fmaf(-Dy, Dy, xx) * inv;
    ds2 = c.on ? ds2 : (Dx * Dy) * inv;
    cand_on = c.on ? cand_on : n2 > 0.0f;
  }
  float V = -INFINITY;
#pragma unroll
  for (int k = 0; k + 1 < P2; k += 2) {
    const float v0 = __builtin_fmaf(vp.b[k], dc2, __builtin_fmaf(vp.c[k], ds2, g[k]));
    const float v1 = __builtin_fmaf(vp.b[k + 1], dc2, __builtin_fmaf(vp.c[k + 1], ds2, g[k + 1]));
    V = __builtin_fmaxf(__builtin_fmaxf(V, v0), v1);
  }
  if (P2 & 1) {
    const float v0 = __builtin_fmaf(vp.b[P2 - 1], dc2, __builtin_fmaf(vp.c[P2 - 1], ds2, g[P2 - 1]));
    V = __builtin_fmaxf(V, v0);
  }
  V = __builtin_fmaxf(V, -c.q0);  // q >= 0
  const float den = __builtin_amdgcn_sqrtf(c.q0 + V) + c.l0;
  const float dl = den > 0.0f ? V * __builtin_amdgcn_rcpf(den) : 0.0f;
  return cand_on ? dl : -c.l0;
}

// Pattern search (six directions at angle alpha_t around d in the
// orthonormal basis of Duff et al. 2017, stencil angles j pi / 3, the best
// strictly-better one taken, first of equals; alpha halves every iteration).
// Each candidate d + du (du = (cos alpha - 1) d + sin alpha (cos j e1 +
// sin j e2), the exact offset of the unit candidate) is compared with the
// centre through the change of the view sum (view_delta), so the decisions
// carry binary32 rounding relative to the cost differences the iteration
// compares, not to the cost; the rounding of the centre and of the basis
// only moves the stencil by ~1e-7 of its size.  cs holds cos alpha_t,
// sin alpha_t and cos alpha_t - 1 (FD_MAX_REFINE entries each).  The six
// changes of an iteration are formed first and then summed over the group,
// so that their cross-lane reads are in flight together.
//
// Stencil cosines and sines: the binary32 roundings of the binary64 values
// of cos(j pi / 3) and sin(j pi / 3) (sin pi rounds to 1.2246468e-16, not 0).
constexpr float kStencilC[6] = {1.0f, 0.5f, -0.5f, -1.0f, -0.5f, 0.5f};
constexpr float kStencilS[6] = {0.0f, 0.866025403784438597f, 0.866025403784438597f,
                                1.22464679914735321e-16f, -0.866025403784438597f,
                                -0.866025403784438597f};

template <int P, int KT>
__device__ __forceinline__ void refine(const ViewPatch<P>& vp, const Group& gr, int iters,
                                       const double* __restrict__ cs, float& dx, float& dy,
                                       float& dz) {
  for (int t = 0; t < iters; ++t) {
    const float sg = copysignf(1.0f, dz);
    const float aa = -__builtin_amdgcn_rcpf(sg + dz);  // |sg + dz| >= 1
    const float bb = dx * dy * aa;
    const float e1x = 1.0f + sg * dx * dx * aa, e1y = sg * bb, e1z = -sg * dx;
    const float e2x = bb, e2y = sg + dy * dy * aa, e2z = -dy;
    float g[P * P];
    const ViewCentre c = view_centre<P>(vp, dx, dy, dz, g);
    const bool any_off = __ballot(!c.on) != 0;
    const float sa = (float)cs[FD_MAX_REFINE + t], cm1 = (float)cs[2 * FD_MAX_REFINE + t];
    const StencilFrame f = stencil_frame<P>(vp, c, sa, e1x, e1y, e1z, e2x, e2y, e2z);
    float dl[6];
#pragma unroll
    for (int jj = 0; jj < 6; ++jj)
      dl[jj] = view_delta<P>(vp, g, c, f, any_off, cm1, kStencilC[jj], kStencilS[jj]);
    float bS = -INFINITY;
    int bj = 0;
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
      const float dS = group_lead_sum<KT>(dl[jj], gr.base, gr.K);
      if (dS > bS) {
        bS = dS;
        bj = jj;
      }
    }
    // the slot-0 lane's decision, in every lane of the group
    bj = lead_value<KT>(bS > 0.0f ? bj : -1, gr.slot);
    if (bj >= 0) {
      float cj = kStencilC[0], sj = kStencilS[0];
#pragma unroll
      for (int jj = 1; jj < 6; ++jj) {
        cj = bj == jj ? kStencilC[jj] : cj;
        sj = bj == jj ? kStencilS[jj] : sj;
      }
      const float ux = __builtin_fmaf(cm1, dx, sa * (cj * e1x + sj * e2x));
      const float uy = __builtin_fmaf(cm1, dy, sa * (cj * e1y + sj * e2y));
      const float uz = __builtin_fmaf(cm1, dz, sa * (cj * e1z + sj * e2z));
      const float nx = dx + ux, ny = dy + uy, nz = dz + uz;
      const float il = __builtin_amdgcn_rsqf(__builtin_fmaf(nx, nx, __builtin_fmaf(ny, ny, nz * nz)));
      dx = nx * il;
      dy = ny * il;
      dz = nz * il;
    }
  }
}

// Output: d and -d are the same line; the representative has z > 0, else
// y > 0, else x >= 0.  cost J = 1 - S / K_eff.
__device__ __forceinline__ void write_result(const SceneDev& s, uint32_t i, double dx, double dy,
                                             double dz, double J) {
  const bool flip = dz != 0.0 ? dz < 0.0 : (dy != 0.0 ? dy < 0.0 : dx < 0.0);
  const double sgn = flip ? -1.0 : 1.0;
  s.dirs[3 * (size_t)i] = (float)(sgn * dx);
  s.dirs[3 * (size_t)i + 1] = (float)(sgn * dy);
  s.dirs[3 * (size_t)i + 2] = (float)(sgn * dz);
  s.costs[i] = (float)J;
}

__device__ __forceinline__ double cost_of(double S, int keff) {
  return keff > 0 ? 1.0 - S / (double)keff : INFINITY;
}

// ---- plain search of one point per lane group ---------------------------------
// Eq. (12) lattice argmin of J (= argmax of the view sum, first of equals),
// then the pattern-search refinement, on the group's patch registers.
// Returns the direction in (dx, dy, dz) and the binary64 view sum in S.
template <int P, int KT>
__device__ __forceinline__ void full_search(ViewPatch<P>& vp, const SearchDev& q,
                                            const Group& gr, double& dx, double& dy, double& dz,
                                            double& S) {
  float Sb = -INFINITY;
  int kb = 0;
  // two candidates per pass (by hand: the group sum's cross-lane reads keep
  // the compiler from unrolling), taken in order so that the first of equals
  // still wins
  int k = 0;
  for (; k + 1 < q.n_candidates; k += 2) {
    const float* c = q.lattice + 3 * k;
    const float S0 = group_lead_sum<KT>(eval_view<P>(vp, c[0], c[1], c[2]), gr.base, gr.K);
    const float S1 = group_lead_sum<KT>(eval_view<P>(vp, c[3], c[4], c[5]), gr.base, gr.K);
    if (S0 > Sb) {
      Sb = S0;
      kb = k;
    }
    if (S1 > Sb) {
      Sb = S1;
      kb = k + 1;
    }
  }
  if (k < q.n_candidates) {
    const float* c = q.lattice + 3 * k;
    const float Sk = group_lead_sum<KT>(eval_view<P>(vp, c[0], c[1], c[2]), gr.base, gr.K);
    if (Sk > Sb) {
      Sb = Sk;
      kb = k;
    }
  }
  kb = lead_value<KT>(kb, gr.slot);
  float fx = q.lattice[3 * kb], fy = q.lattice[3 * kb + 1], fz = q.lattice[3 * kb + 2];
  refine<P, KT>(vp, gr, q.refine_iters, q.steps, fx, fy, fz);
  dx = fx;
  dy = fy;
  dz = fz;
  pin_patch<P>(vp);
  S = group_sum_t<KT>(eval_view64<P>(vp, dx, dy, dz), gr.base, gr.K);
}

// The K lanes of the caller's group fuse processing-order point j of scene s
// (pt_ok false: the group has no point but still takes part in the shuffles).
template <typename T, int P, int KT>
__device__ __forceinline__ void fuse_group(const SceneDev& s, const SearchDev& q, const Group& gr,
                                           bool pt_ok, int64_t j) {
  const uint32_t i = pt_ok ? s.perm[j] : 0u;
  const int keff = pt_ok ? (int)s.kcount[j] : 0;
  const bool slot_ok = pt_ok && gr.slot < keff;
  const int view = slot_ok ? (int)s.views[FD_TOPK_SLOTS * j + gr.slot] : 0;
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  ViewPatch<P> vp;
  build_patch<T, P>(s, q, view, slot_ok, px, py, pz, vp);
  double dx, dy, dz, S;
  full_search<P, KT>(vp, q, gr, dx, dy, dz, S);
  if (pt_ok && gr.slot == 0) {
    if (keff == 0)
      write_result(s, i, 0.0, 0.0, 0.0, INFINITY);
    else
      write_result(s, i, dx, dy, dz, cost_of(S, keff));
  }
}

// ---- learned form: refinement from a proposal, threshold, fallback -------------
// Proposals (x, y, z): l.proposals row prop_base + j when prop_by_j, else
// row i (the point index); without l.proposals, the scene's own s.prop row
// i; with neither, every proposal is invalid.  A point is kept when its proposal
// is a finite non-zero direction and the refined cost satisfies J <= tau;
// otherwise it takes the plain search.  A wave in which at least half of its
// points need the plain search runs it at once on the patch registers it
// already holds (l.fb_count[1] counts those points); otherwise the points
// that need it are appended as list_base + j to the fallback list
// (l.fb_count[0] entries) for a later plain-search launch.  Either way a
// point's result is the plain search's.  The proposal is normalised, refined
// and compared with tau in binary64.
template <typename T, int P, int KT>
__device__ __forceinline__ void learned_group(const SceneDev& s, const SearchDev& q,
                                              const LearnedDev& l, const Group& gr, bool pt_ok,
                                              int64_t j, int prop_by_j, int64_t prop_base,
                                              int64_t list_base) {
  const uint32_t i = pt_ok ? s.perm[j] : 0u;
  const int keff = pt_ok ? (int)s.kcount[j] : 0;
  const bool slot_ok = pt_ok && gr.slot < keff;
  const int view = slot_ok ? (int)s.views[FD_TOPK_SLOTS * j + gr.slot] : 0;
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  ViewPatch<P> vp;
  build_patch<T, P>(s, q, view, slot_ok, px, py, pz, vp);
  double dx = 0.0, dy = 0.0, dz = 0.0;
  const float* pp = nullptr;
  if (pt_ok) {
    if (l.proposals)
      pp = l.proposals + 3 * (size_t)(prop_by_j ? (uint64_t)(prop_base + j) : (uint64_t)i);
    else if (s.prop)
      pp = s.prop + 3 * (size_t)i;
  }
  if (pp) {
    dx = pp[0];
    dy = pp[1];
    dz = pp[2];
  }
  const double len = sqrt(dx * dx + dy * dy + dz * dz);
  const bool valid = keff > 0 && isfinite(len) && len > 0.0;
  float fx = valid ? (float)(dx / len) : 0.0f;
  float fy = valid ? (float)(dy / len) : 0.0f;
  float fz = valid ? (float)(dz / len) : 1.0f;
  refine<P, KT>(vp, gr, l.iters, l.steps, fx, fy, fz);
  dx = fx;
  dy = fy;
  dz = fz;
  pin_patch<P>(vp);
  const double S = group_sum_t<KT>(eval_view64<P>(vp, dx, dy, dz), gr.base, gr.K);
  const double J = cost_of(S, keff);
  const bool keep = valid && J <= l.tau;
  const bool lead = pt_ok && gr.slot == 0;
  if (lead && keep) write_result(s, i, dx, dy, dz, J);
  // the same decision in every lane of the wave
  const int n_pts = __popcll(__ballot(lead));
  const int n_need = __popcll(__ballot(lead && !keep));
  if (n_need == 0) return;
  if (2 * n_need >= n_pts) {
    double fx, fy, fz, fS;
    full_search<P, KT>(vp, q, gr, fx, fy, fz, fS);
    if (lead && !keep) {
      if (keff == 0)
        write_result(s, i, 0.0, 0.0, 0.0, INFINITY);
      else
        write_result(s, i, fx, fy, fz, cost_of(fS, keff));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&l.fb_count[1], (uint32_t)n_need);
  } else if (lead && !keep) {
    const uint32_t pos = atomicAdd(&l.fb_count[0], 1u);
    l.fb_list[pos] = (uint32_t)(list_base + j);
  }
}

// ---- paper-literal candidates: Sec. 3.1.1-3.1.2 (Eqs. 1-7), scored by Eq. (12) ----
// Lane = one view of Eq. (4).  The lane's view gives S candidates: the
// projection u moved by lambda pixels along the observed orientation (the
// patch's centre sample), the depth texel nearest to that pixel shifted by
// delta_s in [-delta, delta], back-projected and taken relative to the point
// (unit).  Per layer s the group fuses the confidence-weighted medoid of its
// lanes' candidates (same fixed order in every lane, so every lane takes the
// same one), and the fused candidate with the largest view sum (lowest J,
// first of equals) is the result.  Positions, candidates, the medoid
// weights, the patch and its score are binary64.
template <typename T, int P, int KT>
__device__ __forceinline__ void fpmvo_group(const SceneDev& s, const SearchDev& q,
                                            const FpmvoDev& f, const Group& gr, bool pt_ok,
                                            int64_t j) {
  const uint32_t i = pt_ok ? s.perm[j] : 0u;
  const int keff = pt_ok ? (int)s.kcount[j] : 0;
  const bool slot_ok = pt_ok && gr.slot < keff;
  const int view = slot_ok ? (int)s.views[FD_TOPK_SLOTS * j + gr.slot] : 0;
  const double px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
               pz = s.pts[3 * (size_t)i + 2];
  ViewPatch64<P> vp;
  build_patch64<T, P>(s, q, view, slot_ok, px, py, pz, vp);

  // Eq. (1): the orientation t of the centre sample (the bilinear,
  // confidence-weighted doubled-angle mean at u, recomputed here in binary64:
  // it places the offset pixel, a discrete choice) and the unit offset
  // (cos t, sin t), t in (-pi/2, pi/2]; the centre confidence is the medoid
  // weight of Eq. (6)
  const float* cam = s.cams + 16 * view;
  Proj pr;
  const bool in_view = slot_ok && project64(cam, px, py, pz, s.W, s.H, q.z_near, pr);
  double w = 0.0, ct = 1.0, st = 0.0;
  bool vok = false;
  if (in_view) {
    const size_t plane = (size_t)s.W * s.H;
    const T* thm = (const T*)s.theta + plane * view;
    const T* cfm = (const T*)s.conf + plane * view;
    const double x0 = floor(pr.u), y0 = floor(pr.v);
    const double fx = pr.u - x0, fy = pr.v - y0;
    const int ix = (int)x0, iy = (int)y0;
    double mx = 0.0, my = 0.0;
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const double wt = (a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy);
        const double th = tex_load_nb<T>(thm, s.W, s.H, ix + a, iy + b);
        const double c = tex_load_nb<T>(cfm, s.W, s.H, ix + a, iy + b);
        w += wt * c;
        mx += wt * c * cos(2.0 * th);
        my += wt * c * sin(2.0 * th);
      }
    vok = sqrt(mx * mx + my * my) > 0.0;
    const double t = 0.5 * atan2(my, mx);
    ct = cos(t);
    st = sin(t);
  }
  const double ux = (in_view ? pr.u : 0.0) + (double)f.lambda * ct;
  const double uy = (in_view ? pr.v : 0.0) + (double)f.lambda * st;
  vok = vok && ux >= 0.0 && ux <= (double)(s.W - 1) && uy >= 0.0 && uy <= (double)(s.H - 1);
  // Eq. (2): depth at the nearest texel of the offset pixel
  double D = 0.0;
  if (vok) {
    const uint32_t xn = (uint32_t)floor(ux + 0.5), yn = (uint32_t)floor(uy + 0.5);
    D = ld_texel<T>((const T*)s.depth + (size_t)s.W * s.H * view, yn * (uint32_t)s.W + xn);
  }
  vok = vok && isfinite(D);
  // Eq. (3): p_s = R^T (X_c - t) with X_c = z_s ((ux - cx)/fx, (uy - cy)/fy, 1)
  const float* R = cam + 4;
  const float* tc = cam + 13;
  const double S1 = f.samples > 1 ? (double)(f.samples - 1) : 1.0;

  double Sb = -INFINITY, bxd = 0.0, byd = 0.0, bzd = 0.0;
  for (int sl = 0; sl < f.samples; ++sl) {
    const double zs =
        D + (f.samples > 1 ? -(double)f.delta + 2.0 * (double)f.delta * (double)sl / S1 : 0.0);
    const double xc0 = (ux - (double)cam[2]) * zs / (double)cam[0] - (double)tc[0];
    const double xc1 = (uy - (double)cam[3]) * zs / (double)cam[1] - (double)tc[1];
    const double xc2 = zs - (double)tc[2];
    double dx = (double)R[0] * xc0 + (double)R[3] * xc1 + (double)R[6] * xc2 - px;
    double dy = (double)R[1] * xc0 + (double)R[4] * xc1 + (double)R[7] * xc2 - py;
    double dz = (double)R[2] * xc0 + (double)R[5] * xc1 + (double)R[8] * xc2 - pz;
    const double n = sqrt(dx * dx + dy * dy + dz * dz);
    const bool ok = vok && zs > 0.0 && n > 0.0;
    // a lane without a candidate shares exact zeros (its depth may be +inf)
    dx = ok ? dx / n : 0.0;
    dy = ok ? dy / n : 0.0;
    dz = ok ? dz / n : 0.0;
    // Eqs. (5)-(6): weighted consistency of this lane's candidate with the
    // group's candidates of the same layer (views in the order of Eq. (4))
    const double wk = ok ? w : 0.0;
    double num = 0.0, den = 0.0;
    const int K = KT > 0 ? KT : gr.K;
    for (int jj = 0; jj < K; ++jj) {
      const int src = gr.base + jj;
      const double xj = __shfl(dx, src, kWave), yj = __shfl(dy, src, kWave),
                   zj = __shfl(dz, src, kWave), wj = __shfl(wk, src, kWave);
      // G_ii = 1 exactly for a unit direction
      num += jj == gr.slot ? wj : wj * fabs(dx * xj + dy * yj + dz * zj);
      den += wj;
    }
    const double sigma = ok ? num / den : -INFINITY;
    // Eq. (7): the medoid, first of equals
    int bj = -1;
    double bs = -INFINITY;
    for (int jj = 0; jj < K; ++jj) {
      const double sj = __shfl(sigma, gr.base + jj, kWave);
      if (sj > bs) {
        bs = sj;
        bj = jj;
      }
    }
    // the same in every lane of the group; the shuffles below run in every lane
    const int src = gr.base + (bj < 0 ? 0 : bj);
    const double fx = __shfl(dx, src, kWave), fy = __shfl(dy, src, kWave),
                 fz = __shfl(dz, src, kWave);
    // Eq. (12): patch consistency of the fused candidate
    const double Sv = group_sum_t<KT>(eval_patch64<P>(vp, fx, fy, fz), gr.base, gr.K);
    if (bj >= 0 && Sv > Sb) {
      Sb = Sv;
      bxd = fx;
      byd = fy;
      bzd = fz;
    }
  }
  if (pt_ok && gr.slot == 0) {
    if (keff == 0 || !(Sb > -INFINITY))
      write_result(s, i, 0.0, 0.0, 0.0, INFINITY);
    else
      write_result(s, i, bxd, byd, bzd, cost_of(Sb, keff));
  }
}

}  // namespace fd
