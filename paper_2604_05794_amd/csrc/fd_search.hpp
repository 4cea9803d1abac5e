// fd_search.hpp -- per-point device code of the direction search, shared by
// the single-scene kernels (fd_fuse.hip) and the batched ones
// (fd_batched.hip).  EfficientMonoHair, Sec. 3.1: Eq. (4) view selection,
// Eqs. (8)-(11) objective, Eq. (12) best candidate, pattern-search
// refinement.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fd_device.hpp"
#include "fd_kernels.hpp"

namespace fd {

constexpr float kInvPi = 0.318309886183790671538f;

// ---- Eq. (4): top-K views by centre confidence ------------------------------
// One lane per point (processing-order index j).  Stable insertion into a
// register list of KS >= K slots: a view enters ahead of a listed one only if
// strictly more confident, so equal confidences keep the lower view index
// first.  Slots 0..KS-1 of the point's view row are written.
template <int KS>
__device__ __forceinline__ void topk_insert(float (&sc)[KS], int (&id)[KS], float c, int v) {
  float cs = c;
  int cv = v;
  bool ins = false;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const bool take = ins || (cs > sc[k]);
    const float ts = sc[k];
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
  const float px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
              pz = s.pts[3 * (size_t)i + 2];
  float sc[KS];
  int id[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    sc[k] = -1.0f;
    id[k] = 0;
  }
  const T* conf = (const T*)s.conf;
  const T* depth = (const T*)s.depth;
  const size_t plane = (size_t)s.W * s.H;
  // Views in groups of four.  Projections and depth texels of a group are
  // issued together; a view that no lane of the wave sees (all hidden, behind
  // or outside, common for the far side of a head) skips its confidence
  // texels and insertion.  The confidence loads of the seen views are issued
  // before any of them is used.
  constexpr int kGroup = 4;
  for (int v0 = 0; v0 < s.V; v0 += kGroup) {
    Proj pr[kGroup];
    bool seen[kGroup];
#pragma unroll
    for (int u = 0; u < kGroup; ++u) {
      const int v = min(v0 + u, s.V - 1);
      const bool ok = project32(s.cams + 16 * v, px, py, pz, s.W, s.H, q.z_near, pr[u]);
      seen[u] = visible_at<T>(depth ? depth + plane * v : nullptr, s.W, ok, pr[u], s.vis_tau) &&
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
      const float c = seen[u] ? conf_combine(tx[u]) : 0.0f;
      if (c > 0.0f) topk_insert<KS>(sc, id, c, v0 + u);
    }
  }
  int keff = 0;
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    if (k < q.K && sc[k] > 0.0f) keff = k + 1;
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
template <typename T, int P>
__device__ __forceinline__ void build_patch(const SceneDev& s, const SearchDev& q, int view,
                                            bool active, float px, float py, float pz,
                                            ViewPatch<P>& vp) {
  constexpr int P2 = P * P, HP = (P - 1) / 2;
#pragma unroll
  for (int k = 0; k < P2; ++k) vp.a[k] = vp.b[k] = vp.c[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < 6; ++k) vp.M[k] = 0.0f;
  if (!active) return;
  const float* cam = s.cams + 16 * view;
  Proj pr;
  project32(cam, px, py, pz, s.W, s.H, q.z_near, pr);
  // r = J_pi d up to the positive factor 1/Z^2:
  //   r_x = fx (Z (R0 . d) - X (R2 . d)),  r_y = fy (Z (R1 . d) - Y (R2 . d))
  const float* R = cam + 4;
  vp.M[0] = cam[0] * (pr.Z * R[0] - pr.X * R[6]);
  vp.M[1] = cam[0] * (pr.Z * R[1] - pr.X * R[7]);
  vp.M[2] = cam[0] * (pr.Z * R[2] - pr.X * R[8]);
  vp.M[3] = cam[1] * (pr.Z * R[3] - pr.Y * R[6]);
  vp.M[4] = cam[1] * (pr.Z * R[4] - pr.Y * R[7]);
  vp.M[5] = cam[1] * (pr.Z * R[5] - pr.Y * R[8]);

  const size_t plane = (size_t)s.W * s.H;
  const T* th = (const T*)s.theta + plane * view;
  const T* cf = (const T*)s.conf + plane * view;
  const float x0 = floorf(pr.u), y0 = floorf(pr.v);
  const float fx = pr.u - x0, fy = pr.v - y0;
  const float gx = 1.0f - fx, gy = 1.0f - fy;
  const float w00 = gx * gy, w10 = fx * gy, w01 = gx * fy, w11 = fx * fy;
  const int ix = (int)x0 - HP, iy = (int)y0 - HP;
  // texel rows of the (P+1)^2 footprint: C, C cos 2theta, C sin 2theta
  float rc[2][P + 1], rx[2][P + 1], ry[2][P + 1];
  // binary16 rows away from the right edge of an even-width map: one 16-byte
  // load per map covers texels [ix & ~1, (ix & ~1) + 7] of the row
  const bool wide_ok = sizeof(T) == 2 && P <= 5 && (s.W & 1) == 0;
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
      const float turns = tv[a] * kInvPi;  // 2 theta in revolutions
      rc[slot][a] = cv[a];
      rx[slot][a] = cv[a] * __builtin_amdgcn_cosf(turns);
      ry[slot][a] = cv[a] * __builtin_amdgcn_sinf(turns);
    }
  };
  load_row(0, iy);
#pragma unroll
  for (int b = 0; b < P; ++b) {
    const int r0 = b & 1, r1 = (b + 1) & 1;
    load_row(r1, iy + b + 1);
#pragma unroll
    for (int a = 0; a < P; ++a) {
      float cb = w00 * rc[r0][a] + w10 * rc[r0][a + 1] + w01 * rc[r1][a] + w11 * rc[r1][a + 1];
      float mx = w00 * rx[r0][a] + w10 * rx[r0][a + 1] + w01 * rx[r1][a] + w11 * rx[r1][a + 1];
      float my = w00 * ry[r0][a] + w10 * ry[r0][a + 1] + w01 * ry[r1][a] + w11 * ry[r1][a + 1];
      float n2 = mx * mx + my * my;
      float al = 0.5f * cb * cb;
      float inv = n2 > 0.0f ? __builtin_amdgcn_rsqf(n2) : 0.0f;
      const int k = b * P + a;
      vp.a[k] = n2 > 0.0f ? al : 0.0f;
      vp.b[k] = al * mx * inv;
      vp.c[k] = 2.0f * al * my * inv;  // the factor 2 of 2 rx ry folded in
    }
  }
}

// max_p C_p |cos(phi(d) - theta_p)| for this lane's view (0 if the tangent
// projects to a point or the lane has no view).  With r = M d, n2 = |r|^2:
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

struct Group {
  int K, G, g, slot, base;
  bool lane_ok;
};

__device__ __forceinline__ Group make_group(int K) {
  Group gr;
  const int lane = threadIdx.x & (kWave - 1);
  gr.K = K;
  gr.G = kWave / K;
  gr.g = lane / K;
  gr.slot = lane - gr.g * K;
  gr.lane_ok = gr.g < gr.G;
  gr.base = (gr.lane_ok ? gr.g : gr.G - 1) * K;
  return gr;
}

// Pattern search (six directions at angle alpha around d in the basis of
// Duff et al. 2017, best strictly-better one taken, alpha halves).  Works on
// the view sum S = sum_v L_v (J = 1 - S / K_eff), larger is better.
template <int P, int KT>
__device__ __forceinline__ void refine(const ViewPatch<P>& vp, const Group& gr, int iters,
                                       float alpha, float& dx, float& dy, float& dz, float& Sd) {
  const float cj[6] = {1.0f, 0.5f, -0.5f, -1.0f, -0.5f, 0.5f};
  const float sj[6] = {0.0f, 0.86602540378443865f, 0.86602540378443865f, 0.0f,
                       -0.86602540378443865f, -0.86602540378443865f};
  for (int t = 0; t < iters; ++t) {
    const float sg = copysignf(1.0f, dz);
    const float aa = -1.0f / (sg + dz);
    const float bb = dx * dy * aa;
    const float e1x = 1.0f + sg * dx * dx * aa, e1y = sg * bb, e1z = -sg * dx;
    const float e2x = bb, e2y = sg + dy * dy * aa, e2z = -dy;
    const float ca = cosf(alpha), sa = sinf(alpha);
    float bS = -INFINITY, bx = dx, by = dy, bz = dz;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float ux = ca * dx + sa * (cj[j] * e1x + sj[j] * e2x);
      float uy = ca * dy + sa * (cj[j] * e1y + sj[j] * e2y);
      float uz = ca * dz + sa * (cj[j] * e1z + sj[j] * e2z);
      const float il = __builtin_amdgcn_rsqf(ux * ux + uy * uy + uz * uz);
      ux *= il;
      uy *= il;
      uz *= il;
      const float S = group_sum_t<KT>(eval_view<P>(vp, ux, uy, uz), gr.base, gr.K);
      if (S > bS) {
        bS = S;
        bx = ux;
        by = uy;
        bz = uz;
      }
    }
    if (bS > Sd) {
      Sd = bS;
      dx = bx;
      dy = by;
      dz = bz;
    }
    alpha *= 0.5f;
  }
}

__device__ __forceinline__ void write_result(const SceneDev& s, uint32_t i, float dx, float dy,
                                             float dz, float J) {
  const bool flip = dz != 0.0f ? dz < 0.0f : (dy != 0.0f ? dy < 0.0f : dx < 0.0f);
  const float sgn = flip ? -1.0f : 1.0f;
  s.dirs[3 * (size_t)i] = sgn * dx;
  s.dirs[3 * (size_t)i + 1] = sgn * dy;
  s.dirs[3 * (size_t)i + 2] = sgn * dz;
  s.costs[i] = J;
}

// ---- plain search of one point per lane group ---------------------------------
// Eq. (12) lattice argmin of J (= argmax of the view sum, first of equals),
// then the pattern-search refinement, on the group's patch registers.
// Returns the direction in (dx, dy, dz) and the view sum in S.
template <int P, int KT>
__device__ __forceinline__ void full_search(const ViewPatch<P>& vp, const SearchDev& q,
                                            const Group& gr, float& dx, float& dy, float& dz,
                                            float& S) {
  float Sb = -INFINITY;
  int kb = 0;
  // two candidates per pass (by hand: the group sum's cross-lane reads keep
  // the compiler from unrolling), taken in order so that the first of equals
  // still wins
  int k = 0;
  for (; k + 1 < q.n_candidates; k += 2) {
    const float* c = q.lattice + 3 * k;
    const float S0 = group_sum_t<KT>(eval_view<P>(vp, c[0], c[1], c[2]), gr.base, gr.K);
    const float S1 = group_sum_t<KT>(eval_view<P>(vp, c[3], c[4], c[5]), gr.base, gr.K);
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
    const float Sk = group_sum_t<KT>(eval_view<P>(vp, c[0], c[1], c[2]), gr.base, gr.K);
    if (Sk > Sb) {
      Sb = Sk;
      kb = k;
    }
  }
  dx = q.lattice[3 * kb];
  dy = q.lattice[3 * kb + 1];
  dz = q.lattice[3 * kb + 2];
  refine<P, KT>(vp, gr, q.refine_iters, q.step0, dx, dy, dz, Sb);
  S = Sb;
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
  const float px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
              pz = s.pts[3 * (size_t)i + 2];
  ViewPatch<P> vp;
  build_patch<T, P>(s, q, view, slot_ok, px, py, pz, vp);
  const float kinv = keff > 0 ? 1.0f / (float)keff : 0.0f;
  float dx, dy, dz, S;
  full_search<P, KT>(vp, q, gr, dx, dy, dz, S);
  if (pt_ok && gr.slot == 0) {
    if (keff == 0)
      write_result(s, i, 0.0f, 0.0f, 0.0f, INFINITY);
    else
      write_result(s, i, dx, dy, dz, 1.0f - S * kinv);
  }
}

// ---- learned form: refinement from a proposal, threshold, fallback -------------
// prop: proposals (x, y, z); row prop_base + j when prop_by_j, else the point
// index i; NULL = every proposal invalid.  A point is kept when its proposal
// is a finite non-zero direction and the refined cost satisfies J <= tau;
// otherwise it takes the plain search.  A wave in which at least half of its
// points need the plain search runs it at once on the patch registers it
// already holds (l.fb_count[1] counts those points); otherwise the points
// that need it are appended as list_base + j to the fallback list
// (l.fb_count[0] entries) for a later plain-search launch.  Either way a
// point's result is the plain search's.
template <typename T, int P, int KT>
__device__ __forceinline__ void learned_group(const SceneDev& s, const SearchDev& q,
                                              const LearnedDev& l, const Group& gr, bool pt_ok,
                                              int64_t j, int prop_by_j, int64_t prop_base,
                                              int64_t list_base) {
  const uint32_t i = pt_ok ? s.perm[j] : 0u;
  const int keff = pt_ok ? (int)s.kcount[j] : 0;
  const bool slot_ok = pt_ok && gr.slot < keff;
  const int view = slot_ok ? (int)s.views[FD_TOPK_SLOTS * j + gr.slot] : 0;
  const float px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
              pz = s.pts[3 * (size_t)i + 2];
  ViewPatch<P> vp;
  build_patch<T, P>(s, q, view, slot_ok, px, py, pz, vp);
  const float kinv = keff > 0 ? 1.0f / (float)keff : 0.0f;
  float dx = 0.0f, dy = 0.0f, dz = 0.0f;
  if (pt_ok && l.proposals) {
    const size_t k = 3 * (size_t)(prop_by_j ? (uint64_t)(prop_base + j) : (uint64_t)i);
    dx = l.proposals[k];
    dy = l.proposals[k + 1];
    dz = l.proposals[k + 2];
  }
  const float len = sqrtf(dx * dx + dy * dy + dz * dz);
  const bool valid = keff > 0 && isfinite(len) && len > 0.0f;
  const float il = valid ? 1.0f / len : 0.0f;
  dx = valid ? dx * il : 0.0f;
  dy = valid ? dy * il : 0.0f;
  dz = valid ? dz * il : 1.0f;
  float S = group_sum_t<KT>(eval_view<P>(vp, dx, dy, dz), gr.base, gr.K);
  refine<P, KT>(vp, gr, l.iters, l.step0, dx, dy, dz, S);
  const float J = 1.0f - S * kinv;
  const bool keep = valid && J <= l.tau;
  const bool lead = pt_ok && gr.slot == 0;
  if (lead && keep) write_result(s, i, dx, dy, dz, J);
  // the same decision in every lane of the wave
  const int n_pts = __popcll(__ballot(lead));
  const int n_need = __popcll(__ballot(lead && !keep));
  if (n_need == 0) return;
  if (2 * n_need >= n_pts) {
    float fx, fy, fz, fS;
    full_search<P, KT>(vp, q, gr, fx, fy, fz, fS);
    if (lead && !keep) {
      if (keff == 0)
        write_result(s, i, 0.0f, 0.0f, 0.0f, INFINITY);
      else
        write_result(s, i, fx, fy, fz, 1.0f - fS * kinv);
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
// first of equals) is the result.
template <typename T, int P, int KT>
__device__ __forceinline__ void fpmvo_group(const SceneDev& s, const SearchDev& q,
                                            const FpmvoDev& f, const Group& gr, bool pt_ok,
                                            int64_t j) {
  constexpr int HP = (P - 1) / 2, kc = HP * P + HP;
  const uint32_t i = pt_ok ? s.perm[j] : 0u;
  const int keff = pt_ok ? (int)s.kcount[j] : 0;
  const bool slot_ok = pt_ok && gr.slot < keff;
  const int view = slot_ok ? (int)s.views[FD_TOPK_SLOTS * j + gr.slot] : 0;
  const float px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
              pz = s.pts[3 * (size_t)i + 2];
  ViewPatch<P> vp;
  build_patch<T, P>(s, q, view, slot_ok, px, py, pz, vp);
  const float kinv = keff > 0 ? 1.0f / (float)keff : 0.0f;

  // Eq. (1): orientation of the centre sample, a = C^2/2, b = a cos 2t,
  // c = 2 a sin 2t; the unit offset (cos t, sin t) with t in (-pi/2, pi/2]
  const float* cam = s.cams + 16 * view;
  Proj pr;
  const bool in_view = slot_ok && project32(cam, px, py, pz, s.W, s.H, q.z_near, pr);
  const float a0 = vp.a[kc];
  bool vok = in_view && a0 > 0.0f;
  const float ia = vok ? 1.0f / a0 : 0.0f;
  const float c2 = vp.b[kc] * ia, s2 = 0.5f * vp.c[kc] * ia;
  const float ct = sqrtf(fmaxf(0.5f * (1.0f + c2), 0.0f));
  const float st = copysignf(sqrtf(fmaxf(0.5f * (1.0f - c2), 0.0f)), s2);
  const float w = slot_ok ? sqrtf(2.0f * a0) : 0.0f;  // centre confidence
  const float ux = (in_view ? pr.u : 0.0f) + f.lambda * ct;
  const float uy = (in_view ? pr.v : 0.0f) + f.lambda * st;
  vok = vok && ux >= 0.0f && ux <= (float)(s.W - 1) && uy >= 0.0f && uy <= (float)(s.H - 1);
  // Eq. (2): depth at the nearest texel of the offset pixel
  float D = 0.0f;
  if (vok) {
    const uint32_t xn = (uint32_t)floorf(ux + 0.5f), yn = (uint32_t)floorf(uy + 0.5f);
    D = ld_texel<T>((const T*)s.depth + (size_t)s.W * s.H * view, yn * (uint32_t)s.W + xn);
  }
  vok = vok && isfinite(D);
  // Eq. (3): p_s = R^T (X_c - t) with X_c = z_s (bx, by, 1), so
  // p_s - p = z_s g + h, g = R^T (bx, by, 1), h = -R^T t - p
  const float* R = cam + 4;
  const float* tc = cam + 13;
  const float bx = (ux - cam[2]) / cam[0], by = (uy - cam[3]) / cam[1];
  const float gx = R[0] * bx + R[3] * by + R[6], gy = R[1] * bx + R[4] * by + R[7],
              gz = R[2] * bx + R[5] * by + R[8];
  const float hx = -(R[0] * tc[0] + R[3] * tc[1] + R[6] * tc[2]) - px;
  const float hy = -(R[1] * tc[0] + R[4] * tc[1] + R[7] * tc[2]) - py;
  const float hz = -(R[2] * tc[0] + R[5] * tc[1] + R[8] * tc[2]) - pz;

  float Sb = -INFINITY, bxd = 0.0f, byd = 0.0f, bzd = 0.0f;
  for (int sl = 0; sl < f.samples; ++sl) {
    const float zs = D + (f.samples > 1 ? -f.delta + 2.0f * f.delta * (float)sl /
                                                        (float)(f.samples - 1)
                                        : 0.0f);
    float dx = __builtin_fmaf(zs, gx, hx), dy = __builtin_fmaf(zs, gy, hy),
          dz = __builtin_fmaf(zs, gz, hz);
    const float n = sqrtf(dx * dx + dy * dy + dz * dz);
    const bool ok = vok && zs > 0.0f && n > 0.0f;
    // a lane without a candidate shares exact zeros (its depth may be +inf)
    const float il = ok ? 1.0f / n : 0.0f;
    dx = ok ? dx * il : 0.0f;
    dy = ok ? dy * il : 0.0f;
    dz = ok ? dz * il : 0.0f;
    // Eqs. (5)-(6): weighted consistency of this lane's candidate with the
    // group's candidates of the same layer (views in the order of Eq. (4))
    const float wk = ok ? w : 0.0f;
    float num = 0.0f, den = 0.0f;
    const int K = KT > 0 ? KT : gr.K;
    for (int jj = 0; jj < K; ++jj) {
      const int src = gr.base + jj;
      const float xj = __shfl(dx, src, kWave), yj = __shfl(dy, src, kWave),
                  zj = __shfl(dz, src, kWave), wj = __shfl(wk, src, kWave);
      // G_ii = 1 exactly for a unit direction
      num += jj == gr.slot ? wj : wj * fabsf(dx * xj + dy * yj + dz * zj);
      den += wj;
    }
    const float sigma = ok ? num / den : -INFINITY;
    // Eq. (7): the medoid, first of equals
    int bj = -1;
    float bs = -INFINITY;
    for (int jj = 0; jj < K; ++jj) {
      const float sj = __shfl(sigma, gr.base + jj, kWave);
      if (sj > bs) {
        bs = sj;
        bj = jj;
      }
    }
    // the same in every lane of the group; the shuffles below run in every lane
    const int src = gr.base + (bj < 0 ? 0 : bj);
    const float fx = __shfl(dx, src, kWave), fy = __shfl(dy, src, kWave),
                fz = __shfl(dz, src, kWave);
    // Eq. (12): patch consistency of the fused candidate
    const float Sv = group_sum_t<KT>(eval_view<P>(vp, fx, fy, fz), gr.base, gr.K);
    if (bj >= 0 && Sv > Sb) {
      Sb = Sv;
      bxd = fx;
      byd = fy;
      bzd = fz;
    }
  }
  if (pt_ok && gr.slot == 0) {
    if (keff == 0 || !(Sb > -INFINITY))
      write_result(s, i, 0.0f, 0.0f, 0.0f, INFINITY);
    else
      write_result(s, i, bxd, byd, bzd, 1.0f - Sb * kinv);
  }
}

}  // namespace fd
