// fd_learned.hip -- learned form of the direction search: proposal-network
// features, the launch sequence proposal -> short refinement -> threshold ->
// plain search of the fallback list.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_device.hpp"
#include "fd_kernels.hpp"

using namespace fd;

namespace fd {
int mlp_forward_dev(const fd_mlp* m, const uint16_t* feats, int64_t n, float* out, hipStream_t st);
}

namespace {

constexpr int kSlots = FD_FEATURE_SLOTS;

__device__ __forceinline__ uint16_t f2bf(float x) {
  // round to nearest even
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Frontal ranking key of a view, decided in binary32 with a fixed order:
//   c = -R^T t  (c_x = -fma(R0, t0, fma(R3, t1, R6*t2)), likewise y, z)
//   a = c - p, b = p - o
//   score = fma(a_x, b_x, fma(a_y, b_y, a_z*b_z)) / sqrt(fma(a_x, a_x, fma(a_y, a_y, a_z*a_z)))
// i.e. the cosine between the point->camera direction and the outward
// direction p - o, times |p - o| (common to every view of the point).
__device__ __forceinline__ float frontal_score32(const float* cam, float px, float py, float pz,
                                                 const float* o, float* vdir) {
  const float* R = cam + 4;
  const float* t = cam + 13;
  const float cx = -__builtin_fmaf(R[0], t[0], __builtin_fmaf(R[3], t[1], R[6] * t[2]));
  const float cy = -__builtin_fmaf(R[1], t[0], __builtin_fmaf(R[4], t[1], R[7] * t[2]));
  const float cz = -__builtin_fmaf(R[2], t[0], __builtin_fmaf(R[5], t[1], R[8] * t[2]));
  const float ax = cx - px, ay = cy - py, az = cz - pz;
  const float bx = px - o[0], by = py - o[1], bz = pz - o[2];
  const float dot = __builtin_fmaf(ax, bx, __builtin_fmaf(ay, by, az * bz));
  const float la = sqrtf(__builtin_fmaf(ax, ax, __builtin_fmaf(ay, ay, az * az)));
  if (vdir) {
    vdir[0] = ax / la;
    vdir[1] = ay / la;
    vdir[2] = az / la;
  }
  return dot / la;
}

// One lane per point: the kSlots most frontal eligible views (stable: equal
// scores keep the lower view index first), then per slot the bilinear
// confidence-weighted doubled-angle vector (m_x, m_y), the bilinear
// confidence C, the unit point->camera direction and 1; empty slots are 0.
// Row r of `feats` (112 bfloat16) is the processing-order index when by_j,
// else the point index.
template <typename T>
__global__ __launch_bounds__(256) void k_features(SceneDev s, float z_near, int by_j,
                                                  uint16_t* __restrict__ feats) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  const uint32_t i = s.perm ? s.perm[j] : (uint32_t)j;
  const float px = s.pts[3 * (size_t)i], py = s.pts[3 * (size_t)i + 1],
              pz = s.pts[3 * (size_t)i + 2];
  float sc[kSlots];
  int id[kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    sc[k] = -INFINITY;
    id[k] = -1;
  }
  for (int v = 0; v < s.V; ++v) {
    Proj pr;
    if (!project32(s.cams + 16 * v, px, py, pz, s.W, s.H, z_near, pr)) continue;
    float cs = frontal_score32(s.cams + 16 * v, px, py, pz, s.hc, nullptr);
    int cv = v;
    bool ins = false;
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      bool take = ins || (cs > sc[k]) || (!ins && id[k] < 0);
      float ts = sc[k];
      int tv = id[k];
      sc[k] = take ? cs : ts;
      id[k] = take ? cv : tv;
      cs = take ? ts : cs;
      cv = take ? tv : cv;
      ins = ins || take;
    }
  }
  const T* th = (const T*)s.theta;
  const T* cf = (const T*)s.conf;
  const size_t plane = (size_t)s.W * s.H;
  const float kInvPi = 0.318309886183790671538f;
  uint16_t out[7 * kSlots];
#pragma unroll
  for (int k = 0; k < kSlots; ++k) {
    float f[7] = {0, 0, 0, 0, 0, 0, 0};
    if (id[k] >= 0) {
      const int v = id[k];
      const float* cam = s.cams + 16 * v;
      Proj pr;
      project32(cam, px, py, pz, s.W, s.H, z_near, pr);
      const float x0 = floorf(pr.u), y0 = floorf(pr.v);
      const float fx = pr.u - x0, fy = pr.v - y0;
      const int ix = (int)x0, iy = (int)y0;
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
      frontal_score32(cam, px, py, pz, s.hc, vd);
      f[0] = mx;
      f[1] = my;
      f[2] = cb;
      f[3] = vd[0];
      f[4] = vd[1];
      f[5] = vd[2];
      f[6] = 1.0f;
    }
#pragma unroll
    for (int e = 0; e < 7; ++e) out[7 * k + e] = f2bf(f[e]);
  }
  uint4* dst = (uint4*)(feats + (size_t)(by_j ? j : (int64_t)i) * (7 * kSlots));
  const uint4* src = (const uint4*)out;
#pragma unroll
  for (int e = 0; e < (7 * kSlots * 2) / 16; ++e) dst[e] = src[e];
}

}  // namespace

static hipError_t launch_features_rows(const SceneDev& s, int dtype, float z_near, int by_j,
                                       uint16_t* feats, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  dim3 grid((unsigned)((s.n + 255) / 256));
  if (dtype == 1)
    hipLaunchKernelGGL(k_features<__half>, grid, dim3(256), 0, st, s, z_near, by_j, feats);
  else
    hipLaunchKernelGGL(k_features<float>, grid, dim3(256), 0, st, s, z_near, by_j, feats);
  return hipGetLastError();
}

int fd::run_learned(fd_context* c, const SceneDev& s, const SearchDev& q, const fd_params* p,
                    hipStream_t st) {
  hipError_t e;
  if ((e = launch_fill_u32(c->fb_count, 1, 0u, st)) != hipSuccess)
    return hip_error(e, "fallback counter reset");
  LearnedDev l;
  l.iters = p->learned_iters;
  l.tau = p->fallback_cost;
  l.fb_list = c->fb_list;
  l.fb_count = c->fb_count;
  float step0 = p->learned_step0;
  if (!(step0 > 0.0f) && p->mlp) {
    float s0 = 0.0f, tau = 0.0f;
    fd_mlp_get_calibration(p->mlp, &s0, &tau);
    step0 = s0;
  }
  if (!(step0 > 0.0f)) step0 = default_step0(p->n_candidates);
  l.step0 = step0;
  int prop_by_j = 0;
  if (p->proposal == FD_PROPOSAL_MLP) {
    StageTimer tf(c, FD_STAGE_FEATURES, st);
    if ((e = launch_features_rows(s, p->map_dtype, p->z_near, 1, c->feats, st)) != hipSuccess)
      return hip_error(e, "feature kernel");
    tf.stop();
    StageTimer tm(c, FD_STAGE_MLP, st);
    int r = mlp_forward_dev(p->mlp, c->feats, s.n, c->prop, st);
    if (r) return r;
    tm.stop();
    l.proposals = c->prop;
    prop_by_j = 1;
  } else if (p->proposal == FD_PROPOSAL_GIVEN) {
    l.proposals = p->proposal_dirs;
  } else {
    l.proposals = nullptr;
  }
  StageTimer tr(c, FD_STAGE_REFINE, st);
  if ((e = launch_learned_refine(s, q, l, p->map_dtype, p->patch, prop_by_j, st)) != hipSuccess)
    return hip_error(e, "learned refinement kernel");
  tr.stop();
  StageTimer tb(c, FD_STAGE_FALLBACK, st);
  if ((e = launch_fuse(s, q, p->map_dtype, p->patch, c->fb_list, c->fb_count, st)) != hipSuccess)
    return hip_error(e, "fallback kernel");
  tb.stop();
  return FD_OK;
}

extern "C" int fd_last_fallback_count(fd_context* c, void* stream, int64_t* out) {
  if (!c || !out) return set_error(FD_E_INVAL, "fd_last_fallback_count: null argument");
  uint32_t v = 0;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(&v, c->fb_count, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "fd_last_fallback_count");
  *out = v;
  return FD_OK;
}

extern "C" int fd_features(const float* points, int64_t n_points, const fd_camera* cams,
                           int32_t n_views, const void* orient_maps, const void* conf_maps,
                           const fd_params* params, void* feats) {
  const char* fn = "fd_features";
  int r;
  if (!params) return set_error(FD_E_INVAL, "%s: params is NULL", fn);
  if (params->map_dtype != FD_F32 && params->map_dtype != FD_F16)
    return set_error(FD_E_INVAL, "%s: unknown map_dtype", fn);
  if (n_points < 0 || n_points > (int64_t)UINT32_MAX)
    return set_error(FD_E_INVAL, "%s: n_points out of range", fn);
  if (n_views < 1 || n_views > FD_MAX_VIEWS) return set_error(FD_E_INVAL, "%s: n_views", fn);
  if (params->width < 1 || params->height < 1 || params->width > 32768 || params->height > 32768)
    return set_error(FD_E_INVAL, "%s: map size out of range", fn);
  if (n_points > 0 && (!points || !cams || !orient_maps || !conf_maps || !feats))
    return set_error(FD_E_INVAL, "%s: null pointer argument", fn);
  if (((uintptr_t)feats & 15) != 0) return set_error(FD_E_INVAL, "%s: feats must be 16-byte aligned", fn);
  if ((r = check_device(nullptr))) return r;
  if (n_points == 0) return FD_OK;
  SceneDev s{};
  s.pts = points;
  s.cams = (const float*)cams;
  s.theta = orient_maps;
  s.conf = conf_maps;
  s.perm = nullptr;
  s.n = n_points;
  s.V = n_views;
  s.W = params->width;
  s.H = params->height;
  for (int k = 0; k < 3; ++k) s.hc[k] = params->head_centre[k];
  hipError_t e = launch_features_rows(s, params->map_dtype, params->z_near, 0, (uint16_t*)feats,
                                      (hipStream_t)params->stream);
  return e == hipSuccess ? FD_OK : hip_error(e, "feature kernel");
}
