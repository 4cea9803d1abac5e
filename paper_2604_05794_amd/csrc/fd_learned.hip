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
#include "fd_features.hpp"

using namespace fd;

namespace fd {
int mlp_forward_dev(const fd_mlp* m, const uint16_t* feats, int64_t n, float* out, hipStream_t st);
}

namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_features(SceneDev s, float z_near, int by_j,
                                                  uint16_t* __restrict__ feats) {
  const int64_t j = xcd_tile(gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  features_point<T>(s, z_near, j, by_j, 0, feats);
}

template <typename T, int KS>
__global__ __launch_bounds__(256) void k_topk_features(SceneDev s, SearchDev q,
                                                       uint16_t* __restrict__ feats) {
  const int64_t j = xcd_tile(gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  topk_features_point<T, KS>(s, q, j, 0, feats);
}

// The same for scenes of at most kMaskViews views, in two kernels (view
// selection with the visibility bits, then the frontal ranking and the
// row), the first held to five waves per SIMD.
template <typename T, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KS <= 5 ? 5 : 4)))
void k_vis_m(SceneDev s, SearchDev q, uint16_t* __restrict__ feats) {
  const int64_t j = xcd_tile(gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  vis_topk_masked<T, KS, kMaskViews / 32>(s, q, s.cam64, j, j, feats);
}

template <typename T>
__global__ __launch_bounds__(256) void k_frontal_row_m(SceneDev s, uint16_t* __restrict__ feats) {
  const int64_t j = xcd_tile(gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  frontal_row_masked<T, kMaskViews / 32>(s, s.cam64, j, j, feats);
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
  if ((e = launch_fill_u32(c->fb_count, 2, 0u, st)) != hipSuccess)
    return hip_error(e, "fallback counter reset");
  LearnedDev l;
  // the learned steps follow the plain ones in the per-call constants
  l.steps = q.steps + 3 * FD_MAX_REFINE;
  l.iters = p->learned_iters;
  l.tau = (double)p->fallback_cost;
  l.fb_list = c->fb_list;
  l.fb_count = c->fb_count;
  int prop_by_j = 0;
  if (p->proposal == FD_PROPOSAL_MLP) {
    // view selection was done together with the features (run_scene skips
    // its own top-K pass in this mode)
    StageTimer tf(c, FD_STAGE_FEATURES, st);
    dim3 grid((unsigned)((s.n + 255) / 256));
    const bool k5 = q.K <= 5;  // a list of 5 slots holds any top-K with K <= 5
    const bool m = s.V <= kMaskViews;
#define FD_TOPK_FEATURES(T, KS)                                                             \
  do {                                                                                      \
    if (m) {                                                                                \
      hipLaunchKernelGGL((k_vis_m<T, KS>), grid, dim3(256), 0, st, s, q, c->feats);          \
      hipLaunchKernelGGL((k_frontal_row_m<T>), grid, dim3(256), 0, st, s, c->feats);         \
    } else {                                                                                \
      hipLaunchKernelGGL((k_topk_features<T, KS>), grid, dim3(256), 0, st, s, q, c->feats);  \
    }                                                                                       \
  } while (0)
    if (p->map_dtype == FD_F16) {
      if (k5)
        FD_TOPK_FEATURES(__half, 5);
      else
        FD_TOPK_FEATURES(__half, FD_TOPK_SLOTS);
    } else {
      if (k5)
        FD_TOPK_FEATURES(float, 5);
      else
        FD_TOPK_FEATURES(float, FD_TOPK_SLOTS);
    }
#undef FD_TOPK_FEATURES
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "view selection + features");
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
  uint32_t v[2] = {0, 0};
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(v, c->fb_count, sizeof v, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "fd_last_fallback_count");
  *out = (int64_t)v[0] + (int64_t)v[1];  // listed + searched in place
  return FD_OK;
}

extern "C" int fd_last_fallback_split(fd_context* c, void* stream, int64_t* listed,
                                      int64_t* in_place) {
  if (!c || !listed || !in_place)
    return set_error(FD_E_INVAL, "fd_last_fallback_split: null argument");
  uint32_t v[2] = {0, 0};
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(v, c->fb_count, sizeof v, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_error(e, "fd_last_fallback_split");
  *listed = v[0];
  *in_place = v[1];
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
  if (!(params->vis_tau >= 0.0f) || !std::isfinite(params->vis_tau))
    return set_error(FD_E_INVAL, "%s: vis_tau must be finite and >= 0", fn);
  if ((r = check_device(nullptr))) return r;
  if (n_points == 0) return FD_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  fd_context* c = default_context(dev, 0, &r, n_views);
  if (!c) return r;
  hipError_t e0 = launch_cams64((const float*)cams, n_views, c->cams64,
                                (hipStream_t)params->stream);
  if (e0 != hipSuccess) return hip_error(e0, "camera table");
  SceneDev s{};
  s.cam64 = c->cams64;
  s.pts = points;
  s.cams = (const float*)cams;
  s.theta = orient_maps;
  s.conf = conf_maps;
  s.depth = params->depth_maps;
  s.vis_tau = params->vis_tau;
  s.perm = nullptr;
  s.n = n_points;
  s.V = n_views;
  s.W = params->width;
  s.H = params->height;
  for (int k = 0; k < 3; ++k) s.hc[k] = params->head_centre[k];
  s.pairs = scene_pairs(params->map_dtype, s.W, orient_maps, conf_maps, params->depth_maps);
  hipError_t e = launch_features_rows(s, params->map_dtype, params->z_near, 0, (uint16_t*)feats,
                                      (hipStream_t)params->stream);
  return e == hipSuccess ? FD_OK : hip_error(e, "feature kernel");
}
