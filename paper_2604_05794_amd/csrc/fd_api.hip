// fd_api.hip -- host side of libfusedir.so: argument checks, workspace,
// launch sequences.  See include/fusedir.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"

using namespace fd;

// ---- errors -------------------------------------------------------------------

static thread_local std::string g_err;

int fd::set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fd::hip_error(hipError_t e, const char* what) {
  return set_error(FD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char* fd_last_error(void) { return g_err.c_str(); }

// ---- device check ---------------------------------------------------------------

int fd::check_device(int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  static std::mutex mu;
  static std::map<int, int> ok;  // device -> 1 gfx950, 0 other
  std::lock_guard<std::mutex> lk(mu);
  auto it = ok.find(dev);
  if (it == ok.end()) {
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDeviceProperties");
    ok[dev] = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    it = ok.find(dev);
  }
  if (!it->second)
    return set_error(FD_E_UNSUPPORTED, "device %d is not gfx950 (MI355X)", dev);
  if (dev_out) *dev_out = dev;
  return FD_OK;
}

// ---- context ---------------------------------------------------------------------

// Every reallocation goes through grow() and bumps this counter; a context
// folds it into the signature of its captured batched graph.
static uint64_t g_generation = 0;

template <typename T>
static int grow(T** p, size_t* cap, size_t need, const char* what) {
  if (*cap >= need && *p) return FD_OK;
  ++g_generation;
  if (*p) {
    hipError_t e = hipFree(*p);
    if (e != hipSuccess) return hip_error(e, what);
    *p = nullptr;
    *cap = 0;
  }
  size_t n = need > 0 ? need : 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) return set_error(FD_E_HIP, "hipMalloc %s (%zu bytes): %s", what,
                                        n * sizeof(T), hipGetErrorString(e));
  *cap = n;
  return FD_OK;
}

int fd::ctx_buffer(void** p, size_t* cap_bytes, size_t bytes, const char* what) {
  return grow((char**)p, cap_bytes, bytes, what);
}

uint64_t fd::workspace_generation() { return g_generation; }
void fd::bump_workspace_generation() { ++g_generation; }

int fd::context_reserve_points(fd_context* c, int64_t n) {
  int r;
  size_t need = (size_t)(n > 0 ? n : 1);
  if ((r = grow(&c->key, &c->cap_key, need, "tile keys"))) return r;
  if ((r = grow(&c->perm, &c->cap_perm, need, "permutation"))) return r;
  if ((r = grow(&c->views, &c->cap_views, need * FD_TOPK_SLOTS, "views"))) return r;
  if ((r = grow(&c->kcount, &c->cap_kcount, need, "view counts"))) return r;
  if ((r = grow(&c->fb_list, &c->cap_fb, need, "fallback list"))) return r;
  if ((r = grow(&c->prop, &c->cap_prop, need * 3, "proposals"))) return r;
  if ((r = grow(&c->feats, &c->cap_feats, need * FD_FEATURE_DIM, "features"))) return r;
  c->max_points = std::max<int64_t>(c->max_points, n);
  return FD_OK;
}

int fd::context_reserve_views(fd_context* c, int64_t views) {
  const size_t need = (size_t)kCam64 * (size_t)(views > 1 ? views : 1);
  return grow(&c->cams64, &c->cap_cams64, need, "camera table");
}

extern "C" int fd_context_create(fd_context** out) {
  if (!out) return set_error(FD_E_INVAL, "fd_context_create: out is NULL");
  int dev, r;
  if ((r = check_device(&dev))) return r;
  fd_context* c = new (std::nothrow) fd_context();
  if (!c) return set_error(FD_E_NOMEM, "fd_context_create: host allocation failed");
  c->device = dev;
  size_t cap = 0;
  if ((r = grow(&c->bbox, &cap, 6, "bbox")) ||
      (r = grow(&c->counts, &(cap = 0), (size_t)tile_cells(), "cell counts")) ||
      (r = grow(&c->cursor, &(cap = 0), (size_t)tile_cells(), "cell cursor")) ||
      (r = grow(&c->scan_sums, &(cap = 0), (size_t)tile_cells() / 1024, "scan sums")) ||
      (r = grow(&c->lattice, &(cap = 0), (size_t)3 * FD_MAX_CANDIDATES, "lattice")) ||
      (r = grow(&c->consts64, &(cap = 0), (size_t)kConstsDoubles, "search constants")) ||
      (r = grow(&c->fb_count, &(cap = 0), (size_t)8, "fallback counters"))) {
    fd_context_destroy(c);
    return r;
  }
  if ((r = context_reserve_points(c, 1)) || (r = context_reserve_views(c, 1024))) {
    fd_context_destroy(c);
    return r;
  }
  *out = c;
  return FD_OK;
}

extern "C" int fd_context_reserve(fd_context* c, int64_t max_points, int32_t max_views,
                                  int32_t max_scenes) {
  if (!c) return set_error(FD_E_INVAL, "fd_context_reserve: ctx is NULL");
  if (max_points < 0 || max_views < 0 || max_scenes < 0)
    return set_error(FD_E_INVAL, "fd_context_reserve: negative size");
  int r;
  if ((r = context_reserve_points(c, max_points))) return r;
  if ((r = context_reserve_views(c, max_views))) return r;
  if ((r = context_reserve_scenes(c, max_scenes, max_points))) return r;
  return FD_OK;
}

extern "C" void fd_context_destroy(fd_context* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  void* bufs[] = {c->bbox, c->counts, c->cursor, c->scan_sums, c->lattice, c->consts64,
                  c->cams64,
                  c->fb_count, c->key,
                  c->perm, c->views, c->kcount, c->fb_list, c->prop, c->feats,
                  c->scene_tab, c->tile_tab, c->tile_queue, c->batch_key, c->batch_perm,
                  c->gabor_bank, c->gabor_raw, c->gabor_max, c->vol_key, c->vol_perm,
                  c->vol_off, c->vol_bsum, c->vol_boff, c->vol_rsum, c->link_counts,
                  c->link_cursor, c->link_sums, c->link_bucket, c->link_perm, c->link_key,
                  c->link_best, c->strand_len};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

// Per-device default context, grown on demand (so calls through it may
// allocate; pass params->ctx for allocation-free calls).
fd_context* fd::default_context(int dev, int64_t n, int* err, int64_t views) {
  static std::mutex mu;
  static std::map<int, fd_context*> ctxs;
  std::lock_guard<std::mutex> lk(mu);
  fd_context*& c = ctxs[dev];
  if (!c) {
    if ((*err = fd_context_create(&c))) {
      c = nullptr;
      return nullptr;
    }
  }
  if (c->max_points < n) {
    if ((*err = context_reserve_points(c, n))) return nullptr;
  }
  if ((int64_t)(c->cap_cams64 / kCam64) < views) {
    if ((*err = context_reserve_views(c, views))) return nullptr;
  }
  *err = FD_OK;
  return c;
}

// ---- stage timing ------------------------------------------------------------------

fd::StageTimer::StageTimer(fd_context* c_, int stage_, hipStream_t st_)
    : c(c_), stage(stage_), st(st_) {
  if (!c || !c->profiling) return;
  if (hipEventCreate(&a) != hipSuccess) {
    a = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

void fd::StageTimer::stop() {
  if (!a) return;
  hipEvent_t b;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    a = nullptr;
    return;
  }
  (void)hipEventRecord(b, st);
  c->pending.push_back({stage, a, b});
  a = nullptr;
}

static void drain_pending(fd_context* c) {
  for (auto& p : c->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->stage_ms[p.stage] += ms;
      c->stage_n[p.stage] += 1;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  c->pending.clear();
}

extern "C" int fd_profile_enable(fd_context* c, int on) {
  if (!c) return set_error(FD_E_INVAL, "fd_profile_enable: ctx is NULL");
  drain_pending(c);
  for (int s = 0; s < FD_N_STAGES; ++s) {
    c->stage_ms[s] = 0.0;
    c->stage_n[s] = 0;
  }
  c->profiling = on != 0;
  return FD_OK;
}

extern "C" int fd_profile_read(fd_context* c, int stage, double* total_ms, int64_t* count) {
  if (!c || !total_ms || !count) return set_error(FD_E_INVAL, "fd_profile_read: null argument");
  if (stage < 0 || stage >= FD_N_STAGES)
    return set_error(FD_E_INVAL, "fd_profile_read: unknown stage %d", stage);
  drain_pending(c);
  *total_ms = c->stage_ms[stage];
  *count = c->stage_n[stage];
  return FD_OK;
}

// ---- params ------------------------------------------------------------------------

extern "C" void fd_params_init(fd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->width = p->height = 0;
  p->map_dtype = FD_F16;
  p->patch = 5;
  p->n_candidates = 128;
  p->refine_iters = 8;
  p->refine_step0 = 0.0f;
  p->top_k = 5;
  p->z_near = 1e-3f;
  p->mode = FD_MODE_PLAIN;
  p->mlp = nullptr;
  p->learned_iters = 2;
  p->learned_step0 = 0.0f;
  p->fallback_cost = INFINITY;
  p->proposal = FD_PROPOSAL_MLP;
  p->proposal_dirs = nullptr;
  p->vis_tau = 5e-3f;
  p->depth_maps = nullptr;
  p->fpmvo_lambda = 3.0f;
  p->fpmvo_samples = 5;
  p->fpmvo_delta = 5e-3f;
  p->stream = nullptr;
  p->ctx = nullptr;
}

int fd::check_search_params(const fd_params* p, const char* fn, bool batched) {
  if (!p) return set_error(FD_E_INVAL, "%s: params is NULL", fn);
  if (p->map_dtype != FD_F32 && p->map_dtype != FD_F16)
    return set_error(FD_E_INVAL, "%s: unknown map_dtype %d", fn, p->map_dtype);
  if (p->patch < 1 || p->patch > FD_MAX_PATCH || (p->patch & 1) == 0)
    return set_error(FD_E_INVAL, "%s: patch must be odd in [1, %d], got %d", fn, FD_MAX_PATCH,
                     p->patch);
  if (p->n_candidates < 1 || p->n_candidates > FD_MAX_CANDIDATES)
    return set_error(FD_E_INVAL, "%s: n_candidates must be in [1, %d], got %d", fn,
                     FD_MAX_CANDIDATES, p->n_candidates);
  if (p->refine_iters < 0 || p->refine_iters > FD_MAX_REFINE)
    return set_error(FD_E_INVAL, "%s: refine_iters must be in [0, %d], got %d", fn,
                     FD_MAX_REFINE, p->refine_iters);
  if (p->top_k < 1 || p->top_k > FD_MAX_TOPK)
    return set_error(FD_E_INVAL, "%s: top_k must be in [1, %d], got %d", fn, FD_MAX_TOPK,
                     p->top_k);
  if (!(p->z_near >= 0.0f) || !std::isfinite(p->z_near))
    return set_error(FD_E_INVAL, "%s: z_near must be finite and >= 0", fn);
  if (!(p->vis_tau >= 0.0f) || !std::isfinite(p->vis_tau))
    return set_error(FD_E_INVAL, "%s: vis_tau must be finite and >= 0", fn);
  if (p->mode != FD_MODE_PLAIN && p->mode != FD_MODE_LEARNED && p->mode != FD_MODE_FPMVO)
    return set_error(FD_E_INVAL, "%s: unknown mode %d", fn, p->mode);
  if (p->mode == FD_MODE_FPMVO) {
    if (!(p->fpmvo_lambda > 0.0f) || !std::isfinite(p->fpmvo_lambda))
      return set_error(FD_E_INVAL, "%s: fpmvo_lambda must be finite and > 0", fn);
    if (p->fpmvo_samples < 1 || p->fpmvo_samples > FD_MAX_FPMVO_SAMPLES)
      return set_error(FD_E_INVAL, "%s: fpmvo_samples must be in [1, %d]", fn,
                       FD_MAX_FPMVO_SAMPLES);
    if (!(p->fpmvo_delta >= 0.0f) || !std::isfinite(p->fpmvo_delta))
      return set_error(FD_E_INVAL, "%s: fpmvo_delta must be finite and >= 0", fn);
  }
  if (p->mode == FD_MODE_LEARNED) {
    if (p->learned_iters < 0 || p->learned_iters > FD_MAX_REFINE)
      return set_error(FD_E_INVAL, "%s: learned_iters must be in [0, %d]", fn, FD_MAX_REFINE);
    if (p->proposal == FD_PROPOSAL_MLP && !p->mlp)
      return set_error(FD_E_INVAL, "%s: learned mode with the network proposal needs mlp", fn);
    if (p->proposal == FD_PROPOSAL_GIVEN && !p->proposal_dirs && !batched)
      return set_error(FD_E_INVAL, "%s: FD_PROPOSAL_GIVEN needs proposal_dirs", fn);
    if (p->proposal < FD_PROPOSAL_MLP || p->proposal > FD_PROPOSAL_NAN)
      return set_error(FD_E_INVAL, "%s: unknown proposal %d", fn, p->proposal);
  }
  return FD_OK;
}

double fd::default_step0(int n_candidates) {
  return 0.5 * std::sqrt(2.0 * 3.14159265358979323846 / (double)n_candidates);
}

void fd::resolve_steps(const fd_params* p, double* step0, double* lstep0) {
  *step0 = p->refine_step0 > 0.0f ? (double)p->refine_step0 : default_step0(p->n_candidates);
  double l = p->learned_step0 > 0.0f ? (double)p->learned_step0 : 0.0;
  if (!(l > 0.0) && p->mlp) {
    float s0 = 0.0f, tau = 0.0f;
    if (fd_mlp_get_calibration(p->mlp, &s0, &tau) == FD_OK && s0 > 0.0f) l = (double)s0;
  }
  *lstep0 = l > 0.0 ? l : default_step0(p->n_candidates);
}

ConstsDev fd::context_consts(fd_context* c) {
  ConstsDev k;
  k.lattice = c->lattice;
  k.lattice64 = c->consts64;
  k.steps = c->consts64 + 3 * FD_MAX_CANDIDATES;
  return k;
}

// ---- single scene ---------------------------------------------------------------------

int fd::check_scene_call(const float* points, int64_t n_points, const fd_camera* cams,
                         int32_t n_views, const void* orient_maps, const void* conf_maps,
                         const fd_params* params, float* dirs, float* costs, const char* fn) {
  int r;
  if ((r = check_search_params(params, fn))) return r;
  if (params->mode == FD_MODE_FPMVO && !params->depth_maps)
    return set_error(FD_E_INVAL, "%s: FD_MODE_FPMVO needs depth_maps", fn);
  if (n_points < 0) return set_error(FD_E_INVAL, "%s: n_points < 0", fn);
  if (n_points > (int64_t)UINT32_MAX)
    return set_error(FD_E_INVAL, "%s: n_points exceeds 2^32 - 1", fn);
  if (n_views < 1 || n_views > FD_MAX_VIEWS)
    return set_error(FD_E_INVAL, "%s: n_views must be in [1, %d], got %d", fn, FD_MAX_VIEWS,
                     n_views);
  if (params->width < 1 || params->height < 1 || params->width > 32768 ||
      params->height > 32768)
    return set_error(FD_E_INVAL, "%s: map size %d x %d out of range", fn, params->width,
                     params->height);
  if (params->top_k > n_views)
    return set_error(FD_E_INVAL, "%s: top_k (%d) > n_views (%d)", fn, params->top_k, n_views);
  if (n_points > 0 && (!points || !cams || !orient_maps || !conf_maps || !dirs || !costs))
    return set_error(FD_E_INVAL, "%s: null pointer argument", fn);
  return check_device(nullptr);
}

fd::SceneArgs fd::scene_args(const float* points, int64_t n_points, const fd_camera* cams,
                             int32_t n_views, const void* orient_maps, const void* conf_maps,
                             const fd_params* params, float* dirs, float* costs) {
  SceneArgs sa;
  sa.points = points;
  sa.n = n_points;
  sa.cams = (const float*)cams;
  sa.V = n_views;
  sa.W = params->width;
  sa.H = params->height;
  sa.theta = orient_maps;
  sa.conf = conf_maps;
  sa.depth = params->depth_maps;
  sa.dirs = dirs;
  sa.costs = costs;
  for (int k = 0; k < 3; ++k) sa.hc[k] = params->head_centre[k];
  return sa;
}

extern "C" int fd_fuse_directions(const float* points, int64_t n_points, const fd_camera* cams,
                                  int32_t n_views, const void* orient_maps,
                                  const void* conf_maps, const fd_params* params, float* dirs,
                                  float* costs) {
  const char* fn = "fd_fuse_directions";
  int r;
  if ((r = check_scene_call(points, n_points, cams, n_views, orient_maps, conf_maps, params,
                            dirs, costs, fn)))
    return r;
  if (n_points == 0) return FD_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  fd_context* c = params->ctx;
  if (c) {
    if (c->device != dev)
      return set_error(FD_E_INVAL, "%s: context belongs to device %d, current is %d", fn,
                       c->device, dev);
    if (c->max_points < n_points)
      return set_error(FD_E_NOMEM, "%s: context reserved for %lld points, call has %lld", fn,
                       (long long)c->max_points, (long long)n_points);
    if ((int64_t)(c->cap_cams64 / kCam64) < n_views)
      return set_error(FD_E_NOMEM, "%s: context reserved for %lld views, call has %d "
                       "(fd_context_reserve max_views)", fn,
                       (long long)(c->cap_cams64 / kCam64), n_views);
  } else {
    c = default_context(dev, n_points, &r, n_views);
    if (!c) return r;
  }
  const SceneArgs sa = scene_args(points, n_points, cams, n_views, orient_maps, conf_maps,
                                  params, dirs, costs);
  return run_scene(c, sa, params, (hipStream_t)params->stream);
}

int fd::run_scene(fd_context* c, const SceneArgs& a, const fd_params* p, hipStream_t st) {
  double step0, lstep0;
  resolve_steps(p, &step0, &lstep0);
  const ConstsDev kc = context_consts(c);
  hipError_t e0 = launch_consts(kc, p->n_candidates, step0, lstep0, st);
  if (e0 != hipSuccess) return hip_error(e0, "search constants");
  TileWork tw{c->bbox, c->key, c->counts, c->cursor, c->scan_sums, c->perm};
  StageTimer t_tile(c, FD_STAGE_TILING, st);
  hipError_t e = launch_tiling(a.points, a.n, tw, st);
  if (e != hipSuccess) return hip_error(e, "tiling kernels");
  t_tile.stop();
  SceneDev s;
  s.prop = nullptr;
  s.pts = a.points;
  s.cams = a.cams;
  s.theta = a.theta;
  s.conf = a.conf;
  s.depth = a.depth;
  s.vis_tau = p->vis_tau;
  s.dirs = a.dirs;
  s.costs = a.costs;
  s.perm = c->perm;
  s.views = c->views;
  s.kcount = c->kcount;
  s.n = a.n;
  s.V = a.V;
  s.W = a.W;
  s.H = a.H;
  for (int k = 0; k < 3; ++k) s.hc[k] = a.hc[k];
  s.pairs = scene_pairs(p->map_dtype, a.W, a.theta, a.conf, a.depth);
  const SearchDev q = make_search(kc, p->n_candidates, p->refine_iters, p->top_k, p->z_near);
  if ((e = launch_cams64(a.cams, a.V, c->cams64, st)) != hipSuccess)
    return hip_error(e, "camera table");
  s.cam64 = c->cams64;
  const bool fused_topk = p->mode == FD_MODE_LEARNED && p->proposal == FD_PROPOSAL_MLP;
  if (!fused_topk) {  // the learned network path selects views with its features
    StageTimer t_topk(c, FD_STAGE_TOPK, st);
    if ((e = launch_topk(s, q, p->map_dtype, st)) != hipSuccess)
      return hip_error(e, "view selection kernel");
    t_topk.stop();
  }
  if (p->mode == FD_MODE_PLAIN) {
    StageTimer t_fuse(c, FD_STAGE_FUSE, st);
    if ((e = launch_fuse(s, q, p->map_dtype, p->patch, nullptr, nullptr, st)) != hipSuccess)
      return hip_error(e, "fusion kernel");
    t_fuse.stop();
    return FD_OK;
  }
  if (p->mode == FD_MODE_FPMVO) {
    FpmvoDev f{p->fpmvo_lambda, p->fpmvo_samples, p->fpmvo_delta};
    StageTimer t_fuse(c, FD_STAGE_FUSE, st);
    if ((e = launch_fpmvo(s, q, f, p->map_dtype, p->patch, st)) != hipSuccess)
      return hip_error(e, "candidate fusion kernel");
    t_fuse.stop();
    return FD_OK;
  }
  return run_learned(c, s, q, p, st);
}
