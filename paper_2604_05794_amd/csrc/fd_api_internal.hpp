// fd_api_internal.hpp -- host-side state shared by the API sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/fusedir.h"
#include "fd_kernels.hpp"

struct fd_context {
  int device = 0;
  int64_t max_points = 0;
  // bumped whenever a workspace buffer is reallocated, so that a captured
  // batched graph or uploaded scene table never keeps a freed pointer
  uint64_t generation = 0;
  // fixed buffers
  int* bbox = nullptr;
  uint32_t* counts = nullptr;
  uint32_t* cursor = nullptr;
  uint32_t* scan_sums = nullptr;
  float* lattice = nullptr;   // search constants (ConstsDev): binary32 lattice
  double* consts64 = nullptr; // binary64 lattice, step tables
  double* cams64 = nullptr;   // binary64 camera table, kCam64 per view
  size_t cap_cams64 = 0;      // doubles
  uint32_t* fb_count = nullptr;
  // per-point buffers
  uint32_t* key = nullptr;
  size_t cap_key = 0;
  uint32_t* perm = nullptr;
  size_t cap_perm = 0;
  uint16_t* views = nullptr;
  size_t cap_views = 0;
  uint8_t* kcount = nullptr;
  size_t cap_kcount = 0;
  uint32_t* fb_list = nullptr;
  size_t cap_fb = 0;
  float* prop = nullptr;
  size_t cap_prop = 0;
  uint16_t* feats = nullptr;
  size_t cap_feats = 0;
  // batched launch
  int32_t max_scenes = 0;
  void* scene_tab = nullptr;
  size_t cap_scene_tab = 0;
  void* tile_tab = nullptr;
  size_t cap_tile_tab = 0;
  uint32_t* tile_queue = nullptr;
  size_t cap_tile_queue = 0;
  uint32_t* batch_key = nullptr;
  size_t cap_batch_key = 0;
  uint32_t* batch_perm = nullptr;
  size_t cap_batch_perm = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t graph_sig = 0;
  uint64_t table_sig = 0;   // scene set whose table is on the device
  hipStream_t cap_stream = nullptr;
  // orientation-map extraction: the filter bank (tap-major), raw confidence,
  // per-frame maxima
  float* gabor_bank = nullptr;
  size_t cap_gabor_bank = 0;
  uint64_t gabor_sig = 0;
  float* gabor_raw = nullptr;
  size_t cap_gabor_raw = 0;
  uint32_t* gabor_max = nullptr;
  size_t cap_gabor_max = 0;
  // orientation volume: counting sort of the points by voxel
  uint32_t* vol_key = nullptr;   // voxel and rank per point
  size_t cap_vol_key = 0;
  uint32_t* vol_perm = nullptr;  // sorted fixed-point terms, 48 B per point
  size_t cap_vol_perm = 0;
  uint32_t* vol_off = nullptr;   // first slot per voxel
  size_t cap_vol_off = 0;
  uint32_t* vol_bsum = nullptr;  // per block of 1024 voxels, padded to 1024 blocks
  size_t cap_vol_bsum = 0;
  uint32_t* vol_boff = nullptr;
  size_t cap_vol_boff = 0;
  uint32_t* vol_rsum = nullptr;
  size_t cap_vol_rsum = 0;
  // segment linking: start hash (counting sort) and proposals
  uint32_t* link_counts = nullptr;
  size_t cap_link_counts = 0;
  uint32_t* link_cursor = nullptr;
  size_t cap_link_cursor = 0;
  uint32_t* link_sums = nullptr;
  size_t cap_link_sums = 0;
  uint32_t* link_bucket = nullptr;
  size_t cap_link_bucket = 0;
  uint32_t* link_perm = nullptr;
  size_t cap_link_perm = 0;
  unsigned long long* link_key = nullptr;
  size_t cap_link_key = 0;
  unsigned long long* link_best = nullptr;
  size_t cap_link_best = 0;
  int64_t* strand_len = nullptr;  // per guide strand, before the scan
  size_t cap_strand_len = 0;
  // tuned shape of the persistent search: tiles per queue pop, resident grid
  int tuned_chunk = 0;
  int tuned_grid = 0;
  // stage timing
  bool profiling = false;
  struct Pending {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double stage_ms[FD_N_STAGES] = {};
  int64_t stage_n[FD_N_STAGES] = {};
};

namespace fd {

struct SceneArgs {
  const float* points;
  int64_t n;
  const float* cams;
  int V, W, H;
  const void* theta;
  const void* conf;
  const void* depth;
  float* dirs;
  float* costs;
  float hc[3];
};

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
int check_device(int* dev_out);
// batched: the proposals of FD_PROPOSAL_GIVEN come with the scenes
int check_search_params(const fd_params* p, const char* fn, bool batched = false);
double default_step0(int n_candidates);
// First step of the plain refinement and of the learned form's short
// refinement (parameter, else the network's calibration, else the default).
void resolve_steps(const fd_params* p, double* step0, double* lstep0);
ConstsDev context_consts(fd_context* c);
int context_reserve_points(fd_context* c, int64_t n);
// Grows the binary64 camera table to at least `views` views.
int context_reserve_views(fd_context* c, int64_t views);
int context_reserve_scenes(fd_context* c, int32_t n_scenes, int64_t total_points);
fd_context* default_context(int dev, int64_t n, int* err, int64_t views = 1);
// Grows a context-owned device buffer to at least `bytes` (no-op if large
// enough; the old contents are not kept).
int ctx_buffer(void** p, size_t* cap_bytes, size_t bytes, const char* what);
// Count of workspace reallocations so far (any context).
uint64_t workspace_generation();
void bump_workspace_generation();
int run_scene(fd_context* c, const SceneArgs& a, const fd_params* p, hipStream_t st);
// Argument checks shared by the single-scene entry points (nothing is
// launched on an error), and the scene they describe.
int check_scene_call(const float* points, int64_t n_points, const fd_camera* cams,
                     int32_t n_views, const void* orient_maps, const void* conf_maps,
                     const fd_params* params, float* dirs, float* costs, const char* fn);
SceneArgs scene_args(const float* points, int64_t n_points, const fd_camera* cams,
                     int32_t n_views, const void* orient_maps, const void* conf_maps,
                     const fd_params* params, float* dirs, float* costs);
// Records HIP events around one stage when the context profiles.
struct StageTimer {
  fd_context* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(fd_context* c_, int stage_, hipStream_t st_);
  ~StageTimer() {
    if (a) (void)hipEventDestroy(a);
  }
  void stop();
};

int run_learned(fd_context* c, const SceneDev& s, const SearchDev& q, const fd_params* p,
                hipStream_t st);

}  // namespace fd
