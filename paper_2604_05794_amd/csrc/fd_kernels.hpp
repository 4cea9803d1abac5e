// fd_kernels.hpp -- internal interface between the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fusedir.h"

namespace fd {

// Register slots of the view selection (>= any top_k the API accepts).
#define FD_TOPK_SLOTS 8

// Workspace of the spatial tiling (fd_tile.hip).
struct TileWork {
  int* bbox;         // 6 ints
  uint32_t* key;     // n
  uint32_t* counts;  // tile_cells()
  uint32_t* cursor;  // tile_cells()
  uint32_t* sums;    // tile_cells() / 1024
  uint32_t* perm;    // n
};

// One scene as the fusion kernels see it.
struct SceneDev {
  const float* pts;     // n x 3
  const float* cams;    // V x 16
  const void* theta;    // V x H x W
  const void* conf;     // V x H x W
  float* dirs;          // n x 3
  float* costs;         // n
  const uint32_t* perm; // n, processing order -> point index
  uint16_t* views;      // n x 8, selected views (processing order)
  uint8_t* kcount;      // n, K_eff (processing order)
  const void* depth;    // V x H x W camera-space Z, or NULL (no visibility test)
  const double* cam64;  // V x 16 binary64 projection rows and centre (launch_cams64)
  const float* prop;    // n x 3 given proposals in point order, or NULL
  int64_t n;
  int V, W, H;
  float hc[3];          // head centre (frontal ranking)
  float vis_tau;        // visibility tolerance on |Z - D|
  int pairs;            // texel pairs may be read with 4-byte loads (scene_pairs)
};

// Texel pairs of a row may be read with dword-aligned loads: binary16 maps
// of even width (at least 4) whose base addresses are 4-byte aligned.
inline int scene_pairs(int map_dtype, int W, const void* theta, const void* conf,
                       const void* depth) {
  const uintptr_t a = (uintptr_t)theta | (uintptr_t)conf | (uintptr_t)depth;
  return map_dtype == FD_F16 && (W & 1) == 0 && W >= 4 && (a & 3u) == 0;
}

// A scene record read from device memory (the batched scene table) would
// hold generic pointers, which the compiler addresses with flat
// instructions.  The table is read through this layout-identical view whose
// pointers are in the global address space, so everything derived from them
// uses global loads and stores (the table only ever holds device-memory
// pointers).
#define FD_GLOBAL __attribute__((address_space(1)))
struct SceneDevGlobal {
  const FD_GLOBAL float* pts;
  const FD_GLOBAL float* cams;
  const FD_GLOBAL void* theta;
  const FD_GLOBAL void* conf;
  FD_GLOBAL float* dirs;
  FD_GLOBAL float* costs;
  const FD_GLOBAL uint32_t* perm;
  FD_GLOBAL uint16_t* views;
  FD_GLOBAL uint8_t* kcount;
  const FD_GLOBAL void* depth;
  const FD_GLOBAL double* cam64;
  const FD_GLOBAL float* prop;
  int64_t n;
  int V, W, H;
  float hc[3];
  float vis_tau;
  int pairs;
};
static_assert(sizeof(SceneDevGlobal) == sizeof(SceneDev), "scene record views differ");

__device__ __forceinline__ SceneDev load_scene(const SceneDev* tab, int s) {
  const SceneDevGlobal& g = reinterpret_cast<const SceneDevGlobal*>(tab)[s];
  SceneDev d;
  d.pts = (const float*)g.pts;
  d.cams = (const float*)g.cams;
  d.theta = (const void*)g.theta;
  d.conf = (const void*)g.conf;
  d.dirs = (float*)g.dirs;
  d.costs = (float*)g.costs;
  d.perm = (const uint32_t*)g.perm;
  d.views = (uint16_t*)g.views;
  d.kcount = (uint8_t*)g.kcount;
  d.depth = g.depth ? (const void*)g.depth : nullptr;
  d.cam64 = (const double*)g.cam64;
  d.prop = g.prop ? (const float*)g.prop : nullptr;
  d.n = g.n;
  d.V = g.V;
  d.W = g.W;
  d.H = g.H;
  for (int k = 0; k < 3; ++k) d.hc[k] = g.hc[k];
  d.vis_tau = g.vis_tau;
  d.pairs = g.pairs;
  return d;
}
#undef FD_GLOBAL

struct SearchDev {
  const float* lattice;    // n_candidates x 3, binary32 (lattice stage)
  const double* lattice64; // the same directions in binary64 (refinement start)
  const double* steps;     // cos alpha_t, sin alpha_t, cos alpha_t - 1 [FD_MAX_REFINE each]
  int n_candidates;
  int refine_iters;
  int K;
  double z_near;
};

// Paper-literal candidate mode.
struct FpmvoDev {
  float lambda;   // pixel offset along the observed orientation
  int samples;    // depth layers S
  float delta;    // layers span [-delta, delta] around the sampled depth
};

// Learned form (fd_learned.hip).
struct LearnedDev {
  const float* proposals;  // n x 3 (see learned_group), or NULL: the scene's own (SceneDev::prop)
  const double* steps;     // cos / sin of the learned refinement's steps (as SearchDev)
  int iters;
  double tau;
  uint32_t* fb_list;       // processing-order indices that fall back
  uint32_t* fb_count;      // [0] fallback list length, [1] points searched in place
};

// Per-call constants of the search in device memory (fd_fuse.hip, k_consts):
// the lattice in binary32 and binary64 and the cos/sin tables of the plain
// and learned refinement steps.
struct ConstsDev {
  float* lattice;     // FD_MAX_CANDIDATES x 3
  double* lattice64;  // FD_MAX_CANDIDATES x 3
  double* steps;      // 3 x FD_MAX_REFINE (plain), then 3 x FD_MAX_REFINE (learned)
};
constexpr int kConstsDoubles = 3 * FD_MAX_CANDIDATES + 6 * FD_MAX_REFINE;

hipError_t launch_fpmvo(const SceneDev& s, const SearchDev& q, const FpmvoDev& f, int dtype,
                        int patch, hipStream_t st);
hipError_t launch_tiling(const float* pts, int64_t n, TileWork w, hipStream_t st);
hipError_t launch_identity_perm(int64_t n, uint32_t* perm, hipStream_t st);
hipError_t launch_scan_runs(const uint32_t* counts, int n_runs, uint32_t* sums, uint32_t* cursor,
                            hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
int tile_cells();

// Fills the per-call constants: lattice of n directions, cos, sin and
// cos - 1 of the plain steps step0 / 2^t (t < FD_MAX_REFINE) and of the
// learned steps lstep0 / 2^t.
hipError_t launch_consts(const ConstsDev& c, int n, double step0, double lstep0, hipStream_t st);
// Per view, kCam64 binary64 slots: the projection rows
// (f_x R_0 + c_x R_2 | f_x t_0 + c_x t_2), (f_y R_1 + c_y R_2 | f_y t_1 + c_y t_2),
// (R_2 | t_2) (R_i the rows of R), so that u = row0 . (p, 1) / row2 . (p, 1),
// then the camera centre -R^T t and a zero; then (slots 16-23, 16-byte
// aligned) the camera record itself, 16 binary32 values, for vector loads.
constexpr int kCam64 = 24;
constexpr int kCam32Off = 16;  // first slot of the binary32 record
hipError_t launch_cams64(const float* cams, int V, double* out, hipStream_t st);
// Search constants as the kernels read them.
SearchDev make_search(const ConstsDev& c, int n_candidates, int refine_iters, int K,
                      float z_near);
hipError_t launch_topk(const SceneDev& s, const SearchDev& q, int dtype, hipStream_t st);
hipError_t launch_fuse(const SceneDev& s, const SearchDev& q, int dtype, int patch,
                       const uint32_t* list, const uint32_t* list_count, hipStream_t st);
hipError_t launch_learned_refine(const SceneDev& s, const SearchDev& q, const LearnedDev& l,
                                 int dtype, int patch, int prop_by_j, hipStream_t st);

}  // namespace fd
