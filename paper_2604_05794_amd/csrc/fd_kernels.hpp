// fd_kernels.hpp -- internal interface between the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
  int64_t n;
  int V, W, H;
  float hc[3];          // head centre (frontal ranking)
  float vis_tau;        // visibility tolerance on |Z - D|
};

struct SearchDev {
  const float* lattice;  // n_candidates x 3
  int n_candidates;
  int refine_iters;
  float step0;
  int K;
  float z_near;
};

// Learned form (fd_learned.hip).
struct LearnedDev {
  const float* proposals;  // n x 3 in point order, or NULL for NaN proposals
  int iters;
  float step0;
  float tau;
  uint32_t* fb_list;       // processing-order indices that fall back
  uint32_t* fb_count;      // 1 counter
};

hipError_t launch_tiling(const float* pts, int64_t n, TileWork w, hipStream_t st);
hipError_t launch_identity_perm(int64_t n, uint32_t* perm, hipStream_t st);
hipError_t launch_scan_runs(const uint32_t* counts, int n_runs, uint32_t* sums, uint32_t* cursor,
                            hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
int tile_cells();

hipError_t launch_lattice(float* lattice, int n, hipStream_t st);
hipError_t launch_topk(const SceneDev& s, const SearchDev& q, int dtype, hipStream_t st);
hipError_t launch_fuse(const SceneDev& s, const SearchDev& q, int dtype, int patch,
                       const uint32_t* list, const uint32_t* list_count, hipStream_t st);
hipError_t launch_learned_refine(const SceneDev& s, const SearchDev& q, const LearnedDev& l,
                                 int dtype, int patch, int prop_by_j, hipStream_t st);

}  // namespace fd
