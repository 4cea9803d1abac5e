// fd_batched.hip -- many scenes (uneven point counts, view counts and map
// sizes) fused by one captured launch sequence on gfx950.
//
// All scenes share one concatenated point range; a scene table (one SceneDev
// per scene, its per-point workspace pointers offset to the scene's range)
// lets every kernel find its scene: per-point kernels from a block table
// (blocks never straddle scenes), the search kernels by a binary search of
// the point offsets per lane group.  The searches (plain, learned, fallback)
// have a persistent form: a grid sized to what stays resident pops tiles of
// points from XCD-blocked atomic queues until they are empty, so uneven
// scenes balance across the compute units; the autotuner picks it or one
// wave per tile.  The sequence (tiling, view selection, [features,
// network, refinement,] search) is captured once into a HIP graph and
// replayed while the scene set and the parameters stay the same.  Every
// point runs the same per-point code as a single-scene call, so results are
// bit-identical to fd_fuse_directions on each scene.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_features.hpp"
#include "fd_kernels.hpp"
#include "fd_search.hpp"

using namespace fd;

namespace fd {
int mlp_forward_dev(const fd_mlp* m, const uint16_t* feats, int64_t n, float* out, hipStream_t st);
}

namespace {

constexpr int kBCellBits = 6;  // per axis: 64^3 cells per scene (as one scene's tiling)
constexpr int kBCells = 1 << (3 * kBCellBits);
constexpr int kBlock = 256;

struct BatchDev {
  const SceneDev* tab;     // n_scenes
  const int64_t* pt_off;   // n_scenes + 1, global point offsets
  const int64_t* blk_off;  // n_scenes + 1, first 256-thread block of each scene
  const int64_t* tile_off; // n_scenes + 1, first search tile (G points) of each scene
  int n_scenes;
  int64_t total;
  int64_t n_tiles;         // tile_off[n_scenes]
};

constexpr int kQueues = 8;  // one tile range and queue per XCD

// largest s with off[s] <= x (off ascending, off[0] = 0)
__device__ __forceinline__ int find_scene(const int64_t* off, int n, int64_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int float_to_ordered(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float ordered_to_float(int i) {
  return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff);
}

// per-scene point index of this thread (block table), or -1; `blk` is the
// logical block index (blockIdx.x, or its XCD-aware remapping)
__device__ __forceinline__ int64_t block_point(const BatchDev& b, int* scene,
                                               int64_t blk = -1) {
  if (blk < 0) blk = blockIdx.x;
  const int s = find_scene(b.blk_off, b.n_scenes, blk);
  *scene = s;
  const int64_t j = (blk - b.blk_off[s]) * blockDim.x + threadIdx.x;
  return j < b.tab[s].n ? j : -1;
}

// The bounding boxes are folded through kBboxRep copies per scene (workgroup
// w updates copy w % kBboxRep): an atomic on an address that every workgroup
// of a scene updates is serialised in memory, about 0.14 us each, which made
// this stage 137 us for 2M points.  k_b_bbox_final folds the copies.
constexpr int kBboxRep = 64;

__global__ void k_b_init(uint32_t* counts, int64_t n_counts, int* rep, int n_scenes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n_counts; k += stride) counts[k] = 0u;
  for (int64_t k = i; k < (int64_t)6 * kBboxRep * n_scenes; k += stride)
    rep[k] = (k % 6) < 3 ? INT32_MAX : INT32_MIN;
}

__global__ void k_b_bbox_final(const int* __restrict__ rep, int n_scenes,
                               int* __restrict__ bbox) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= 6 * n_scenes) return;
  const int s = i / 6, a = i - 6 * s;
  const int* r = rep + (size_t)s * kBboxRep * 6 + a;
  int v = r[0];
  for (int k = 1; k < kBboxRep; ++k) v = a < 3 ? min(v, r[6 * k]) : max(v, r[6 * k]);
  bbox[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_b_bbox(BatchDev b, int* __restrict__ rep) {
  __shared__ int red[kBlock / 64][6];
  int s;
  const int64_t j = block_point(b, &s);
  int v[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
  if (j >= 0) {
    const float* p = b.tab[s].pts + 3 * j;
    for (int a = 0; a < 3; ++a) {
      const float f = p[a];
      if (f == f) {
        v[a] = float_to_ordered(f);
        v[3 + a] = v[a];
      }
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int off = 32; off > 0; off >>= 1) {
      v[a] = min(v[a], __shfl_xor(v[a], off, 64));
      v[3 + a] = max(v[3 + a], __shfl_xor(v[3 + a], off, 64));
    }
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 6; ++a) red[threadIdx.x >> 6][a] = v[a];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    int r = red[0][a];
    for (int k = 1; k < kBlock / 64; ++k) r = a < 3 ? min(r, red[k][a]) : max(r, red[k][a]);
    int* dst = rep + ((size_t)s * kBboxRep + blockIdx.x % kBboxRep) * 6 + a;
    if (a < 3)
      atomicMin(dst, r);
    else
      atomicMax(dst, r);
  }
}

__device__ __forceinline__ uint32_t spread3_b(uint32_t x) {
  uint32_t r = 0;
  for (int k = 0; k < kBCellBits; ++k) r |= ((x >> k) & 1u) << (3 * k);
  return r;
}

__global__ __launch_bounds__(kBlock) void k_b_count(BatchDev b, const int* __restrict__ bbox,
                                                    uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ counts) {
  int s;
  const int64_t j = block_point(b, &s);
  if (j < 0) return;
  const float* p = b.tab[s].pts + 3 * j;
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    const float lo = ordered_to_float(bbox[6 * s + a]), hi = ordered_to_float(bbox[6 * s + 3 + a]);
    const float f = p[a];
    const float ext = hi - lo;
    const float u = ext > 0.0f ? (f - lo) / ext : 0.0f;
    int c = (int)(u * (float)(1 << kBCellBits));
    c = (f == f) ? c : 0;
    q[a] = (uint32_t)min(max(c, 0), (1 << kBCellBits) - 1);
  }
  const uint32_t k = spread3_b(q[0]) | (spread3_b(q[1]) << 1) | (spread3_b(q[2]) << 2);
  key[b.pt_off[s] + j] = k;
  atomicAdd(&counts[(size_t)s * kBCells + k], 1u);
}

// cursor holds global positions (scenes concatenated, cells scene-major);
// perm receives the scene-local point index
__global__ __launch_bounds__(kBlock) void k_b_scatter(BatchDev b, const uint32_t* __restrict__ key,
                                                      uint32_t* __restrict__ cursor,
                                                      uint32_t* __restrict__ perm) {
  int s;
  const int64_t j = block_point(b, &s);
  if (j < 0) return;
  const uint32_t pos = atomicAdd(&cursor[(size_t)s * kBCells + key[b.pt_off[s] + j]], 1u);
  perm[pos] = (uint32_t)j;
}

template <typename T, int KS>
__global__ __launch_bounds__(kBlock) void k_b_topk(BatchDev b, SearchDev q) {
  int s;
  const int64_t j = block_point(b, &s, xcd_tile(gridDim.x));
  if (j < 0) return;
  const SceneDev sc = load_scene(b.tab, s);
  topk_point<T, KS>(sc, q, j);
}

template <typename T, int KS>
__global__ __launch_bounds__(kBlock) void k_b_topk_features(BatchDev b, SearchDev q,
                                                            uint16_t* __restrict__ feats) {
  int s;
  const int64_t j = block_point(b, &s, xcd_tile(gridDim.x));
  if (j < 0) return;
  const SceneDev sc = load_scene(b.tab, s);
  topk_features_point<T, KS>(sc, q, j, b.pt_off[s], feats);
}

// The same for batches whose scenes have at most kMaskViews views, in two
// kernels (view selection with the visibility bits, then the frontal
// ranking and the row); a workgroup's points belong to one scene, whose
// camera records both read at wave-uniform addresses, through the scalar
// cache.  The first is held to five waves per SIMD (96 registers: two
// spilled) for its gather loop: at four it measured 0.18 ms slower on 2M
// points of 128 views.
template <typename T, int KS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(KS <= 5 ? 5 : 4)))
void k_b_vis_m(BatchDev b, SearchDev q, uint16_t* __restrict__ feats) {
  int s;
  const int64_t j = block_point(b, &s, xcd_tile(gridDim.x));
  if (j < 0) return;
  const SceneDev sc = load_scene(b.tab, s);
  vis_topk_masked<T, KS, kMaskViews / 32>(sc, q, sc.cam64, j, b.pt_off[s] + j, feats);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_b_frontal_row_m(BatchDev b,
                                                            uint16_t* __restrict__ feats) {
  int s;
  const int64_t j = block_point(b, &s, xcd_tile(gridDim.x));
  if (j < 0) return;
  const SceneDev sc = load_scene(b.tab, s);
  frontal_row_masked<T, kMaskViews / 32>(sc, sc.cam64, j, b.pt_off[s] + j, feats);
}

// Persistent search.  Without a list, the items are the scenes' points in
// tiles of G that never straddle a scene (tile_off), so a wave's scene is
// uniform and its record is read through the scalar cache; with a list
// (n_items = *list_count global point positions) each lane finds its own
// scene.  Tiles are dealt to kQueues queues, one per XCD (workgroups go to the
// XCDs round-robin), in blocks of kQueueRun consecutive tiles: queue x owns
// blocks x, x + kQueues, ...  Neighbouring tiles, which share most patch
// texels, are then searched under one L2 while all XCDs move through the
// (spatially sorted) tiles together.  A wave pops `chunk` tiles at a time from
// its own queue, then from the others once it is empty; lane 0 pops and
// broadcasts, so the whole wave leaves the loop together when every queue is
// exhausted.
constexpr int64_t kQueueRun = 32;

__device__ __forceinline__ int64_t queue_tile(int qi, int64_t v) {
  return (v / kQueueRun) * (kQueueRun * kQueues) + qi * kQueueRun + (v % kQueueRun);
}

template <typename T, int P, int KT, bool LIST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_b_fuse(BatchDev b, SearchDev q, const uint32_t* list,
                                                   const uint32_t* list_count,
                                                   uint32_t* __restrict__ queue, int chunk) {
  const Group gr = make_group<KT>(q.K);
  const int64_t n_items = LIST ? (int64_t)*list_count : b.total;
  const int64_t n_tiles = LIST ? (n_items + gr.G - 1) / gr.G : b.n_tiles;
  if (n_tiles <= 0) return;  // uniform: nothing to search
  const int home = (int)(blockIdx.x % kQueues);
  for (int r = 0; r < kQueues; ++r) {
    const int qi = (home + r) % kQueues;
    // a plain read first: an exhausted queue is passed without an atomic
    if (queue_tile(qi, (int64_t)__builtin_amdgcn_readfirstlane(
                           __atomic_load_n(&queue[qi], __ATOMIC_RELAXED))) >= n_tiles)
      continue;
    for (;;) {
      uint32_t v0 = 0;
      if ((threadIdx.x & 63) == 0) v0 = atomicAdd(&queue[qi], (uint32_t)chunk);
      v0 = __builtin_amdgcn_readfirstlane(v0);
      if (queue_tile(qi, v0) >= n_tiles) break;  // tiles of a queue only increase
      for (int c = 0; c < chunk; ++c) {
        const int64_t tile = queue_tile(qi, (int64_t)v0 + c);
        if (tile >= n_tiles) break;  // uniform
        if constexpr (LIST) {
          const int64_t item = tile * gr.G + gr.g;
          const bool pt_ok = gr.lane_ok && item < n_items;
          const int64_t gpos = pt_ok ? (int64_t)list[item] : 0;
          const int s = find_scene(b.pt_off, b.n_scenes, gpos);
          const SceneDev sc = load_scene(b.tab, s);
          fuse_group<T, P, KT>(sc, q, gr, pt_ok, gpos - b.pt_off[s]);
        } else {
          const int s = find_scene(b.tile_off, b.n_scenes, tile);
          const SceneDev sc = load_scene(b.tab, s);
          const int64_t j = (tile - b.tile_off[s]) * gr.G + gr.g;
          fuse_group<T, P, KT>(sc, q, gr, gr.lane_ok && j < sc.n, j);
        }
      }
    }
  }
}

// Non-persistent form of the plain search (one wave per scene-uniform tile,
// tiles in XCD-aware block order), which the autotuner may pick instead.
template <typename T, int P, int KT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_b_fuse_tiles(BatchDev b, SearchDev q) {
  const Group gr = make_group<KT>(q.K);
  const int64_t tile = wave_tile(gridDim.x);
  if (tile >= b.n_tiles) return;
  const int s = find_scene(b.tile_off, b.n_scenes, tile);
  const SceneDev sc = load_scene(b.tab, s);
  const int64_t j = (tile - b.tile_off[s]) * gr.G + gr.g;
  fuse_group<T, P, KT>(sc, q, gr, gr.lane_ok && j < sc.n, j);
}

// One wave per scene-uniform tile, tiles in XCD-aware block order.
template <typename T, int P, int KT>
__device__ __forceinline__ void b_learned_body(const BatchDev& b, const SearchDev& q,
                                               const LearnedDev& l) {
  const Group gr = make_group<KT>(q.K);
  const int64_t tile = wave_tile(gridDim.x);
  if (tile >= b.n_tiles) return;
  const int s = find_scene(b.tile_off, b.n_scenes, tile);
  const SceneDev sc = load_scene(b.tab, s);
  const int64_t j = (tile - b.tile_off[s]) * gr.G + gr.g;
  const bool pt_ok = gr.lane_ok && j < sc.n;
  learned_group<T, P, KT>(sc, q, l, gr, pt_ok, pt_ok ? j : 0, 1, b.pt_off[s], b.pt_off[s]);
}

template <typename T, int P, int KT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_b_learned(BatchDev b, SearchDev q, LearnedDev l) {
  b_learned_body<T, P, KT>(b, q, l);
}

// Persistent form of the learned search: the same per-tile work as
// k_b_learned, tiles popped from the XCD-blocked queues as in k_b_fuse.
template <typename T, int P, int KT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_b_learned_q(BatchDev b, SearchDev q, LearnedDev l, uint32_t* __restrict__ queue,
                   int chunk) {
  const Group gr = make_group<KT>(q.K);
  const int64_t n_tiles = b.n_tiles;
  if (n_tiles <= 0) return;
  const int home = (int)(blockIdx.x % kQueues);
  for (int r = 0; r < kQueues; ++r) {
    const int qi = (home + r) % kQueues;
    if (queue_tile(qi, (int64_t)__builtin_amdgcn_readfirstlane(
                           __atomic_load_n(&queue[qi], __ATOMIC_RELAXED))) >= n_tiles)
      continue;
    for (;;) {
      uint32_t v0 = 0;
      if ((threadIdx.x & 63) == 0) v0 = atomicAdd(&queue[qi], (uint32_t)chunk);
      v0 = __builtin_amdgcn_readfirstlane(v0);
      if (queue_tile(qi, v0) >= n_tiles) break;  // tiles of a queue only increase
      for (int c = 0; c < chunk; ++c) {
        const int64_t tile = queue_tile(qi, (int64_t)v0 + c);
        if (tile >= n_tiles) break;  // uniform
        const int s = find_scene(b.tile_off, b.n_scenes, tile);
        const SceneDev sc = load_scene(b.tab, s);
        const int64_t j = (tile - b.tile_off[s]) * gr.G + gr.g;
        const bool pt_ok = gr.lane_ok && j < sc.n;
        learned_group<T, P, KT>(sc, q, l, gr, pt_ok, pt_ok ? j : 0, 1, b.pt_off[s],
                                b.pt_off[s]);
      }
    }
  }
}

template <typename T, int P, int KT>
hipError_t launch_b_search(const BatchDev& b, const SearchDev& q, const LearnedDev* l,
                           const uint32_t* list, const uint32_t* count, uint32_t* queue,
                           int chunk, int grid, hipStream_t st) {
  if (l) {
    if (grid > 0) {
      hipLaunchKernelGGL((k_b_learned_q<T, P, KT>), dim3(grid), dim3(kBlock), 0, st, b, q, *l,
                         queue, chunk);
    } else {
      const int64_t nb = (b.n_tiles + 3) / 4;  // 4 waves per block
      hipLaunchKernelGGL((k_b_learned<T, P, KT>), dim3((unsigned)nb), dim3(kBlock), 0, st, b,
                         q, *l);
    }
  } else {
    if (list)
      hipLaunchKernelGGL((k_b_fuse<T, P, KT, true>), dim3(grid), dim3(kBlock), 0, st, b, q, list,
                         count, queue, chunk);
    else if (grid <= 0)  // one wave per tile instead of the persistent queue
      hipLaunchKernelGGL((k_b_fuse_tiles<T, P, KT>), dim3((unsigned)((b.n_tiles + 3) / 4)),
                         dim3(kBlock), 0, st, b, q);
    else
      hipLaunchKernelGGL((k_b_fuse<T, P, KT, false>), dim3(grid), dim3(kBlock), 0, st, b, q,
                         list, count, queue, chunk);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_search(int patch, const BatchDev& b, const SearchDev& q, const LearnedDev* l,
                           const uint32_t* list, const uint32_t* count, uint32_t* queue,
                           int chunk, int grid, hipStream_t st) {
#define FD_B_CASE(P)                                                                   \
  return q.K == 5 ? launch_b_search<T, P, 5>(b, q, l, list, count, queue, chunk, grid, st) \
                  : launch_b_search<T, P, 0>(b, q, l, list, count, queue, chunk, grid, st);
  switch (patch) {
    case 1: FD_B_CASE(1)
    case 3: FD_B_CASE(3)
    case 5: FD_B_CASE(5)
    case 7: FD_B_CASE(7)
    default: return hipErrorInvalidValue;
  }
#undef FD_B_CASE
}

hipError_t search(int dtype, int patch, const BatchDev& b, const SearchDev& q, const LearnedDev* l,
                  const uint32_t* list, const uint32_t* count, uint32_t* queue, int chunk,
                  int grid, hipStream_t st) {
  return dtype == 1 ? dispatch_search<__half>(patch, b, q, l, list, count, queue, chunk, grid, st)
                    : dispatch_search<float>(patch, b, q, l, list, count, queue, chunk, grid, st);
}

// resident workgroups of the persistent search kernel on this device
int persistent_grid(int dtype, int patch, int per_cu_cap) {
  static int cache[2][8][2] = {};  // [dtype][patch][0 = grid]
  int& g = cache[dtype & 1][patch & 7][0];
  if (g) return per_cu_cap > 0 ? std::min(g, per_cu_cap) : g;
  int dev = 0, cus = 256, occ = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = nullptr;
#define FD_FN(T, P) (const void*)(&k_b_fuse<T, P, 5, false>)
  if (dtype == 1)
    fn = patch == 1 ? FD_FN(__half, 1) : patch == 3 ? FD_FN(__half, 3) : patch == 5 ? FD_FN(__half, 5) : FD_FN(__half, 7);
  else
    fn = patch == 1 ? FD_FN(float, 1) : patch == 3 ? FD_FN(float, 3) : patch == 5 ? FD_FN(float, 5) : FD_FN(float, 7);
#undef FD_FN
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, kBlock, 0) != hipSuccess || occ < 1)
    occ = 1;
  g = cus * occ;
  return g;
}

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

}  // namespace

// ---- workspace --------------------------------------------------------------------------

int fd::context_reserve_scenes(fd_context* c, int32_t n_scenes, int64_t total_points) {
  if (n_scenes <= 0) return FD_OK;
  if (n_scenes > FD_MAX_BATCH_SCENES)
    return set_error(FD_E_INVAL, "fd_context_reserve: at most %d scenes per batched call",
                     FD_MAX_BATCH_SCENES);
  if (c->max_scenes >= n_scenes && c->scene_tab) return FD_OK;
  auto fr = [](void* p) {
    if (p) (void)hipFree(p);
  };
  bump_workspace_generation();
  fr(c->scene_tab);
  fr(c->tile_tab);
  fr(c->tile_queue);
  fr(c->batch_key);
  fr(c->batch_perm);
  c->scene_tab = c->tile_tab = nullptr;
  c->tile_queue = c->batch_key = c->batch_perm = nullptr;
  const size_t S = (size_t)FD_MAX_BATCH_SCENES;
  hipError_t e = hipMalloc(&c->scene_tab, S * sizeof(SceneDev) + 3 * (S + 1) * sizeof(int64_t));
  // bboxes, then their kBboxRep copies per scene
  if (e == hipSuccess) e = hipMalloc(&c->tile_tab, S * 6 * (1 + kBboxRep) * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&c->tile_queue, kQueues * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&c->batch_key, S * kBCells * sizeof(uint32_t));
  // cell cursors, then the scan's run sums
  if (e == hipSuccess)
    e = hipMalloc((void**)&c->batch_perm, (S * kBCells + S * (kBCells / 1024)) * sizeof(uint32_t));
  if (e != hipSuccess) {
    c->max_scenes = 0;
    return hip_error(e, "batched workspace");
  }
  c->max_scenes = (int32_t)S;
  (void)total_points;
  return FD_OK;
}

// ---- the batched call --------------------------------------------------------------------

static int record_batch(fd_context* c, const fd_params* p, int n_scenes, int64_t total,
                        const int64_t* blk_off_host, int64_t n_tiles, const float* const* cams,
                        const int* views, const int64_t* view_off, hipStream_t st) {
  SceneDev* tab = (SceneDev*)c->scene_tab;
  int64_t* pt_off = (int64_t*)(tab + FD_MAX_BATCH_SCENES);
  int64_t* blk_off = pt_off + (FD_MAX_BATCH_SCENES + 1);
  int64_t* tile_off = blk_off + (FD_MAX_BATCH_SCENES + 1);
  BatchDev b{tab, pt_off, blk_off, tile_off, n_scenes, total, n_tiles};
  const int64_t nblocks = blk_off_host[n_scenes];
  uint32_t* counts = c->batch_key;
  uint32_t* cursor = c->batch_perm;
  uint32_t* sums = c->batch_perm + FD_MAX_BATCH_SCENES * kBCells;
  int* bbox = (int*)c->tile_tab;
  hipError_t e;
  // binary64 camera tables of every scene
  for (int s = 0; s < n_scenes; ++s)
    if ((e = launch_cams64(cams[s], views[s], c->cams64 + (size_t)kCam64 * view_off[s], st)) !=
        hipSuccess)
      return hip_error(e, "camera tables");
  // tiling
  StageTimer t_tile(c, FD_STAGE_TILING, st);
  int* rep = bbox + 6 * FD_MAX_BATCH_SCENES;
  hipLaunchKernelGGL(k_b_init, dim3(256), dim3(256), 0, st, counts, (int64_t)n_scenes * kBCells,
                     rep, n_scenes);
  hipLaunchKernelGGL(k_b_bbox, dim3((unsigned)nblocks), dim3(kBlock), 0, st, b, rep);
  hipLaunchKernelGGL(k_b_bbox_final, dim3(1), dim3(256), 0, st, rep, n_scenes, bbox);
  hipLaunchKernelGGL(k_b_count, dim3((unsigned)nblocks), dim3(kBlock), 0, st, b, bbox, c->key,
                     counts);
  if ((e = launch_scan_runs(counts, n_scenes * (kBCells / 1024), sums, cursor, st)) != hipSuccess)
    return hip_error(e, "batched scan");
  hipLaunchKernelGGL(k_b_scatter, dim3((unsigned)nblocks), dim3(kBlock), 0, st, b, c->key, cursor,
                     c->perm);
  t_tile.stop();
  double step0, lstep0;
  resolve_steps(p, &step0, &lstep0);
  const ConstsDev kc = context_consts(c);
  if ((e = launch_consts(kc, p->n_candidates, step0, lstep0, st)) != hipSuccess)
    return hip_error(e, "search constants");
  const SearchDev q = make_search(kc, p->n_candidates, p->refine_iters, p->top_k, p->z_near);
  const bool net = p->mode == FD_MODE_LEARNED && p->proposal == FD_PROPOSAL_MLP;
  if (!net) {  // the network path selects views together with its features
    StageTimer t_topk(c, FD_STAGE_TOPK, st);
    const dim3 grid((unsigned)nblocks), block(kBlock);
    const bool k5 = q.K <= 5;  // a list of 5 slots holds any top-K with K <= 5
    if (p->map_dtype == FD_F16) {
      if (k5)
        hipLaunchKernelGGL((k_b_topk<__half, 5>), grid, block, 0, st, b, q);
      else
        hipLaunchKernelGGL((k_b_topk<__half, FD_TOPK_SLOTS>), grid, block, 0, st, b, q);
    } else {
      if (k5)
        hipLaunchKernelGGL((k_b_topk<float, 5>), grid, block, 0, st, b, q);
      else
        hipLaunchKernelGGL((k_b_topk<float, FD_TOPK_SLOTS>), grid, block, 0, st, b, q);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "batched view selection");
    t_topk.stop();
  }
  const int chunk = c->tuned_chunk > 0 ? c->tuned_chunk : 2;
  // tuned_grid: 0 = the full resident grid, > 0 = at most that many
  // workgroups, < 0 = the plain search as one wave per tile (the fallback
  // list always takes the persistent form)
  const int grid = persistent_grid(p->map_dtype, p->patch, c->tuned_grid > 0 ? c->tuned_grid : 0);
  const int plain_grid = c->tuned_grid < 0 ? 0 : grid;
  uint32_t* queue = c->tile_queue;
  if (p->mode == FD_MODE_PLAIN) {
    if ((e = launch_fill_u32(queue, kQueues, 0u, st)) != hipSuccess)
      return hip_error(e, "queue reset");
    StageTimer t_fuse(c, FD_STAGE_FUSE, st);
    if ((e = search(p->map_dtype, p->patch, b, q, nullptr, nullptr, nullptr, queue, chunk,
                    plain_grid, st)) != hipSuccess)
      return hip_error(e, "batched search");
    t_fuse.stop();
    return FD_OK;
  }
  // learned
  LearnedDev l;
  l.steps = q.steps + 3 * FD_MAX_REFINE;
  l.iters = p->learned_iters;
  l.tau = (double)p->fallback_cost;
  l.fb_list = c->fb_list;
  l.fb_count = c->fb_count;
  if (net) {
    {
      StageTimer t_feat(c, FD_STAGE_FEATURES, st);
      const dim3 grid((unsigned)nblocks), block(kBlock);
      const bool k5 = q.K <= 5;
      int max_views = 0;
      for (int s = 0; s < n_scenes; ++s) max_views = views[s] > max_views ? views[s] : max_views;
      const bool m = max_views <= kMaskViews;
#define FD_B_TOPK_FEATURES(T, KS)                                                          \
  do {                                                                                     \
    if (m) {                                                                               \
      hipLaunchKernelGGL((k_b_vis_m<T, KS>), grid, block, 0, st, b, q, c->feats);           \
      hipLaunchKernelGGL((k_b_frontal_row_m<T>), grid, block, 0, st, b, c->feats);          \
    } else {                                                                               \
      hipLaunchKernelGGL((k_b_topk_features<T, KS>), grid, block, 0, st, b, q, c->feats);  \
    }                                                                                      \
  } while (0)
      if (p->map_dtype == FD_F16) {
        if (k5)
          FD_B_TOPK_FEATURES(__half, 5);
        else
          FD_B_TOPK_FEATURES(__half, FD_TOPK_SLOTS);
      } else {
        if (k5)
          FD_B_TOPK_FEATURES(float, 5);
        else
          FD_B_TOPK_FEATURES(float, FD_TOPK_SLOTS);
      }
#undef FD_B_TOPK_FEATURES
      if ((e = hipGetLastError()) != hipSuccess)
        return hip_error(e, "batched view selection + features");
      t_feat.stop();
    }
    StageTimer t_mlp(c, FD_STAGE_MLP, st);
    int r = mlp_forward_dev(p->mlp, c->feats, total, c->prop, st);
    if (r) return r;
    t_mlp.stop();
    l.proposals = c->prop;
  } else {
    // given proposals are read from each scene's own array (SceneDev::prop);
    // FD_PROPOSAL_NAN leaves that NULL, so every point falls back
    l.proposals = nullptr;
  }
  if ((e = launch_fill_u32(c->fb_count, 2, 0u, st)) != hipSuccess)
    return hip_error(e, "fallback counter reset");
  if ((e = launch_fill_u32(queue, kQueues, 0u, st)) != hipSuccess)
    return hip_error(e, "queue reset");
  StageTimer t_ref(c, FD_STAGE_REFINE, st);
  // tuned_grid < 0: one wave per tile, else the persistent queue
  if ((e = search(p->map_dtype, p->patch, b, q, &l, nullptr, nullptr, queue, chunk, plain_grid,
                  st)) != hipSuccess)
    return hip_error(e, "batched learned refinement");
  t_ref.stop();
  if ((e = launch_fill_u32(queue, kQueues, 0u, st)) != hipSuccess)
    return hip_error(e, "queue reset");
  StageTimer t_fb(c, FD_STAGE_FALLBACK, st);
  if ((e = search(p->map_dtype, p->patch, b, q, nullptr, c->fb_list, c->fb_count, queue, chunk,
                  grid, st)) != hipSuccess)
    return hip_error(e, "batched fallback search");
  t_fb.stop();
  return FD_OK;
}

extern "C" int fd_fuse_directions_batched(const fd_scene* scenes, int32_t n_scenes,
                                          const fd_params* params, fd_context* ctx) {
  const char* fn = "fd_fuse_directions_batched";
  int r;
  if ((r = check_search_params(params, fn, true))) return r;
  if (!ctx) return set_error(FD_E_INVAL, "%s: a context is required", fn);
  if (n_scenes < 0 || (n_scenes > 0 && !scenes))
    return set_error(FD_E_INVAL, "%s: bad scene array", fn);
  if (n_scenes > FD_MAX_BATCH_SCENES)
    return set_error(FD_E_INVAL, "%s: at most %d scenes per call, got %d", fn,
                     FD_MAX_BATCH_SCENES, n_scenes);
  if (params->mode == FD_MODE_FPMVO)
    return set_error(FD_E_INVAL, "%s: FD_MODE_FPMVO is not batched", fn);
  if (params->mode == FD_MODE_LEARNED && params->proposal == FD_PROPOSAL_GIVEN)
    for (int s = 0; s < n_scenes; ++s)
      if (scenes[s].n_points > 0 && !scenes[s].proposal_dirs)
        return set_error(FD_E_INVAL, "%s: FD_PROPOSAL_GIVEN needs proposal_dirs in scene %d",
                         fn, s);
  int64_t total = 0;
  const int G = 64 / params->top_k;  // points per search tile (one wave)
  std::vector<int64_t> pt_off(n_scenes + 1, 0), blk_off(n_scenes + 1, 0),
      tile_off(n_scenes + 1, 0), view_off(n_scenes + 1, 0);
  std::vector<const float*> cam_ptrs(n_scenes);
  std::vector<int> n_views(n_scenes);
  for (int s = 0; s < n_scenes; ++s) {
    const fd_scene& sc = scenes[s];
    if (sc.n_points < 0) return set_error(FD_E_INVAL, "%s: scene %d has n_points < 0", fn, s);
    if (sc.n_views < 1 || sc.n_views > FD_MAX_VIEWS)
      return set_error(FD_E_INVAL, "%s: scene %d n_views out of range", fn, s);
    if (params->top_k > sc.n_views)
      return set_error(FD_E_INVAL, "%s: scene %d has fewer views than top_k", fn, s);
    if (sc.width < 1 || sc.height < 1 || sc.width > 32768 || sc.height > 32768)
      return set_error(FD_E_INVAL, "%s: scene %d map size out of range", fn, s);
    if (sc.n_points > 0 && (!sc.points || !sc.cams || !sc.orient_maps || !sc.conf_maps ||
                            !sc.dirs || !sc.costs))
      return set_error(FD_E_INVAL, "%s: scene %d has a null pointer", fn, s);
    total += sc.n_points;
    pt_off[s + 1] = total;
    blk_off[s + 1] = blk_off[s] + (sc.n_points + kBlock - 1) / kBlock;
    tile_off[s + 1] = tile_off[s] + (sc.n_points + G - 1) / G;
    view_off[s + 1] = view_off[s] + sc.n_views;
    cam_ptrs[s] = (const float*)sc.cams;
    n_views[s] = sc.n_views;
  }
  if (total > (int64_t)UINT32_MAX) return set_error(FD_E_INVAL, "%s: too many points", fn);
  if ((r = check_device(nullptr))) return r;
  if (total == 0) return FD_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (ctx->device != dev)
    return set_error(FD_E_INVAL, "%s: context belongs to device %d", fn, ctx->device);
  if (ctx->max_points < total)
    return set_error(FD_E_NOMEM, "%s: context reserved for %lld points, call has %lld", fn,
                     (long long)ctx->max_points, (long long)total);
  if ((int64_t)(ctx->cap_cams64 / kCam64) < view_off[n_scenes])
    return set_error(FD_E_NOMEM, "%s: context reserved for %lld views, the scenes have %lld "
                     "(fd_context_reserve max_views)", fn,
                     (long long)(ctx->cap_cams64 / kCam64), (long long)view_off[n_scenes]);
  if (ctx->max_scenes < n_scenes || !ctx->scene_tab)
    return set_error(FD_E_NOMEM, "%s: context has no batched workspace (fd_context_reserve "
                     "with max_scenes)", fn);
  hipStream_t st = (hipStream_t)params->stream;
  // signature of everything the captured sequence depends on
  uint64_t sig = 1469598103934665603ull;
  sig = fnv(sig, scenes, sizeof(fd_scene) * (size_t)n_scenes);
  fd_params pc = *params;
  pc.stream = nullptr;
  sig = fnv(sig, &pc, sizeof pc);
  sig = fnv(sig, &ctx->tuned_chunk, sizeof ctx->tuned_chunk);
  sig = fnv(sig, &ctx->tuned_grid, sizeof ctx->tuned_grid);
  // the workspace pointers the table and the graph hold, and the learned
  // form's first step as resolved now (it may come from the network's
  // calibration, which the caller can change between calls)
  const uint64_t gen = workspace_generation();
  sig = fnv(sig, &gen, sizeof gen);
  double step0 = 0.0, lstep0 = 0.0;
  resolve_steps(params, &step0, &lstep0);
  sig = fnv(sig, &lstep0, sizeof lstep0);
  if (ctx->table_sig != sig) {
    // scene table (host -> device once per scene set, outside the graph)
    std::vector<SceneDev> tab(n_scenes);
    for (int s = 0; s < n_scenes; ++s) {
      const fd_scene& sc = scenes[s];
      SceneDev d{};
      d.pts = sc.points;
      d.cams = (const float*)sc.cams;
      d.theta = sc.orient_maps;
      d.conf = sc.conf_maps;
      d.depth = sc.depth_maps;
      d.cam64 = ctx->cams64 + (size_t)kCam64 * view_off[s];
      d.prop = (params->mode == FD_MODE_LEARNED && params->proposal == FD_PROPOSAL_GIVEN)
                   ? sc.proposal_dirs
                   : nullptr;
      d.vis_tau = params->vis_tau;
      d.dirs = sc.dirs;
      d.costs = sc.costs;
      d.perm = ctx->perm + pt_off[s];
      d.views = ctx->views + (size_t)FD_TOPK_SLOTS * pt_off[s];
      d.kcount = ctx->kcount + pt_off[s];
      d.n = sc.n_points;
      d.V = sc.n_views;
      d.W = sc.width;
      d.H = sc.height;
      for (int k = 0; k < 3; ++k) d.hc[k] = sc.head_centre[k];
      d.pairs = scene_pairs(params->map_dtype, sc.width, sc.orient_maps, sc.conf_maps,
                            sc.depth_maps);
      tab[s] = d;
    }
    SceneDev* dtab = (SceneDev*)ctx->scene_tab;
    int64_t* dpt = (int64_t*)(dtab + FD_MAX_BATCH_SCENES);
    int64_t* dblk = dpt + (FD_MAX_BATCH_SCENES + 1);
    int64_t* dtile = dblk + (FD_MAX_BATCH_SCENES + 1);
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(dtab, tab.data(), sizeof(SceneDev) * n_scenes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dpt, pt_off.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dblk, blk_off.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dtile, tile_off.data(), sizeof(int64_t) * (n_scenes + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "batched scene table upload");
    ctx->table_sig = sig;
  }
  StageTimer tb(ctx, FD_STAGE_BATCHED, st);
  if (ctx->profiling) {
    // stage timing: the same kernels launched directly, with events between
    // the stages (a graph would hold no event records)
    r = record_batch(ctx, params, n_scenes, total, blk_off.data(), tile_off[n_scenes],
                     cam_ptrs.data(), n_views.data(), view_off.data(), st);
    if (r) return r;
    tb.stop();
    return FD_OK;
  }
  if (!ctx->graph_exec || ctx->graph_sig != sig) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    (void)persistent_grid(params->map_dtype, params->patch, 0);  // host query, before capture
    hipError_t e;
    if (!ctx->cap_stream) {
      e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_error(e, "capture stream");
    }
    e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "hipStreamBeginCapture");
    r = record_batch(ctx, params, n_scenes, total, blk_off.data(), tile_off[n_scenes],
                     cam_ptrs.data(), n_views.data(), view_off.data(), ctx->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (r) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_error(e, "hipGraphInstantiate");
    }
    ctx->graph = g;
    ctx->graph_exec = ge;
    ctx->graph_sig = sig;
  }
  hipError_t e = hipGraphLaunch(ctx->graph_exec, st);
  if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
  tb.stop();
  return FD_OK;
}

// ---- tuning --------------------------------------------------------------------------------

struct TuneEntry {
  std::string key;
  int chunk, grid;
};

// Cache file: one JSON object {"<shape class>": {"chunk": c, "grid": g}, ...}.
static std::vector<TuneEntry> load_cache(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    int chunk = 0, grid = 0;
    if (key != "chunk" && key != "grid" &&
        sscanf(s.c_str() + end + 1, " : {\"chunk\": %d, \"grid\": %d}", &chunk, &grid) == 2)
      out.push_back({key, chunk, grid});
    pos = end + 1;
  }
  return out;
}

static void save_cache(const char* path, const std::vector<TuneEntry>& es) {
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  for (size_t i = 0; i < es.size(); ++i)
    fprintf(f, "  \"%s\": {\"chunk\": %d, \"grid\": %d}%s\n", es[i].key.c_str(), es[i].chunk,
            es[i].grid, i + 1 < es.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

static std::string shape_class(const fd_params* p, int64_t total) {
  int lg = 0;
  while ((int64_t)1 << (lg + 1) <= total) ++lg;
  char buf[96];
  snprintf(buf, sizeof buf, "P%d_K%d_%s_%s_n2e%d", p->patch, p->top_k,
           p->map_dtype == FD_F16 ? "f16" : "f32", p->mode == FD_MODE_PLAIN ? "plain" : "learned",
           lg);
  return buf;
}

extern "C" int fd_autotune(fd_context* ctx, const fd_scene* sample, int32_t n_scenes,
                           const fd_params* params, const char* cache_path) {
  const char* fn = "fd_autotune";
  int r;
  if (!ctx || !params) return set_error(FD_E_INVAL, "%s: null argument", fn);
  int64_t total = 0;
  for (int s = 0; s < n_scenes; ++s) total += sample[s].n_points;
  const std::string key = shape_class(params, total);
  std::vector<TuneEntry> cache;
  if (cache_path) {
    cache = load_cache(cache_path);
    for (const TuneEntry& t : cache)
      if (t.key == key && t.chunk > 0) {
        ctx->tuned_chunk = t.chunk;
        ctx->tuned_grid = t.grid;
        return FD_OK;
      }
  }
  hipStream_t st = (hipStream_t)params->stream;
  const int full = persistent_grid(params->map_dtype, params->patch, 0);
  const int chunks[] = {1, 2, 4, 8};
  const int grids[] = {-1, full / 2, (3 * full) / 4, full};  // -1: one wave per tile
  float best = INFINITY;
  int best_chunk = 2, best_grid = full;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return set_error(FD_E_HIP, "%s: event creation failed", fn);
  for (int ci : chunks) {
    for (int gi : grids) {
      if (gi == 0 || (gi < 0 && ci != chunks[0])) continue;  // the tile grid has no chunk
      ctx->tuned_chunk = ci;
      ctx->tuned_grid = gi;
      if ((r = fd_fuse_directions_batched(sample, n_scenes, params, ctx))) goto done;  // capture
      (void)hipEventRecord(a, st);
      for (int rep = 0; rep < 3; ++rep)
        if ((r = fd_fuse_directions_batched(sample, n_scenes, params, ctx))) goto done;
      (void)hipEventRecord(b, st);
      (void)hipEventSynchronize(b);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, a, b);
      if (ms < best) {
        best = ms;
        best_chunk = ci;
        best_grid = gi;
      }
    }
  }
  r = FD_OK;
done:
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ctx->tuned_chunk = best_chunk;
  ctx->tuned_grid = best_grid;
  if (r) return r;
  if (cache_path) {
    cache.push_back({key, best_chunk, best_grid});
    save_cache(cache_path, cache);
  }
  return FD_OK;
}

extern "C" int fd_tuned_shape(const fd_context* ctx, int32_t* chunk, int32_t* grid) {
  if (!ctx || !chunk || !grid) return set_error(FD_E_INVAL, "fd_tuned_shape: null argument");
  *chunk = ctx->tuned_chunk > 0 ? ctx->tuned_chunk : 2;
  *grid = ctx->tuned_grid;
  return FD_OK;
}

extern "C" int fd_set_tuned_shape(fd_context* ctx, int32_t chunk, int32_t grid) {
  if (!ctx) return set_error(FD_E_INVAL, "fd_set_tuned_shape: ctx is NULL");
  if (chunk < 1 || grid < -1)
    return set_error(FD_E_INVAL, "fd_set_tuned_shape: chunk >= 1 and grid >= -1 required");
  ctx->tuned_chunk = chunk;
  ctx->tuned_grid = grid;
  return FD_OK;
}
