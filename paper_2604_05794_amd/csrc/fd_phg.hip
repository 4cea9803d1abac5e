// fd_phg.hip -- parallel hair growing on gfx950: guide strands and segments
// traced through the occupancy / orientation volume with deferred occupancy
// (Sec. 3.2.1), and segment connection by the test of Eq. 13 (Sec. 3.2.2).
// The rules are documented with fd_grow_strands and fd_link_segments in
// fusedir.h.
//
// Growing: one thread per strand.  A batch of strands is one launch of
// k_grow, which reads the crossing counts as the earlier batches left them;
// the launch boundary is the batch barrier, after which k_cross adds every
// step of the batch to the count of the voxel it read (integer atomics, so
// the counts do not depend on the order of the additions).  Each step is a
// voxel lookup, four loads (count, coherence, crossings, orientation) issued
// together, and binary32 arithmetic written as fused multiply-adds in a
// fixed order: a trace is a deterministic function of its inputs.
//
// Linking: the pieces that accept a predecessor are bucketed by the cell of
// their start point (cells a little larger than d_max, hashed into 2^20
// buckets, counting sort with the library's two-level scan); each piece end
// scans the 27 cells around its own and proposes its nearest compatible
// start (then the lowest index); each start keeps its nearest proposer
// through a 64-bit atomic minimum of (squared distance bits, proposer).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"
#include "fd_voxel.hpp"

using namespace fd;

namespace {

constexpr int kBucketBits = 20;
constexpr uint32_t kBuckets = 1u << kBucketBits;
constexpr uint32_t kNoBucket = 0xffffffffu;

struct GrowDev {
  GridDev g;
  const uint32_t* occ;
  const float* dir;
  const float* coh;
  float step;
  int32_t max_steps;
  float min_coh;
  float bend_cos;
  uint32_t cap;  // 0: none
  int32_t mode;
  float centre[3];
};

__device__ __forceinline__ float dot3(const float* a, const float* b) {
  return __builtin_fmaf(a[2], b[2], __builtin_fmaf(a[1], b[1], a[0] * b[0]));
}

__global__ __launch_bounds__(256) void k_grow(GrowDev d, const float* __restrict__ seeds,
                                              const float* __restrict__ seed_dirs, int32_t b0,
                                              int32_t b1, const uint32_t* __restrict__ crossings,
                                              float* __restrict__ verts,
                                              int32_t* __restrict__ n_verts,
                                              float* __restrict__ last_dir) {
  const int32_t i = b0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= b1) return;
  float x[3] = {seeds[3 * (size_t)i], seeds[3 * (size_t)i + 1], seeds[3 * (size_t)i + 2]};
  float r[3] = {0.0f, 0.0f, 0.0f};
  if (d.mode == FD_SEED_GIVEN) {
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = seed_dirs[3 * (size_t)i + a];
  } else {
    const int64_t v = voxel_index(d.g, x[0], x[1], x[2]);
    if (v >= 0) {
      const float t[3] = {d.dir[3 * v], d.dir[3 * v + 1], d.dir[3 * v + 2]};
      const float off[3] = {x[0] - d.centre[0], x[1] - d.centre[1], x[2] - d.centre[2]};
      const bool away = !(dot3(t, off) < 0.0f);
      const float sg = (away == (d.mode == FD_SEED_AWAY)) ? 1.0f : -1.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) r[a] = sg * t[a];
    }
  }
  float* out = verts + (size_t)i * (size_t)(d.max_steps + 1) * 3;
  out[0] = x[0];
  out[1] = x[1];
  out[2] = x[2];
  int n = 1;
  for (int k = 1; k <= d.max_steps; ++k) {
    const int64_t v = voxel_index(d.g, x[0], x[1], x[2]);
    if (v < 0) break;
    const uint32_t o = d.occ[v];
    const float c0 = d.coh[v];
    const uint32_t cr = crossings[v];
    float t[3] = {d.dir[3 * v], d.dir[3 * v + 1], d.dir[3 * v + 2]};
    if (o == 0u || !(c0 >= d.min_coh)) break;
    if (d.cap > 0u && cr >= d.cap) break;
    if (t[0] == 0.0f && t[1] == 0.0f && t[2] == 0.0f) break;
    float c = dot3(t, r);
    if (c < 0.0f) {
      t[0] = -t[0];
      t[1] = -t[1];
      t[2] = -t[2];
      c = -c;
    }
    if (k > 1 && c < d.bend_cos) break;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] = __builtin_fmaf(d.step, t[a], x[a]);
      r[a] = t[a];
      out[3 * n + a] = x[a];
    }
    ++n;
  }
  n_verts[i] = n;
  const float sg = d.mode == FD_SEED_TOWARDS ? -1.0f : 1.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) last_dir[3 * (size_t)i + a] = n > 1 ? sg * r[a] : 0.0f;
}

// The deferred occupancy update of one batch: every step counts once in the
// voxel it read (the voxel of the vertex it started from).  One wave per
// strand, its lanes over the steps: the vertex reads coalesce and the
// atomics of a strand issue together.
__global__ __launch_bounds__(256) void k_cross(GridDev g, const float* __restrict__ verts,
                                               const int32_t* __restrict__ n_verts, int32_t b0,
                                               int32_t b1, int32_t stride,
                                               uint32_t* __restrict__ crossings) {
  const int lane = (int)(threadIdx.x & 63u);
  const int32_t i = b0 + (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (i >= b1) return;  // wave-uniform
  const float* p = verts + (size_t)i * (size_t)stride * 3;
  const int32_t n = n_verts[i];
  for (int k = lane; k + 1 < n; k += 64) {
    const int64_t v = voxel_index(g, p[3 * k], p[3 * k + 1], p[3 * k + 2]);
    if (v >= 0) atomicAdd(&crossings[v], 1u);
  }
}

// ---- linking -----------------------------------------------------------------

__device__ __forceinline__ int32_t cell_of(float x, float cell) {
  const float q = floorf(x / cell);
  return (int32_t)fminf(fmaxf(q, -1073741824.0f), 1073741824.0f);
}

__device__ __forceinline__ uint32_t bucket_of(int32_t cx, int32_t cy, int32_t cz) {
  return (((uint32_t)cx * 73856093u) ^ ((uint32_t)cy * 19349663u) ^ ((uint32_t)cz * 83492791u)) &
         (kBuckets - 1u);
}

__global__ __launch_bounds__(256) void k_link_hash(const float* __restrict__ starts,
                                                   const uint8_t* __restrict__ flags, int32_t n,
                                                   float cell, uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ bucket_rank) {
  const int32_t j = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= n) return;
  if ((flags[j] & 3u) != 3u) {
    bucket_rank[2 * (size_t)j] = kNoBucket;
    return;
  }
  const uint32_t b = bucket_of(cell_of(starts[3 * (size_t)j], cell),
                               cell_of(starts[3 * (size_t)j + 1], cell),
                               cell_of(starts[3 * (size_t)j + 2], cell));
  bucket_rank[2 * (size_t)j] = b;
  bucket_rank[2 * (size_t)j + 1] = atomicAdd(&counts[b], 1u);
}

__global__ __launch_bounds__(256) void k_link_place(const uint32_t* __restrict__ bucket_rank,
                                                    int32_t n, const uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ perm) {
  const int32_t j = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= n) return;
  const uint32_t b = bucket_rank[2 * (size_t)j];
  if (b == kNoBucket) return;
  perm[cursor[b] + bucket_rank[2 * (size_t)j + 1]] = (uint32_t)j;
}

__global__ __launch_bounds__(256) void k_link_propose(
    const float* __restrict__ starts, const float* __restrict__ start_dirs,
    const float* __restrict__ ends, const float* __restrict__ end_dirs,
    const uint8_t* __restrict__ flags, int32_t n, float d2max, float min_cos, float cell,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ cursor,
    const uint32_t* __restrict__ perm, int32_t* __restrict__ succ,
    unsigned long long* __restrict__ key, unsigned long long* __restrict__ best) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  succ[i] = -1;
  key[i] = ~0ull;
  if (!(flags[i] & 1u)) return;
  const float e[3] = {ends[3 * (size_t)i], ends[3 * (size_t)i + 1], ends[3 * (size_t)i + 2]};
  const float u[3] = {end_dirs[3 * (size_t)i], end_dirs[3 * (size_t)i + 1],
                      end_dirs[3 * (size_t)i + 2]};
  const int32_t cx = cell_of(e[0], cell), cy = cell_of(e[1], cell), cz = cell_of(e[2], cell);
  int32_t bj = -1;
  float bd = 0.0f;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const uint32_t b = bucket_of(cx + dx, cy + dy, cz + dz);
        const uint32_t s0 = cursor[b], s1 = s0 + counts[b];
        for (uint32_t s = s0; s < s1; ++s) {
          const int32_t j = (int32_t)perm[s];
          if (j == i) continue;
          const float* sj = starts + 3 * (size_t)j;
          const float ddx = e[0] - sj[0], ddy = e[1] - sj[1], ddz = e[2] - sj[2];
          const float d2 = __builtin_fmaf(ddz, ddz, __builtin_fmaf(ddy, ddy, ddx * ddx));
          if (!(d2 < d2max)) continue;
          if (!(dot3(u, start_dirs + 3 * (size_t)j) > min_cos)) continue;
          if (bj < 0 || d2 < bd || (d2 == bd && j < bj)) {
            bj = j;
            bd = d2;
          }
        }
      }
  if (bj < 0) return;
  const unsigned long long k = ((unsigned long long)__float_as_uint(bd) << 32) | (uint32_t)i;
  succ[i] = bj;
  key[i] = k;
  atomicMin(&best[bj], k);
}

__global__ __launch_bounds__(256) void k_link_accept(int32_t n,
                                                     const unsigned long long* __restrict__ key,
                                                     const unsigned long long* __restrict__ best,
                                                     int32_t* __restrict__ succ) {
  const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  const int32_t j = succ[i];
  if (j >= 0 && best[j] != key[i]) succ[i] = -1;
}


// ---- strands from linked pieces ------------------------------------------------
// Piece g < n_guide is guide trace g; piece n_guide + s is segment s (its
// backward trace reversed without the seed, then its forward trace).  A
// chain ends at -1, at a guide piece, or after n_guide + n_seg hops.

struct PiecesDev {
  const int32_t* gn;
  const int32_t* fn;
  const int32_t* bn;
  const int32_t* succ;
  int32_t n_guide, n_seg;
};

__global__ __launch_bounds__(256) void k_strand_len(PiecesDev P, int64_t* __restrict__ len,
                                                    int32_t* __restrict__ pieces) {
  const int32_t g = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (g >= P.n_guide) return;
  int64_t L = P.gn[g];
  int32_t np = 1;
  int32_t j = P.succ[g];
  for (int32_t hop = 0; j >= P.n_guide && j < P.n_guide + P.n_seg && hop < P.n_guide + P.n_seg;
       ++hop) {
    const int32_t sg = j - P.n_guide;
    L += (int64_t)(P.bn[sg] - 1) + P.fn[sg];
    ++np;
    j = P.succ[j];
  }
  len[g] = L;
  if (pieces) pieces[g] = np;
}

// Inclusive scan of one value per thread across a block of 1024 threads:
// within each wave by shuffles, then over the 16 wave totals.  Every thread
// of the block calls it once.
__device__ __forceinline__ int64_t block_incl_scan(int64_t x, int64_t* wsum) {
  const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int64_t y = lane < 1024 / 64 ? wsum[lane] : 0;
    for (int o = 1; o < 1024 / 64; o <<= 1) {
      const int64_t z = __shfl_up(y, o, 64);
      if (lane >= o) y += z;
    }
    if (lane < 1024 / 64) wsum[lane] = y;
  }
  __syncthreads();
  return x + (wv > 0 ? wsum[wv - 1] : 0);
}

// Exclusive scan of n entries into off (n + 1 entries, off[n] = the total)
// in one block: thread t owns a contiguous run, summed in order, and writes
// it after the block scan of the run sums.  Used on the per-block sums of
// the lengths (and on an empty list).
__global__ __launch_bounds__(1024) void k_len_scan(const int64_t* __restrict__ len, int32_t n,
                                                   int64_t* __restrict__ off) {
  __shared__ int64_t wsum[1024 / 64];
  const int t = (int)threadIdx.x;
  const int32_t per = (n + 1023) / 1024;
  const int32_t a = t * per, b = min(n, a + per);
  int64_t s = 0;
  for (int32_t i = a; i < b; ++i) s += len[i];
  const int64_t incl = block_incl_scan(s, wsum);
  if (t == 1023) off[n] = incl;
  int64_t acc = incl - s;
  for (int32_t i = a; i < b; ++i) {
    off[i] = acc;
    acc += len[i];
  }
}

// The lengths in blocks of 1024 (coalesced): each block's sum, then, once
// those are scanned, each entry's offset.
__global__ __launch_bounds__(1024) void k_len_bsum(const int64_t* __restrict__ len, int32_t n,
                                                   int64_t* __restrict__ bsum) {
  __shared__ int64_t wsum[1024 / 64];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t incl = block_incl_scan(i < n ? len[i] : 0, wsum);
  if (threadIdx.x == 1023) bsum[blockIdx.x] = incl;
}

__global__ __launch_bounds__(1024) void k_len_apply(const int64_t* __restrict__ len, int32_t n,
                                                    const int64_t* __restrict__ boff,
                                                    int64_t* __restrict__ off) {
  __shared__ int64_t wsum[1024 / 64];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t v = i < n ? len[i] : 0;
  const int64_t incl = block_incl_scan(v, wsum);
  if (i < n) off[i] = boff[blockIdx.x] + incl - v;
  if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = boff[gridDim.x];
}

__global__ __launch_bounds__(256) void k_assemble(PiecesDev P, const float* __restrict__ gv,
                                                  int32_t gs, const float* __restrict__ fv,
                                                  int32_t fs, const float* __restrict__ bv,
                                                  int32_t bs, const int64_t* __restrict__ off,
                                                  int64_t cap, float* __restrict__ out) {
  const int lane = (int)(threadIdx.x & 63u);
  const int32_t g = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (g >= P.n_guide) return;  // wave-uniform
  int64_t pos = off[g];
  auto put = [&](int64_t at, const float* src) {
    if (at < cap) {
      out[3 * at] = src[0];
      out[3 * at + 1] = src[1];
      out[3 * at + 2] = src[2];
    }
  };
  {
    const float* src = gv + (size_t)g * gs * 3;
    const int32_t n = min(max(P.gn[g], 0), gs);  // reads stay inside the trace
    for (int32_t k = lane; k < n; k += 64) put(pos + k, src + 3 * k);
    pos += n;
  }
  int32_t j = P.succ[g];
  for (int32_t hop = 0; j >= P.n_guide && j < P.n_guide + P.n_seg && hop < P.n_guide + P.n_seg;
       ++hop) {
    const int32_t sg = j - P.n_guide;
    const int32_t nb = min(max(P.bn[sg], 1), bs), nf = min(max(P.fn[sg], 0), fs);
    const float* b = bv + (size_t)sg * bs * 3;
    const float* f = fv + (size_t)sg * fs * 3;
    for (int32_t k = lane; k < nb - 1; k += 64) put(pos + k, b + 3 * (nb - 1 - k));
    pos += nb - 1;
    for (int32_t k = lane; k < nf; k += 64) put(pos + k, f + 3 * k);
    pos += nf;
    j = P.succ[j];
  }
}

int check_grid(const fd_volume_grid* grid, const char* fn, GridDev* g) {
  if (!grid) return set_error(FD_E_INVAL, "%s: grid is NULL", fn);
  if (!(grid->voxel > 0.0f) || !std::isfinite(grid->voxel))
    return set_error(FD_E_INVAL, "%s: voxel edge must be finite and > 0", fn);
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(grid->origin[a]))
      return set_error(FD_E_INVAL, "%s: grid origin must be finite", fn);
    if (grid->dims[a] < 1 || grid->dims[a] > FD_MAX_VOLUME_DIM)
      return set_error(FD_E_INVAL, "%s: dims must be in [1, %d]", fn, FD_MAX_VOLUME_DIM);
    g->o[a] = grid->origin[a];
    g->dims[a] = grid->dims[a];
  }
  if ((int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2] > FD_MAX_VOLUME_VOXELS)
    return set_error(FD_E_INVAL, "%s: too many voxels", fn);
  g->h = grid->voxel;
  return FD_OK;
}

fd_context* context_for(fd_context* ctx, const char* fn, int* err) {
  int dev = 0;
  if ((*err = check_device(&dev))) return nullptr;
  if (ctx) {
    if (ctx->device != dev) {
      *err = set_error(FD_E_INVAL, "%s: context belongs to device %d", fn, ctx->device);
      return nullptr;
    }
    return ctx;
  }
  return default_context(dev, 0, err);
}

}  // namespace

extern "C" void fd_grow_params_init(fd_grow_params* p) {
  if (!p) return;
  p->step = 1e-3f;
  p->max_steps = 200;
  p->min_coherence = 0.2f;
  p->max_bend_cos = 0.8660254f;  // 30 degrees
  p->voxel_cap = 8;
  p->batch = 4096;
  p->seed_mode = FD_SEED_GIVEN;
  p->centre[0] = p->centre[1] = p->centre[2] = 0.0f;
  p->stream = nullptr;
  p->ctx = nullptr;
}

extern "C" int fd_grow_strands(const fd_volume_grid* grid, const uint32_t* occ, const float* dir,
                               const float* coherence, const float* seeds,
                               const float* seed_dirs, int32_t n_seeds,
                               const fd_grow_params* p, uint32_t* crossings, float* verts,
                               int32_t* n_verts, float* last_dir) {
  const char* fn = "fd_grow_strands";
  int r;
  GrowDev d;
  if ((r = check_grid(grid, fn, &d.g))) return r;
  if (!p) return set_error(FD_E_INVAL, "%s: params is NULL", fn);
  if (!(p->step > 0.0f) || !std::isfinite(p->step))
    return set_error(FD_E_INVAL, "%s: step must be finite and > 0", fn);
  if (p->max_steps < 1 || p->max_steps > FD_MAX_GROW_STEPS)
    return set_error(FD_E_INVAL, "%s: max_steps must be in [1, %d]", fn, FD_MAX_GROW_STEPS);
  if (!std::isfinite(p->min_coherence) || !std::isfinite(p->max_bend_cos))
    return set_error(FD_E_INVAL, "%s: thresholds must be finite", fn);
  if (p->voxel_cap < 0 || p->batch < 1)
    return set_error(FD_E_INVAL, "%s: voxel_cap must be >= 0 and batch >= 1", fn);
  if (p->seed_mode != FD_SEED_GIVEN && p->seed_mode != FD_SEED_AWAY &&
      p->seed_mode != FD_SEED_TOWARDS)
    return set_error(FD_E_INVAL, "%s: unknown seed_mode %d", fn, p->seed_mode);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->centre[a]))
      return set_error(FD_E_INVAL, "%s: centre must be finite", fn);
  if (n_seeds < 0 || n_seeds > FD_MAX_GROW_SEEDS)
    return set_error(FD_E_INVAL, "%s: n_seeds must be in [0, %d]", fn, FD_MAX_GROW_SEEDS);
  if (!occ || !dir || !coherence || !crossings)
    return set_error(FD_E_INVAL, "%s: null volume or crossings pointer", fn);
  if (n_seeds > 0 && (!seeds || !verts || !n_verts || !last_dir))
    return set_error(FD_E_INVAL, "%s: null seed or output pointer", fn);
  if (n_seeds > 0 && p->seed_mode == FD_SEED_GIVEN && !seed_dirs)
    return set_error(FD_E_INVAL, "%s: FD_SEED_GIVEN needs seed_dirs", fn);
  fd_context* c = context_for(p->ctx, fn, &r);
  if (!c) return r;
  if (n_seeds == 0) return FD_OK;
  d.occ = occ;
  d.dir = dir;
  d.coh = coherence;
  d.step = p->step;
  d.max_steps = p->max_steps;
  d.min_coh = p->min_coherence;
  d.bend_cos = p->max_bend_cos;
  d.cap = (uint32_t)p->voxel_cap;
  d.mode = p->seed_mode;
  for (int a = 0; a < 3; ++a) d.centre[a] = p->centre[a];
  hipStream_t st = (hipStream_t)p->stream;
  hipError_t e;
  for (int32_t b0 = 0; b0 < n_seeds; b0 += p->batch) {
    const int32_t b1 = n_seeds - b0 > p->batch ? b0 + p->batch : n_seeds;
    const unsigned nb = (unsigned)((b1 - b0 + 255) / 256);
    {
      StageTimer t(c, FD_STAGE_GROW, st);
      hipLaunchKernelGGL(k_grow, dim3(nb), dim3(256), 0, st, d, seeds, seed_dirs, b0, b1,
                         crossings, verts, n_verts, last_dir);
      if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "grow");
      t.stop();
    }
    {
      StageTimer t(c, FD_STAGE_GROW_CROSS, st);
      const unsigned nbw = (unsigned)(((int64_t)(b1 - b0) * 64 + 255) / 256);
      hipLaunchKernelGGL(k_cross, dim3(nbw), dim3(256), 0, st, d.g, verts, n_verts, b0, b1,
                         p->max_steps + 1, crossings);
      if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "crossing update");
      t.stop();
    }
  }
  return FD_OK;
}

extern "C" int fd_link_segments(const float* starts, const float* start_dirs, const float* ends,
                                const float* end_dirs, const uint8_t* flags, int32_t n,
                                float max_dist, float min_cos, void* stream, fd_context* ctx,
                                int32_t* succ) {
  const char* fn = "fd_link_segments";
  int r;
  if (n < 0 || n > FD_MAX_LINK_PIECES)
    return set_error(FD_E_INVAL, "%s: n must be in [0, %d]", fn, FD_MAX_LINK_PIECES);
  if (!(max_dist > 0.0f) || !std::isfinite(max_dist) || !std::isfinite(min_cos))
    return set_error(FD_E_INVAL, "%s: max_dist must be finite and > 0, min_cos finite", fn);
  if (n > 0 && (!starts || !start_dirs || !ends || !end_dirs || !flags || !succ))
    return set_error(FD_E_INVAL, "%s: null pointer argument", fn);
  fd_context* c = context_for(ctx, fn, &r);
  if (!c) return r;
  if (n == 0) return FD_OK;
  const size_t un = (size_t)n;
  if ((r = ctx_buffer((void**)&c->link_counts, &c->cap_link_counts, 4 * (size_t)kBuckets,
                      "link buckets")) ||
      (r = ctx_buffer((void**)&c->link_cursor, &c->cap_link_cursor, 4 * (size_t)kBuckets,
                      "link offsets")) ||
      (r = ctx_buffer((void**)&c->link_sums, &c->cap_link_sums, 4 * 1024, "link run sums")) ||
      (r = ctx_buffer((void**)&c->link_bucket, &c->cap_link_bucket, 8 * un, "link slots")) ||
      (r = ctx_buffer((void**)&c->link_perm, &c->cap_link_perm, 4 * un, "link order")) ||
      (r = ctx_buffer((void**)&c->link_key, &c->cap_link_key, 8 * un, "link proposals")) ||
      (r = ctx_buffer((void**)&c->link_best, &c->cap_link_best, 8 * un, "link winners")))
    return r;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  // cells a little wider than max_dist: every start within max_dist of an
  // end lies in the 27 cells around the end's cell despite the rounding of
  // the cell division
  const float cell = max_dist * 1.001f;
  const float d2max = max_dist * max_dist;
  const unsigned nb = (unsigned)((n + 255) / 256);
  StageTimer t(c, FD_STAGE_LINK, st);
  if ((e = launch_fill_u32(c->link_counts, kBuckets, 0u, st)) != hipSuccess ||
      (e = launch_fill_u32((uint32_t*)c->link_best, 2 * (int64_t)n, 0xffffffffu, st)) !=
          hipSuccess)
    return hip_error(e, "link reset");
  hipLaunchKernelGGL(k_link_hash, dim3(nb), dim3(256), 0, st, starts, flags, n, cell,
                     c->link_counts, c->link_bucket);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "link hash");
  if ((e = launch_scan_runs(c->link_counts, (int)(kBuckets / 1024), c->link_sums,
                            c->link_cursor, st)) != hipSuccess)
    return hip_error(e, "link scan");
  hipLaunchKernelGGL(k_link_place, dim3(nb), dim3(256), 0, st, c->link_bucket, n,
                     c->link_cursor, c->link_perm);
  hipLaunchKernelGGL(k_link_propose, dim3(nb), dim3(256), 0, st, starts, start_dirs, ends,
                     end_dirs, flags, n, d2max, min_cos, cell, c->link_counts, c->link_cursor,
                     c->link_perm, succ, c->link_key, c->link_best);
  hipLaunchKernelGGL(k_link_accept, dim3(nb), dim3(256), 0, st, n, c->link_key, c->link_best,
                     succ);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "link kernels");
  t.stop();
  return FD_OK;
}

static int check_pieces(const int32_t* gn, int32_t n_guide, const int32_t* fn,
                        const int32_t* bn, int32_t n_seg, const int32_t* succ, const char* name) {
  if (n_guide < 0 || n_seg < 0 || n_guide > FD_MAX_GROW_SEEDS || n_seg > FD_MAX_GROW_SEEDS)
    return set_error(FD_E_INVAL, "%s: piece counts out of range", name);
  if (n_guide > 0 && (!gn || !succ))
    return set_error(FD_E_INVAL, "%s: null guide lengths or links", name);
  if (n_seg > 0 && (!fn || !bn))
    return set_error(FD_E_INVAL, "%s: null segment lengths", name);
  return FD_OK;
}

extern "C" int fd_strand_offsets(const int32_t* guide_n, int32_t n_guide, const int32_t* fwd_n,
                                 const int32_t* bwd_n, int32_t n_seg, const int32_t* succ,
                                 void* stream, fd_context* ctx, int64_t* offsets,
                                 int32_t* pieces) {
  const char* fn = "fd_strand_offsets";
  int r;
  if ((r = check_pieces(guide_n, n_guide, fwd_n, bwd_n, n_seg, succ, fn))) return r;
  if (!offsets) return set_error(FD_E_INVAL, "%s: offsets is NULL", fn);
  fd_context* c = context_for(ctx, fn, &r);
  if (!c) return r;
  hipStream_t st = (hipStream_t)stream;
  // lengths (n_guide), then the block sums (nb) and their offsets (nb + 1)
  const int32_t nb = (n_guide + 1023) / 1024;
  if ((r = ctx_buffer((void**)&c->strand_len, &c->cap_strand_len,
                      8 * ((size_t)n_guide + 2 * (size_t)nb + 1), "strand lengths")))
    return r;
  PiecesDev P{guide_n, fwd_n, bwd_n, succ, n_guide, n_seg};
  if (n_guide > 0) {
    int64_t* bsum = c->strand_len + n_guide;
    int64_t* boff = bsum + nb;
    hipLaunchKernelGGL(k_strand_len, dim3((unsigned)((n_guide + 255) / 256)), dim3(256), 0, st,
                       P, c->strand_len, pieces);
    hipLaunchKernelGGL(k_len_bsum, dim3((unsigned)nb), dim3(1024), 0, st, c->strand_len,
                       n_guide, bsum);
    hipLaunchKernelGGL(k_len_scan, dim3(1), dim3(1024), 0, st, bsum, nb, boff);
    hipLaunchKernelGGL(k_len_apply, dim3((unsigned)nb), dim3(1024), 0, st, c->strand_len,
                       n_guide, boff, offsets);
  } else {
    hipLaunchKernelGGL(k_len_scan, dim3(1), dim3(1024), 0, st, c->strand_len, 0, offsets);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "strand offsets");
}

extern "C" int fd_assemble_strands(const float* guide_v, const int32_t* guide_n, int32_t n_guide,
                                   int32_t g_stride, const float* fwd_v, const int32_t* fwd_n,
                                   int32_t f_stride, const float* bwd_v, const int32_t* bwd_n,
                                   int32_t b_stride, int32_t n_seg, const int32_t* succ,
                                   const int64_t* offsets, int64_t capacity, void* stream,
                                   fd_context* ctx, float* out) {
  const char* fn = "fd_assemble_strands";
  int r;
  if ((r = check_pieces(guide_n, n_guide, fwd_n, bwd_n, n_seg, succ, fn))) return r;
  if (g_stride < 1 || f_stride < 1 || b_stride < 1)
    return set_error(FD_E_INVAL, "%s: strides must be >= 1", fn);
  if (capacity < 0) return set_error(FD_E_INVAL, "%s: capacity must be >= 0", fn);
  if (n_guide > 0 && (!guide_v || !offsets || (capacity > 0 && !out)))
    return set_error(FD_E_INVAL, "%s: null pointer argument", fn);
  if (n_seg > 0 && (!fwd_v || !bwd_v))
    return set_error(FD_E_INVAL, "%s: null segment traces", fn);
  fd_context* c = context_for(ctx, fn, &r);
  if (!c) return r;
  if (n_guide == 0) return FD_OK;
  hipStream_t st = (hipStream_t)stream;
  PiecesDev P{guide_n, fwd_n, bwd_n, succ, n_guide, n_seg};
  hipLaunchKernelGGL(k_assemble, dim3((unsigned)(((int64_t)n_guide * 64 + 255) / 256)), dim3(256),
                     0, st, P, guide_v, g_stride, fwd_v, f_stride, bwd_v, b_stride, offsets,
                     capacity, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "strand assembly");
}

