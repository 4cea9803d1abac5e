// fd_volume.hip -- occupancy and orientation volume from oriented points on
// gfx950 (the fused volume of Sec. 3.2, opening paragraph; the rule is
// documented with fd_fuse_volume in fusedir.h).
//
// A counting sort of the points by voxel, then one thread per voxel:
//   k_vol_key       one thread per point: binary32 voxel index and one u32
//                   atomic on the voxel's count, whose old value is the
//                   point's rank within its voxel (the counts are the
//                   occupancy output itself);
//   k_scan_*        exclusive scan of the counts (blocks of 1024, the block
//                   sums through the library's two-level scan);
//   k_vol_place     each point to slot offset[v] + rank with its
//                   structure-tensor terms w d d^T, each formed in binary64
//                   and rounded to a multiple of 2^-32 (48 B per point);
//   k_busy_*        the busy voxels into a list, in voxel order (the same
//                   scan over busy flags; empty voxels get their outputs);
//   k_vol_reduce    one thread per busy voxel: its slots summed as 64-bit
//                   integers in registers, then cyclic Jacobi rotations to
//                   the top eigenvector and the coherence (l1 - l2) / l1.
// Integer sums do not depend on the order of the points within a voxel, so
// the volume is deterministic.  Device-scope atomics on memory shared by
// all XCDs are performed past the L2 (each one a 32-byte transaction), so
// this form issues one per point where summing in place would issue seven.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_kernels.hpp"
#include "fd_voxel.hpp"

using namespace fd;

namespace {

constexpr double kFix = 4294967296.0;        // 2^32 units per 1.0
constexpr double kUnfix = 1.0 / 4294967296.0;
constexpr uint32_t kOutside = 0xffffffffu;
constexpr int kRun = 1024;  // scan block

__device__ __forceinline__ unsigned long long fix(double t) {
  t = fmin(fmax(t, -1.0), 1.0);
  return (unsigned long long)__double2ll_rn(t * kFix);
}

__global__ __launch_bounds__(256) void k_vol_key(const float* __restrict__ points, int64_t n,
                                                 GridDev g, uint32_t* __restrict__ cnt,
                                                 uint32_t* __restrict__ key_rank) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = voxel_index(g, points[3 * i], points[3 * i + 1], points[3 * i + 2]);
  if (v < 0) {
    key_rank[2 * i] = kOutside;
    return;
  }
  key_rank[2 * i] = (uint32_t)v;
  key_rank[2 * i + 1] = atomicAdd(&cnt[v], 1u);
}

// inclusive scan of one value per thread over a block of kRun threads
__device__ __forceinline__ uint32_t run_incl_scan(uint32_t x, uint32_t* wsum) {
  const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(x, off, 64);
    if (lane >= off) x += o;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    uint32_t t = lane < kRun / 64 ? wsum[lane] : 0u;
    for (int off = 1; off < kRun / 64; off <<= 1) {
      const uint32_t o = __shfl_up(t, off, 64);
      if (lane >= off) t += o;
    }
    if (lane < kRun / 64) wsum[lane] = t;
  }
  __syncthreads();
  return x + (w > 0 ? wsum[w - 1] : 0u);
}

__global__ __launch_bounds__(kRun) void k_scan_sums(const uint32_t* __restrict__ cnt, int64_t nv,
                                                    uint32_t* __restrict__ bsum) {
  __shared__ uint32_t wsum[kRun / 64];
  const int64_t v = (int64_t)blockIdx.x * kRun + threadIdx.x;
  const uint32_t x = run_incl_scan(v < nv ? cnt[v] : 0u, wsum);
  if (threadIdx.x == kRun - 1) bsum[blockIdx.x] = x;
}

__global__ __launch_bounds__(kRun) void k_scan_apply(const uint32_t* __restrict__ cnt, int64_t nv,
                                                     const uint32_t* __restrict__ boff,
                                                     uint32_t* __restrict__ off) {
  __shared__ uint32_t wsum[kRun / 64];
  const int64_t v = (int64_t)blockIdx.x * kRun + threadIdx.x;
  const uint32_t x = v < nv ? cnt[v] : 0u;
  const uint32_t incl = run_incl_scan(x, wsum);
  if (v < nv) off[v] = boff[blockIdx.x] + incl - x;
}

// Each point to slot offset[v] + rank, with its six fixed-point terms, so
// the per-voxel sums read contiguous, independent records.
__global__ __launch_bounds__(256) void k_vol_place(const uint32_t* __restrict__ key_rank,
                                                   const float* __restrict__ dirs,
                                                   const float* __restrict__ weights, int64_t n,
                                                   const uint32_t* __restrict__ off,
                                                   longlong2* __restrict__ terms) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t v = key_rank[2 * i];
  if (v == kOutside) return;
  const uint64_t slot = (uint64_t)off[v] + key_rank[2 * i + 1];
  if (slot >= (uint64_t)n) return;
  float w = weights ? weights[i] : 1.0f;
  w = w > 0.0f ? fminf(w, 1.0f) : 0.0f;  // NaN and negatives count as 0
  const double dx = dirs[3 * i], dy = dirs[3 * i + 1], dz = dirs[3 * i + 2];
  longlong2 t0 = make_longlong2(0, 0), t1 = t0, t2 = t0;
  if (w != 0.0f && !(dx == 0.0 && dy == 0.0 && dz == 0.0)) {
    const double wd = (double)w;
    t0 = make_longlong2((long long)fix(wd * dx * dx), (long long)fix(wd * dy * dy));
    t1 = make_longlong2((long long)fix(wd * dz * dz), (long long)fix(wd * dx * dy));
    t2 = make_longlong2((long long)fix(wd * dx * dz), (long long)fix(wd * dy * dz));
  }
  terms[3 * slot] = t0;
  terms[3 * slot + 1] = t1;
  terms[3 * slot + 2] = t2;
}

// One Jacobi rotation in the (P, Q) plane of the symmetric A, accumulated
// into the columns of V (Golub and Van Loan, symmetric Schur step).
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&A)[3][3], double (&V)[3][3]) {
  const double apq = A[P][Q];
  if (apq == 0.0) return;
  const double th = (A[Q][Q] - A[P][P]) / (2.0 * apq);
  const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = A[k][P], b = A[k][Q];
    A[k][P] = c * a - s * b;
    A[k][Q] = s * a + c * b;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = A[P][k], b = A[Q][k];
    A[P][k] = c * a - s * b;
    A[Q][k] = s * a + c * b;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double a = V[k][P], b = V[k][Q];
    V[k][P] = c * a - s * b;
    V[k][Q] = s * a + c * b;
  }
}

// Busy voxels into a list in voxel order: per block of kRun voxels the
// number of busy ones, a scan of those (the library's two-level scan), then
// each block writes its busy voxels at its offset.  Empty voxels get their
// zero outputs here.
__global__ __launch_bounds__(kRun) void k_busy_sums(const uint32_t* __restrict__ cnt, int64_t nv,
                                                    uint32_t* __restrict__ bsum) {
  __shared__ uint32_t wsum[kRun / 64];
  const int64_t v = (int64_t)blockIdx.x * kRun + threadIdx.x;
  const uint32_t x = run_incl_scan(v < nv && cnt[v] != 0u ? 1u : 0u, wsum);
  if (threadIdx.x == kRun - 1) bsum[blockIdx.x] = x;
}

__global__ __launch_bounds__(kRun) void k_busy_apply(const uint32_t* __restrict__ cnt, int64_t nv,
                                                     const uint32_t* __restrict__ boff,
                                                     uint32_t* __restrict__ list,
                                                     uint32_t* __restrict__ list_count,
                                                     float* __restrict__ dir_out,
                                                     float* __restrict__ coh_out,
                                                     double* __restrict__ tensor_out) {
  __shared__ uint32_t wsum[kRun / 64];
  const int64_t v = (int64_t)blockIdx.x * kRun + threadIdx.x;
  const bool busy = v < nv && cnt[v] != 0u;
  const uint32_t incl = run_incl_scan(busy ? 1u : 0u, wsum);
  if (busy) {
    list[boff[blockIdx.x] + incl - 1u] = (uint32_t)v;
  } else if (v < nv) {
    dir_out[3 * v] = 0.0f;
    dir_out[3 * v + 1] = 0.0f;
    dir_out[3 * v + 2] = 0.0f;
    coh_out[v] = 0.0f;
    if (tensor_out) {
#pragma unroll
      for (int k = 0; k < 6; ++k) tensor_out[6 * v + k] = 0.0;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kRun - 1) *list_count = boff[blockIdx.x] + incl;
}

__global__ __launch_bounds__(256) void k_vol_reduce(const longlong2* __restrict__ terms,
                                                    int64_t n, const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ off, int64_t nv,
                                                    const uint32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ list_count,
                                                    float* __restrict__ dir_out,
                                                    float* __restrict__ coh_out,
                                                    double* __restrict__ tensor_out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)*list_count) return;
  const int64_t v = list[e];
  if (v >= nv) return;
  unsigned long long S[6] = {0ull, 0ull, 0ull, 0ull, 0ull, 0ull};
  const uint32_t c = cnt[v];
  {
    const uint64_t s0 = off[v];
    const uint64_t s1 = s0 + c < (uint64_t)n ? s0 + c : (uint64_t)n;
    for (uint64_t j = s0; j < s1; ++j) {
      const longlong2 a = terms[3 * j], b = terms[3 * j + 1], d = terms[3 * j + 2];
      S[0] += (unsigned long long)a.x;
      S[1] += (unsigned long long)a.y;
      S[2] += (unsigned long long)b.x;
      S[3] += (unsigned long long)b.y;
      S[4] += (unsigned long long)d.x;
      S[5] += (unsigned long long)d.y;
    }
  }
  double T[6];
  bool any = false;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    any |= S[k] != 0ull;
    T[k] = (double)(long long)S[k] * kUnfix;
  }
  if (tensor_out) {
#pragma unroll
    for (int k = 0; k < 6; ++k) tensor_out[6 * v + k] = T[k];
  }
  float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, coh = 0.0f;
  if (any) {
    double A[3][3] = {{T[0], T[3], T[4]}, {T[3], T[1], T[5]}, {T[4], T[5], T[2]}};
    double V[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
    for (int sweep = 0; sweep < 32; ++sweep) {
      const double od = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
      const double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
      if (od == 0.0 || od <= 1e-36 * dg) break;
      jacobi_rotate<0, 1>(A, V);
      jacobi_rotate<0, 2>(A, V);
      jacobi_rotate<1, 2>(A, V);
    }
    // largest, then second largest eigenvalue (first index wins ties)
    const double l0 = A[0][0], l1 = A[1][1], l2 = A[2][2];
    int top = 0;
    double lt = l0;
    if (l1 > lt) { top = 1; lt = l1; }
    if (l2 > lt) { top = 2; lt = l2; }
    const double lo = top == 0 ? fmax(l1, l2) : (top == 1 ? fmax(l0, l2) : fmax(l0, l1));
    double e0 = V[0][top], e1 = V[1][top], e2 = V[2][top];
    const double nr = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    e0 /= nr;
    e1 /= nr;
    e2 /= nr;
    const double key = e2 != 0.0 ? e2 : (e1 != 0.0 ? e1 : e0);
    if (key < 0.0) {
      e0 = -e0;
      e1 = -e1;
      e2 = -e2;
    }
    d0 = (float)e0;
    d1 = (float)e1;
    d2 = (float)e2;
    coh = lt > 0.0 ? (float)((lt - lo) / lt) : 0.0f;
  }
  dir_out[3 * v] = d0;
  dir_out[3 * v + 1] = d1;
  dir_out[3 * v + 2] = d2;
  coh_out[v] = coh;
}

}  // namespace

extern "C" int fd_fuse_volume(const float* points, const float* dirs, const float* weights,
                              int64_t n_points, const fd_volume_grid* grid, void* stream,
                              fd_context* ctx, uint32_t* occ_out, float* dir_out,
                              float* coherence_out, double* tensor_out) {
  const char* fn = "fd_fuse_volume";
  int r;
  if (!grid) return set_error(FD_E_INVAL, "%s: grid is NULL", fn);
  if (!(grid->voxel > 0.0f) || !std::isfinite(grid->voxel))
    return set_error(FD_E_INVAL, "%s: voxel edge must be finite and > 0", fn);
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(grid->origin[a]))
      return set_error(FD_E_INVAL, "%s: grid origin must be finite", fn);
    if (grid->dims[a] < 1 || grid->dims[a] > FD_MAX_VOLUME_DIM)
      return set_error(FD_E_INVAL, "%s: dims must be in [1, %d]", fn, FD_MAX_VOLUME_DIM);
  }
  const int64_t nv = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
  if (nv > FD_MAX_VOLUME_VOXELS)
    return set_error(FD_E_INVAL, "%s: %lld voxels, at most %lld", fn, (long long)nv,
                     (long long)FD_MAX_VOLUME_VOXELS);
  if (n_points < 0 || n_points > FD_MAX_VOLUME_POINTS)
    return set_error(FD_E_INVAL, "%s: n_points must be in [0, %lld]", fn,
                     (long long)FD_MAX_VOLUME_POINTS);
  if (n_points > 0 && (!points || !dirs))
    return set_error(FD_E_INVAL, "%s: points and dirs are required", fn);
  if (!occ_out || !dir_out || !coherence_out)
    return set_error(FD_E_INVAL, "%s: null output pointer", fn);
  int dev = 0;
  if ((r = check_device(&dev))) return r;
  fd_context* c = ctx;
  if (c) {
    if (c->device != dev)
      return set_error(FD_E_INVAL, "%s: context belongs to device %d", fn, c->device);
  } else {
    c = default_context(dev, 0, &r);
    if (!c) return r;
  }
  const int64_t nb = (nv + kRun - 1) / kRun;       // <= 2^20 scan blocks
  const int64_t runs = (nb + kRun - 1) / kRun;       // <= 1024 runs of block sums
  const size_t un = (size_t)(n_points > 0 ? n_points : 1);
  if ((r = ctx_buffer((void**)&c->vol_key, &c->cap_vol_key, 8 * un, "volume keys")) ||
      (r = ctx_buffer((void**)&c->vol_perm, &c->cap_vol_perm, 48 * un, "volume terms")) ||
      (r = ctx_buffer((void**)&c->vol_off, &c->cap_vol_off, 4 * (size_t)nv, "volume offsets")) ||
      (r = ctx_buffer((void**)&c->vol_bsum, &c->cap_vol_bsum, 4 * (size_t)(runs * kRun),
                      "volume block sums")) ||
      (r = ctx_buffer((void**)&c->vol_boff, &c->cap_vol_boff,
                      4 * (size_t)(runs * kRun + (nv < n_points ? nv : n_points) + 1),
                      "volume block offsets and busy list")) ||
      (r = ctx_buffer((void**)&c->vol_rsum, &c->cap_vol_rsum, 4 * (kRun + 1),
                      "volume run sums and list count")))
    return r;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  GridDev g;
  for (int a = 0; a < 3; ++a) {
    g.o[a] = grid->origin[a];
    g.dims[a] = grid->dims[a];
  }
  g.h = grid->voxel;
  {
    StageTimer t(c, FD_STAGE_VOLUME_CLEAR, st);
    if ((e = launch_fill_u32(occ_out, nv, 0u, st)) != hipSuccess ||
        (e = launch_fill_u32(c->vol_bsum, runs * kRun, 0u, st)) != hipSuccess)
      return hip_error(e, "volume clear");
    t.stop();
  }
  {
    StageTimer t(c, FD_STAGE_VOLUME_SCATTER, st);
    if (n_points > 0)
      hipLaunchKernelGGL(k_vol_key, dim3((unsigned)((n_points + 255) / 256)), dim3(256), 0, st,
                         points, n_points, g, occ_out, c->vol_key);
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kRun), 0, st, occ_out, nv,
                       c->vol_bsum);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume keys");
    if ((e = launch_scan_runs(c->vol_bsum, (int)runs, c->vol_rsum, c->vol_boff, st)) !=
        hipSuccess)
      return hip_error(e, "volume scan");
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kRun), 0, st, occ_out, nv,
                       c->vol_boff, c->vol_off);
    if (n_points > 0)
      hipLaunchKernelGGL(k_vol_place, dim3((unsigned)((n_points + 255) / 256)), dim3(256), 0,
                         st, c->vol_key, dirs, weights, n_points, c->vol_off,
                         (longlong2*)c->vol_perm);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume sort");
    t.stop();
  }
  {
    StageTimer t(c, FD_STAGE_VOLUME_FINAL, st);
    uint32_t* list = c->vol_boff + runs * kRun;  // after the block offsets
    uint32_t* list_count = c->vol_rsum + kRun;
    if ((e = launch_fill_u32(c->vol_bsum, runs * kRun, 0u, st)) != hipSuccess)
      return hip_error(e, "volume list reset");
    hipLaunchKernelGGL(k_busy_sums, dim3((unsigned)nb), dim3(kRun), 0, st, occ_out, nv,
                       c->vol_bsum);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume busy count");
    if ((e = launch_scan_runs(c->vol_bsum, (int)runs, c->vol_rsum, c->vol_boff, st)) !=
        hipSuccess)
      return hip_error(e, "volume busy scan");
    hipLaunchKernelGGL(k_busy_apply, dim3((unsigned)nb), dim3(kRun), 0, st, occ_out, nv,
                       c->vol_boff, list, list_count, dir_out, coherence_out, tensor_out);
    const int64_t max_busy = nv < n_points ? nv : n_points;
    if (max_busy > 0)
      hipLaunchKernelGGL(k_vol_reduce, dim3((unsigned)((max_busy + 255) / 256)), dim3(256), 0,
                         st, (const longlong2*)c->vol_perm, n_points, occ_out, c->vol_off, nv,
                         list, list_count, dir_out, coherence_out, tensor_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume reduce");
    t.stop();
  }
  return FD_OK;
}
