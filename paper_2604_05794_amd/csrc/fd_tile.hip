// fd_tile.hip -- spatial tiling of the points (gfx950).
//
// Points are grouped by a Morton-ordered cell of a 64^3 grid over their
// bounding box, so that the points one wavefront fuses together project to
// neighbouring pixels and their patch gathers share cache lines.  Cell order
// is a counting sort (histogram, exclusive scan, scatter).  The order of
// points inside one cell depends on atomic timing; nothing downstream
// depends on it, because every point is fused independently of the others.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fd_kernels.hpp"

namespace fd {

constexpr int kCellBits = 6;  // per axis
constexpr int kCells = 1 << (3 * kCellBits);

__device__ __forceinline__ int float_to_ordered(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float ordered_to_float(int i) {
  return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// bbox[0..2] = ordered min, bbox[3..5] = ordered max (pre-filled by the host
// path with INT_MAX / INT_MIN through k_fill_u32).  Grid-stride loop, then a
// wave and a workgroup reduction, so there are 6 atomics per workgroup.
__global__ __launch_bounds__(256) void k_bbox(const float* __restrict__ pts,
                                              int64_t n, int* __restrict__ bbox) {
  __shared__ int red[4][6];
  int v[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MIN, INT32_MIN, INT32_MIN};
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    for (int a = 0; a < 3; ++a) {
      float f = pts[3 * i + a];
      if (f == f) {  // skip NaN
        int o = float_to_ordered(f);
        v[a] = min(v[a], o);
        v[3 + a] = max(v[3 + a], o);
      }
    }
  }
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      v[a] = min(v[a], __shfl_xor(v[a], off, 64));
      v[3 + a] = max(v[3 + a], __shfl_xor(v[3 + a], off, 64));
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 6; ++a) red[w][a] = v[a];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int a = threadIdx.x;
    int r = red[0][a];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
      r = a < 3 ? min(r, red[k][a]) : max(r, red[k][a]);
    if (a < 3)
      atomicMin(&bbox[a], r);
    else
      atomicMax(&bbox[a], r);
  }
}

__device__ __forceinline__ uint32_t spread3(uint32_t x) {
  // 6-bit x -> bits at positions 0, 3, 6, ...
  uint32_t r = 0;
  for (int b = 0; b < kCellBits; ++b) r |= ((x >> b) & 1u) << (3 * b);
  return r;
}

__global__ __launch_bounds__(256) void k_cell_count(const float* __restrict__ pts,
                                                    int64_t n, const int* __restrict__ bbox,
                                                    uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ counts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t q[3];
  for (int a = 0; a < 3; ++a) {
    float lo = ordered_to_float(bbox[a]), hi = ordered_to_float(bbox[3 + a]);
    float f = pts[3 * i + a];
    float ext = hi - lo;
    float s = ext > 0.0f ? (f - lo) / ext : 0.0f;
    int c = (int)(s * (float)(1 << kCellBits));
    c = (f == f) ? c : 0;
    q[a] = (uint32_t)min(max(c, 0), (1 << kCellBits) - 1);
  }
  uint32_t k = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  key[i] = k;
  atomicAdd(&counts[k], 1u);
}

// Exclusive scan of the kCells counts in two passes: k_cell_block_sums
// reduces each run of 1024 cells; k_cell_scan scans those sums and then its
// own run, writing the cell start offsets into `cursor` (the scatter
// advances them).  Both read coalesced.
constexpr int kScanRun = 1024;
constexpr int kScanRuns = kCells / kScanRun;  // 256

__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  if (w == 0) {
    uint32_t s = lane < nw ? wsum[lane] : 0u;
    for (int off = 1; off < 16; off <<= 1) {
      uint32_t o = __shfl_up(s, off, 64);
      if (lane >= off) s += o;
    }
    if (lane < nw) wsum[lane] = s;
  }
  __syncthreads();
  return v + (w > 0 ? wsum[w - 1] : 0u);
}

__global__ __launch_bounds__(1024) void k_cell_block_sums(const uint32_t* __restrict__ counts,
                                                          uint32_t* __restrict__ sums) {
  __shared__ uint32_t wsum[16];
  uint32_t v = counts[blockIdx.x * kScanRun + threadIdx.x];
  uint32_t incl = block_incl_scan(v, wsum);
  if (threadIdx.x == kScanRun - 1) sums[blockIdx.x] = incl;
}

__global__ __launch_bounds__(1024) void k_cell_scan(const uint32_t* __restrict__ counts,
                                                    const uint32_t* __restrict__ sums,
                                                    uint32_t* __restrict__ cursor) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t base;
  // prefix of the run sums before this block (kScanRuns <= 1024)
  uint32_t s = threadIdx.x < (unsigned)blockIdx.x ? sums[threadIdx.x] : 0u;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) b += wsum[k];
    base = b;
  }
  __syncthreads();
  const uint32_t b = base;
  __syncthreads();
  uint32_t v = counts[blockIdx.x * kScanRun + threadIdx.x];
  uint32_t incl = block_incl_scan(v, wsum);
  cursor[blockIdx.x * kScanRun + threadIdx.x] = b + incl - v;
}

__global__ __launch_bounds__(256) void k_cell_scatter(const uint32_t* __restrict__ key,
                                                      int64_t n,
                                                      uint32_t* __restrict__ cursor,
                                                      uint32_t* __restrict__ perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t pos = atomicAdd(&cursor[key[i]], 1u);
  perm[pos] = (uint32_t)i;
}

__global__ void k_iota(uint32_t* __restrict__ perm, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) perm[i] = (uint32_t)i;
}

hipError_t launch_tiling(const float* pts, int64_t n, TileWork w, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  const int64_t nb = (n + bs - 1) / bs;
  // bbox <- (INT_MAX x3, INT_MIN x3), counts <- 0, through fill kernels so
  // the sequence stays valid under stream capture
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)w.bbox, (int64_t)3,
                     (uint32_t)INT32_MAX);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t*)(w.bbox + 3),
                     (int64_t)3, (uint32_t)INT32_MIN);
  hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, st, w.counts, (int64_t)kCells, 0u);
  int gb = (int)(nb < 256 ? nb : 256);
  hipLaunchKernelGGL(k_bbox, dim3(gb), dim3(bs), 0, st, pts, n, w.bbox);
  hipLaunchKernelGGL(k_cell_count, dim3((unsigned)nb), dim3(bs), 0, st, pts, n, w.bbox,
                     w.key, w.counts);
  hipLaunchKernelGGL(k_cell_block_sums, dim3(kScanRuns), dim3(kScanRun), 0, st, w.counts,
                     w.sums);
  hipLaunchKernelGGL(k_cell_scan, dim3(kScanRuns), dim3(kScanRun), 0, st, w.counts, w.sums,
                     w.cursor);
  hipLaunchKernelGGL(k_cell_scatter, dim3((unsigned)nb), dim3(bs), 0, st, w.key, n, w.cursor,
                     w.perm);
  return hipGetLastError();
}

// Exclusive scan in place of the n run sums (one block; each thread scans
// a chunk of at most kMaxRunsPerThread consecutive sums).
constexpr int kMaxRunsPerThread = 16;
__global__ __launch_bounds__(1024) void k_run_scan(uint32_t* __restrict__ sums, int n) {
  __shared__ uint32_t wsum[16];
  const int per = (n + kScanRun - 1) / kScanRun;
  const int r0 = threadIdx.x * per;
  uint32_t loc = 0;
  for (int k = 0; k < per; ++k)
    if (r0 + k < n) loc += sums[r0 + k];
  uint32_t run = block_incl_scan(loc, wsum) - loc;
  for (int k = 0; k < per; ++k)
    if (r0 + k < n) {
      const uint32_t v = sums[r0 + k];
      sums[r0 + k] = run;
      run += v;
    }
}

// Run r's cell starts: its exclusive prefix (sums[r]) plus the scan within
// the run.
__global__ __launch_bounds__(1024) void k_cell_scan_from(const uint32_t* __restrict__ counts,
                                                         const uint32_t* __restrict__ sums,
                                                         uint32_t* __restrict__ cursor) {
  __shared__ uint32_t wsum[16];
  const uint32_t b = sums[blockIdx.x];
  const uint32_t v = counts[(size_t)blockIdx.x * kScanRun + threadIdx.x];
  const uint32_t incl = block_incl_scan(v, wsum);
  cursor[(size_t)blockIdx.x * kScanRun + threadIdx.x] = b + incl - v;
}

// Exclusive scan of n_runs x 1024 counts (n_runs <= 16384) into cursor, in
// three passes: run sums, their scan, the runs; `sums` (n_runs entries)
// ends up holding each run's exclusive prefix.
hipError_t launch_scan_runs(const uint32_t* counts, int n_runs, uint32_t* sums, uint32_t* cursor,
                            hipStream_t st) {
  if (n_runs < 1 || n_runs > kScanRun * kMaxRunsPerThread) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cell_block_sums, dim3(n_runs), dim3(kScanRun), 0, st, counts, sums);
  hipLaunchKernelGGL(k_run_scan, dim3(1), dim3(kScanRun), 0, st, sums, n_runs);
  hipLaunchKernelGGL(k_cell_scan_from, dim3(n_runs), dim3(kScanRun), 0, st, counts, sums,
                     cursor);
  return hipGetLastError();
}

hipError_t launch_identity_perm(int64_t n, uint32_t* perm, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, st, p,
                     n, v);
  return hipGetLastError();
}

int tile_cells() { return kCells; }

}  // namespace fd
