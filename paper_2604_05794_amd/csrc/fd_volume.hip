// fd_volume.hip -- occupancy and orientation volume from oriented points on
// gfx950 (the fused volume of Sec. 3.2, opening paragraph; the rule is
// documented with fd_fuse_volume in fusedir.h).
//
// Three launches, all bound by HBM traffic and atomics rather than
// arithmetic:
//   k_vol_clear     zero the occupancy and the fixed-point tensor sums
//                   (16-byte stores; a kernel, so the sequence can be
//                   captured in a graph);
//   k_vol_scatter   one thread per point: binary32 voxel index, one u32
//                   atomic for the occupancy, six 64-bit integer atomics for
//                   the structure tensor w d d^T, each term formed in binary64
//                   and rounded to a multiple of 2^-32.  Integer addition is
//                   associative, so the sums do not depend on the order in
//                   which the atomics land: the volume is deterministic;
//   k_vol_finalize  one thread per voxel: the sums back to binary64, cyclic
//                   Jacobi rotations to the top eigenvector and the
//                   coherence (l1 - l2) / l1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"
#include "fd_voxel.hpp"

using namespace fd;

namespace {

constexpr double kFix = 4294967296.0;        // 2^32 units per 1.0
constexpr double kUnfix = 1.0 / 4294967296.0;

__global__ __launch_bounds__(256) void k_vol_clear(uint4* __restrict__ acc, int64_t n16,
                                                   uint32_t* __restrict__ occ, int64_t nv) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    acc[i] = z;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride)
    occ[i] = 0u;
}

__device__ __forceinline__ unsigned long long fix(double t) {
  t = fmin(fmax(t, -1.0), 1.0);
  return (unsigned long long)__double2ll_rn(t * kFix);
}

__global__ __launch_bounds__(256) void k_vol_scatter(const float* __restrict__ points,
                                                     const float* __restrict__ dirs,
                                                     const float* __restrict__ weights, int64_t n,
                                                     GridDev g,
                                                     unsigned long long* __restrict__ acc,
                                                     uint32_t* __restrict__ occ) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = voxel_index(g, points[3 * i], points[3 * i + 1], points[3 * i + 2]);
  if (v < 0) return;
  atomicAdd(&occ[v], 1u);
  float w = weights ? weights[i] : 1.0f;
  w = w > 0.0f ? fminf(w, 1.0f) : 0.0f;  // NaN and negatives count as 0
  const double dx = dirs[3 * i], dy = dirs[3 * i + 1], dz = dirs[3 * i + 2];
  if (w == 0.0f || (dx == 0.0 && dy == 0.0 && dz == 0.0)) return;
  const double wd = (double)w;
  unsigned long long* T = acc + 6 * v;
  atomicAdd(T + 0, fix(wd * dx * dx));
  atomicAdd(T + 1, fix(wd * dy * dy));
  atomicAdd(T + 2, fix(wd * dz * dz));
  atomicAdd(T + 3, fix(wd * dx * dy));
  atomicAdd(T + 4, fix(wd * dx * dz));
  atomicAdd(T + 5, fix(wd * dy * dz));
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

__global__ __launch_bounds__(256) void k_vol_finalize(const long long* __restrict__ acc,
                                                      const uint32_t* __restrict__ occ,
                                                      int64_t nv, float* __restrict__ dir_out,
                                                      float* __restrict__ coh_out,
                                                      double* __restrict__ tensor_out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double T[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  bool any = false;
  if (occ[v] != 0u) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const long long x = acc[6 * v + k];
      any |= x != 0;
      T[k] = (double)x * kUnfix;
    }
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
      const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
      const double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
      if (off == 0.0 || off <= 1e-36 * dg) break;
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
  if ((r = ctx_buffer((void**)&c->vol_acc, &c->cap_vol_acc, sizeof(long long) * 6 * (size_t)nv,
                      "volume sums")))
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
    const int64_t n16 = 3 * nv;  // 48 bytes of sums per voxel
    const int64_t nb = (n16 + 255) / 256;
    hipLaunchKernelGGL(k_vol_clear, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(256), 0, st,
                       (uint4*)c->vol_acc, n16, occ_out, nv);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume clear");
    t.stop();
  }
  if (n_points > 0) {
    StageTimer t(c, FD_STAGE_VOLUME_SCATTER, st);
    hipLaunchKernelGGL(k_vol_scatter, dim3((unsigned)((n_points + 255) / 256)), dim3(256), 0, st,
                       points, dirs, weights, n_points, g, (unsigned long long*)c->vol_acc,
                       occ_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume scatter");
    t.stop();
  }
  {
    StageTimer t(c, FD_STAGE_VOLUME_FINAL, st);
    hipLaunchKernelGGL(k_vol_finalize, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st,
                       (const long long*)c->vol_acc, occ_out, nv, dir_out, coherence_out,
                       tensor_out);
    if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "volume finalize");
    t.stop();
  }
  return FD_OK;
}
