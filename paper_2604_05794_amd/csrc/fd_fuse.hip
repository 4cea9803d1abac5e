// fd_fuse.hip -- direction fusion kernels for gfx950.
//
// EfficientMonoHair, Sec. 3.1.  Per point: the K most confident eligible
// views (Eq. 4), a P x P patch of bilinear doubled-angle samples around the
// projection in each of them, and the objective
//   J(d) = 1 - (1/K_eff) sum_v max_p C_p |cos(phi_v(d) - theta_p)|
// (Eqs. 8-11: phi_v(d) is the image angle of the tangent d, the maximum runs
// over the patch, the views are averaged), minimised over a hemisphere
// Fibonacci lattice (Eq. 12) and refined by a six-direction pattern search.
//
// Mapping onto the hardware.  A wavefront fuses floor(64 / K) points; the K
// lanes of a point each own one selected view and keep that view's patch in
// registers as quadratic-form coefficients
//   (a, b, c) = C^2/2 * (1, cos 2theta, sin 2theta),
// so that for an image direction r with n2 = |r|^2,
//   C^2 cos^2(phi - theta) = a + b (rx^2 - ry^2)/n2 + c (2 rx ry)/n2,
// and the patch maximum costs two FMAs and half a max3 per sample.  The view
// sum of a candidate is a fixed-order shuffle sum over the point's K lanes,
// so all K lanes hold bit-identical J and take the same argmin decisions
// without any synchronisation.  Candidates are wave-uniform (scalar loads).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fd_device.hpp"
#include "fd_kernels.hpp"
#include "fd_search.hpp"

namespace fd {

// ---- per-call constants -------------------------------------------------------
// Hemisphere Fibonacci lattice (Gonzalez 2010): z_k = 1 - (k + 1/2)/n,
// psi_k = k pi (3 - sqrt 5), in binary64 and rounded to binary32 for the
// lattice stage.  Refinement steps alpha_t = step0 / 2^t (exact halvings) with
// their cosines, sines and cosines minus one, for the plain search and for
// the learned form's short refinement.
__global__ void k_consts(ConstsDev c, int n, double step0, double lstep0) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const double golden = 3.14159265358979323846 * (3.0 - sqrt(5.0));
    const double z = 1.0 - ((double)k + 0.5) / (double)n;
    const double rho = sqrt(fmax(0.0, 1.0 - z * z));
    const double psi = golden * (double)k;
    const double x = rho * cos(psi), y = rho * sin(psi);
    c.lattice64[3 * k] = x;
    c.lattice64[3 * k + 1] = y;
    c.lattice64[3 * k + 2] = z;
    c.lattice[3 * k] = (float)x;
    c.lattice[3 * k + 1] = (float)y;
    c.lattice[3 * k + 2] = (float)z;
  }
  if (k < 2 * FD_MAX_REFINE) {
    const int t = k % FD_MAX_REFINE;
    const double a = (k < FD_MAX_REFINE ? step0 : lstep0) * ldexp(1.0, -t);
    double* dst = c.steps + (k < FD_MAX_REFINE ? 0 : 3 * FD_MAX_REFINE);
    const double h = sin(0.5 * a);
    dst[t] = cos(a);
    dst[FD_MAX_REFINE + t] = sin(a);
    dst[2 * FD_MAX_REFINE + t] = -2.0 * h * h;  // cos a - 1 without cancellation
  }
}

hipError_t launch_consts(const ConstsDev& c, int n, double step0, double lstep0, hipStream_t st) {
  const int m = n > 2 * FD_MAX_REFINE ? n : 2 * FD_MAX_REFINE;
  hipLaunchKernelGGL(k_consts, dim3((m + 255) / 256), dim3(256), 0, st, c, n, step0, lstep0);
  return hipGetLastError();
}

// ---- per-call camera table ----------------------------------------------------
__global__ void k_cams64(const float* __restrict__ cams, int V, double* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const float* c = cams + 16 * v;
  const double fx = c[0], fy = c[1], cx = c[2], cy = c[3];
  const float* R = c + 4;
  const float* t = c + 13;
  double* o = out + (size_t)kCam64 * v;
  for (int k = 0; k < 3; ++k) {
    o[k] = fx * (double)R[k] + cx * (double)R[6 + k];
    o[4 + k] = fy * (double)R[3 + k] + cy * (double)R[6 + k];
    o[8 + k] = (double)R[6 + k];
  }
  o[3] = fx * (double)t[0] + cx * (double)t[2];
  o[7] = fy * (double)t[1] + cy * (double)t[2];
  o[11] = (double)t[2];
  for (int k = 0; k < 3; ++k)
    o[12 + k] = -((double)R[k] * t[0] + (double)R[3 + k] * t[1] + (double)R[6 + k] * t[2]);
  o[15] = 0.0;
  for (int k = 0; k < 8; ++k)
    o[kCam32Off + k] = __builtin_bit_cast(double, make_float2(c[2 * k], c[2 * k + 1]));
}

hipError_t launch_cams64(const float* cams, int V, double* out, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cams64, dim3((V + 127) / 128), dim3(128), 0, st, cams, V, out);
  return hipGetLastError();
}

SearchDev make_search(const ConstsDev& c, int n_candidates, int refine_iters, int K,
                      float z_near) {
  SearchDev q;
  q.lattice = c.lattice;
  q.lattice64 = c.lattice64;
  q.steps = c.steps;
  q.n_candidates = n_candidates;
  q.refine_iters = refine_iters;
  q.K = K;
  q.z_near = (double)z_near;
  return q;
}

template <typename T, int KS>
__global__ __launch_bounds__(256) void k_topk(SceneDev s, SearchDev q) {
  const int64_t j = xcd_tile(gridDim.x) * blockDim.x + threadIdx.x;
  if (j >= s.n) return;
  topk_point<T, KS>(s, q, j);
}

hipError_t launch_topk(const SceneDev& s, const SearchDev& q, int dtype, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  dim3 grid((unsigned)((s.n + 255) / 256));
  const bool k5 = q.K <= 5;  // a list of 5 slots holds any top-K with K <= 5
  if (dtype == 1) {
    if (k5)
      hipLaunchKernelGGL((k_topk<__half, 5>), grid, dim3(256), 0, st, s, q);
    else
      hipLaunchKernelGGL((k_topk<__half, FD_TOPK_SLOTS>), grid, dim3(256), 0, st, s, q);
  } else {
    if (k5)
      hipLaunchKernelGGL((k_topk<float, 5>), grid, dim3(256), 0, st, s, q);
    else
      hipLaunchKernelGGL((k_topk<float, FD_TOPK_SLOTS>), grid, dim3(256), 0, st, s, q);
  }
  return hipGetLastError();
}

// ---- plain search: lattice argmin + refinement ---------------------------------
// `list` (optional): processing-order indices to fuse, *list_count of them
// (read on the device; the grid is sized for the worst case).
template <typename T, int P, int KT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_fuse(SceneDev s, SearchDev q, const uint32_t* list, const uint32_t* list_count) {
  const Group gr = make_group<KT>(q.K);
  const int64_t wave = wave_tile(gridDim.x);
  const int64_t t = wave * gr.G + gr.g;
  const int64_t limit = list ? (int64_t)*list_count : s.n;
  if (wave * gr.G >= limit) return;  // whole wave idle (uniform exit)
  const bool pt_ok = gr.lane_ok && t < limit;
  const int64_t j = pt_ok ? (list ? (int64_t)list[t] : t) : 0;
  fuse_group<T, P, KT>(s, q, gr, pt_ok, j);
}

template <typename T>
static hipError_t launch_fuse_t(const SceneDev& s, const SearchDev& q, int patch,
                                const uint32_t* list, const uint32_t* list_count,
                                hipStream_t st) {
  const int G = kWave / q.K;
  const int64_t pts_per_block = 4 * (int64_t)G;
  const int64_t nb = (s.n + pts_per_block - 1) / pts_per_block;
  if (nb <= 0) return hipSuccess;
  dim3 grid((unsigned)nb), block(256);
#define FD_FUSE_CASE(P)                                                                  \
  if (q.K == 5)                                                                          \
    hipLaunchKernelGGL((k_fuse<T, P, 5>), grid, block, 0, st, s, q, list, list_count);    \
  else                                                                                   \
    hipLaunchKernelGGL((k_fuse<T, P, 0>), grid, block, 0, st, s, q, list, list_count);
  switch (patch) {
    case 1: FD_FUSE_CASE(1) break;
    case 3: FD_FUSE_CASE(3) break;
    case 5: FD_FUSE_CASE(5) break;
    case 7: FD_FUSE_CASE(7) break;
    default: return hipErrorInvalidValue;
  }
#undef FD_FUSE_CASE
  return hipGetLastError();
}

hipError_t launch_fuse(const SceneDev& s, const SearchDev& q, int dtype, int patch,
                       const uint32_t* list, const uint32_t* list_count, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  return dtype == 1 ? launch_fuse_t<__half>(s, q, patch, list, list_count, st)
                    : launch_fuse_t<float>(s, q, patch, list, list_count, st);
}

template <typename T, int P, int KT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(search_waves(P))))
void k_learned(SceneDev s, SearchDev q, LearnedDev l, int prop_by_j) {
  const Group gr = make_group<KT>(q.K);
  const int64_t wave = wave_tile(gridDim.x);
  const int64_t j = wave * gr.G + gr.g;
  if (wave * gr.G >= s.n) return;
  const bool pt_ok = gr.lane_ok && j < s.n;
  learned_group<T, P, KT>(s, q, l, gr, pt_ok, pt_ok ? j : 0, prop_by_j, 0, 0);
}

hipError_t launch_learned_refine(const SceneDev& s, const SearchDev& q, const LearnedDev& l,
                                 int dtype, int patch, int prop_by_j, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  const int G = kWave / q.K;
  const int64_t nb = (s.n + 4 * (int64_t)G - 1) / (4 * (int64_t)G);
  dim3 grid((unsigned)nb), block(256);
#define FD_LEARNED_CASE(T, P)                                                             \
  if (q.K == 5)                                                                           \
    hipLaunchKernelGGL((k_learned<T, P, 5>), grid, block, 0, st, s, q, l, prop_by_j);     \
  else                                                                                    \
    hipLaunchKernelGGL((k_learned<T, P, 0>), grid, block, 0, st, s, q, l, prop_by_j);
  if (dtype == 1) {
    switch (patch) {
      case 1: FD_LEARNED_CASE(__half, 1) break;
      case 3: FD_LEARNED_CASE(__half, 3) break;
      case 5: FD_LEARNED_CASE(__half, 5) break;
      case 7: FD_LEARNED_CASE(__half, 7) break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (patch) {
      case 1: FD_LEARNED_CASE(float, 1) break;
      case 3: FD_LEARNED_CASE(float, 3) break;
      case 5: FD_LEARNED_CASE(float, 5) break;
      case 7: FD_LEARNED_CASE(float, 7) break;
      default: return hipErrorInvalidValue;
    }
  }
#undef FD_LEARNED_CASE
  return hipGetLastError();
}

// ---- paper-literal candidates ---------------------------------------------------
template <typename T, int P, int KT>
__global__ __launch_bounds__(256) void k_fpmvo(SceneDev s, SearchDev q, FpmvoDev f) {
  const Group gr = make_group<KT>(q.K);
  const int64_t wave = wave_tile(gridDim.x);
  const int64_t j = wave * gr.G + gr.g;
  if (wave * gr.G >= s.n) return;  // whole wave idle (uniform exit)
  const bool pt_ok = gr.lane_ok && j < s.n;
  fpmvo_group<T, P, KT>(s, q, f, gr, pt_ok, pt_ok ? j : 0);
}

hipError_t launch_fpmvo(const SceneDev& s, const SearchDev& q, const FpmvoDev& f, int dtype,
                        int patch, hipStream_t st) {
  if (s.n <= 0) return hipSuccess;
  const int G = kWave / q.K;
  const int64_t nb = (s.n + 4 * (int64_t)G - 1) / (4 * (int64_t)G);
  dim3 grid((unsigned)nb), block(256);
#define FD_FPMVO_CASE(T, P)                                                     \
  if (q.K == 5)                                                                 \
    hipLaunchKernelGGL((k_fpmvo<T, P, 5>), grid, block, 0, st, s, q, f);        \
  else                                                                          \
    hipLaunchKernelGGL((k_fpmvo<T, P, 0>), grid, block, 0, st, s, q, f);
  if (dtype == 1) {
    switch (patch) {
      case 1: FD_FPMVO_CASE(__half, 1) break;
      case 3: FD_FPMVO_CASE(__half, 3) break;
      case 5: FD_FPMVO_CASE(__half, 5) break;
      case 7: FD_FPMVO_CASE(__half, 7) break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (patch) {
      case 1: FD_FPMVO_CASE(float, 1) break;
      case 3: FD_FPMVO_CASE(float, 3) break;
      case 5: FD_FPMVO_CASE(float, 5) break;
      case 7: FD_FPMVO_CASE(float, 7) break;
      default: return hipErrorInvalidValue;
    }
  }
#undef FD_FPMVO_CASE
  return hipGetLastError();
}

}  // namespace fd
