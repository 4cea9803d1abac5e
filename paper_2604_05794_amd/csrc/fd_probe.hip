// fd_probe.hip -- read-bandwidth probe for the roofline of the search
// (measures the L2 ceiling, which has no published figure).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"

using namespace fd;

namespace {

// Every workgroup walks the whole buffer with 16-byte loads; lane values
// are folded so that no load is dead.
__global__ __launch_bounds__(256) void k_probe_read(const uint4* __restrict__ buf, int64_t n16,
                                                    int reps, uint32_t* __restrict__ sink) {
  uint32_t acc = 0;
  for (int r = 0; r < reps; ++r) {
    for (int64_t i = threadIdx.x; i < n16; i += 4 * 256) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t k = i + u * 256;
        v[u] = k < n16 ? buf[k] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    acc = (acc << 1) | (acc >> 31);
  }
  sink[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

extern "C" int fd_probe_read(const void* buf, int64_t bytes, int32_t reps, int32_t blocks,
                             uint32_t* sink, void* stream) {
  if (!buf || !sink) return set_error(FD_E_INVAL, "fd_probe_read: null pointer");
  if (bytes <= 0 || (bytes & 15) || bytes > ((int64_t)1 << 31))
    return set_error(FD_E_INVAL, "fd_probe_read: bytes must be a positive multiple of 16, "
                     "at most 2^31");
  if (reps < 1 || blocks < 1) return set_error(FD_E_INVAL, "fd_probe_read: reps and blocks >= 1");
  int r;
  if ((r = check_device(nullptr))) return r;
  hipLaunchKernelGGL(k_probe_read, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const uint4*)buf, bytes / 16, reps, sink);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? FD_OK : hip_error(e, "fd_probe_read");
}
