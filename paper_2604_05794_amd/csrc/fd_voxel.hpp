// fd_voxel.hpp -- the binary32 voxel rule shared by the volume and the
// strand-growing kernels (documented with fd_fuse_volume in fusedir.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fd {

struct GridDev {
  float o[3];
  float h;
  int32_t dims[3];
};

// binary32 voxel index (subtraction, IEEE division, floor), -1 outside
__device__ __forceinline__ int64_t voxel_index(const GridDev& g, float x, float y, float z) {
  const float p[3] = {x, y, z};
  int32_t ix[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float q = (p[a] - g.o[a]) / g.h;
    if (!(q >= 0.0f) || !(q < (float)g.dims[a])) return -1;
    ix[a] = (int32_t)q;  // q >= 0: truncation is the floor
  }
  return ((int64_t)ix[2] * g.dims[1] + ix[1]) * g.dims[0] + ix[0];
}

}  // namespace fd
