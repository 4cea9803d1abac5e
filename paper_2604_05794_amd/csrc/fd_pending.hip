// fd_pending.hip -- entry points whose kernels are not in this build yet.
#include <hip/hip_runtime.h>

#include "../../include/fusedir.h"
#include "fd_api_internal.hpp"

using namespace fd;

#define PENDING(fn) return set_error(FD_E_UNSUPPORTED, "%s is not available in this build", fn)

int fd::context_reserve_scenes(fd_context*, int32_t, int64_t) { return FD_OK; }
extern "C" int fd_fuse_directions_batched(const fd_scene*, int32_t, const fd_params*,
                                          fd_context*) {
  PENDING("fd_fuse_directions_batched");
}
extern "C" int fd_autotune(fd_context*, const fd_scene*, int32_t, const fd_params*,
                           const char*) {
  PENDING("fd_autotune");
}
