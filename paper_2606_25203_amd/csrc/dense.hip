// dense.hip -- dense (fully connected) instances: placeholder until the
// int8 matrix-core field kernels land.
#include <hip/hip_runtime.h>

#include "../../include/pamc.h"
#include "instance.hpp"

namespace pamc {
hipError_t launch_dense_generate(pamc_instance*, uint64_t) { return hipErrorNotSupported; }
hipError_t launch_init_dense(pamc_instance*) { return hipErrorNotSupported; }
hipError_t launch_dense_step(pamc_instance*, const Schedule&, int32_t) { return hipErrorNotSupported; }
hipError_t launch_dense_prim_sweep(pamc_instance*, double, int32_t) { return hipErrorNotSupported; }
hipError_t launch_dense_prim_resample(pamc_instance*, double) { return hipErrorNotSupported; }
hipError_t launch_dense_prim_update_best(pamc_instance*) { return hipErrorNotSupported; }
}  // namespace pamc

extern "C" {
pamc_status pamc_create_instance_dense_i8(int32_t, const int8_t*, int64_t, pamc_mem, int32_t,
                                          const pamc_config*, pamc_instance** out) {
  if (out) *out = nullptr;
  return PAMC_ERR_UNSUPPORTED;
}
pamc_status pamc_create_instance_dense_random(int32_t, uint64_t, const pamc_config*, pamc_instance** out) {
  if (out) *out = nullptr;
  return PAMC_ERR_UNSUPPORTED;
}
}
