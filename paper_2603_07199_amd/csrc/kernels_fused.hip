// Fused path (placeholder until the persistent fused kernel lands).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mppi {

int fused_tile_rollouts(int, int, int) { return 16; }

hipError_t launch_fused(const FusedBatch&, const DeviceWeights&, int, hipStream_t, hipEvent_t,
                        hipEvent_t) {
  return hipErrorNotSupported;
}

int pack_lowp_weights(int, int, int, const mppi_sdf_weights*, std::vector<uint8_t>&,
                      std::vector<float>&, std::vector<float>&, std::vector<float>&) {
  return MPPI_EINVAL;
}

}  // namespace mppi
