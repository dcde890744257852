// Fused patch-group solver (placeholder until the optimized kernel lands).
#include "hydro_internal.h"

namespace hy {
bool fused_supported(int, int, int, int) { return false; }
hipError_t launch_fused(const FusedArgs<float>&, int, int, int, const FusedCfg&, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fused(const FusedArgs<double>&, int, int, int, const FusedCfg&, hipStream_t) {
  return hipErrorInvalidValue;
}
int fused_block_threads() { return 256; }
}  // namespace hy
