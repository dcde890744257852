// Instantiations of the fused MHM kernel for float, in a file of their own so
// that they can be compiled with other scheduler options than the VL second
// stage.
#include "fused_muscl_launch.hpp"

namespace hy {

hipError_t launch_mhm_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st) {
  return muscl_launch::launch_mode<0>(a, recon, riemann, cfg, st);
}

}  // namespace hy
