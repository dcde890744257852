// Dispatch of the fused patch-group solvers.  The CTU kernel (fused_ctu.hpp)
// is instantiated per arithmetic type in fused_ctu_f32.hip / fused_ctu_f64.hip.
#include "hydro_internal.h"

namespace hy {

hipError_t launch_ctu_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st);
hipError_t launch_ctu_f64(const FusedArgs<double>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st);

bool fused_supported(int scheme, int recon, int riemann, int charlim) {
  (void)charlim;
  return scheme == 2 && (recon == 0 || recon == 1) && riemann >= 0 && riemann <= 2;
}

hipError_t launch_fused(const FusedArgs<float>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st) {
  if (scheme != 2) return hipErrorInvalidValue;
  return launch_ctu_f32(a, recon, riemann, cfg, st);
}
hipError_t launch_fused(const FusedArgs<double>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st) {
  if (scheme != 2) return hipErrorInvalidValue;
  return launch_ctu_f64(a, recon, riemann, cfg, st);
}
int fused_block_threads() { return 512; }

}  // namespace hy
