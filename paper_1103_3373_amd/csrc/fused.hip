// Dispatch of the fused patch-group solvers: CTU (fused_ctu.hpp), MHM and the
// VL second stage (fused_muscl.hpp), and the VL predictor (fused_vlpred.hpp),
// instantiated per arithmetic type in the fused_*_{f32,f64}.hip files.
#include "hydro_internal.h"

namespace hy {

hipError_t launch_ctu_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st);
hipError_t launch_ctu_f64(const FusedArgs<double>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st);
hipError_t launch_muscl_f32(const FusedArgs<float>& a, int mode, int recon, int riemann, const FusedCfg& cfg,
                            hipStream_t st);
hipError_t launch_muscl_f64(const FusedArgs<double>& a, int mode, int recon, int riemann, const FusedCfg& cfg,
                            hipStream_t st);
hipError_t launch_vlpred_f32(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st);
hipError_t launch_vlpred_f64(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st);

bool fused_supported(int scheme, int recon, int riemann, int charlim) {
  (void)charlim;
  return scheme >= 0 && scheme <= 2 && (recon == 0 || recon == 1) && riemann >= 0 && riemann <= 2;
}

long long fused_scratch_per_group(int scheme, int recon, int box_segs) {
  if (scheme != 1) return 0;
  if (box_segs) return 5 * 4096;  // half step of the interiors, grouped like the box
  const long long n = 16 + 2 * (recon == 1 ? 3 : 2);
  return 5 * n * n * n;
}

template <typename T>
static hipError_t dispatch(const FusedArgs<T>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                           hipStream_t st,
                           hipError_t (*ctu)(const FusedArgs<T>&, int, int, const FusedCfg&, hipStream_t),
                           hipError_t (*muscl)(const FusedArgs<T>&, int, int, int, const FusedCfg&, hipStream_t),
                           hipError_t (*pred)(const FusedArgs<T>&, int, int, int, hipStream_t)) {
  if (scheme == 2) return ctu(a, recon, riemann, cfg, st);
  if (scheme == 0) return muscl(a, 0, recon, riemann, cfg, st);
  if (scheme == 1) {
    if (!a.wstar) return hipErrorInvalidValue;
    hipError_t e = pred(a, recon, riemann, cfg.grid_pred > 0 ? cfg.grid_pred : cfg.grid, st);
    if (e != hipSuccess) return e;
    return muscl(a, 1, recon, riemann, cfg, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fused(const FusedArgs<float>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st) {
  return dispatch<float>(a, scheme, recon, riemann, cfg, st, launch_ctu_f32, launch_muscl_f32, launch_vlpred_f32);
}
hipError_t launch_fused(const FusedArgs<double>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st) {
  return dispatch<double>(a, scheme, recon, riemann, cfg, st, launch_ctu_f64, launch_muscl_f64, launch_vlpred_f64);
}
int fused_block_threads() { return 512; }

}  // namespace hy
