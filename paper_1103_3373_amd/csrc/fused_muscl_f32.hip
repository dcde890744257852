// Instantiations of the fused VL-second-stage kernel and the VL predictor for
// float; MHM's are in their own file (other scheduler options).
#include "fused_muscl_launch.hpp"
#include "fused_vlpred.hpp"

namespace hy {

hipError_t launch_mhm_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st);

hipError_t launch_muscl_f32(const FusedArgs<float>& a, int mode, int recon, int riemann, const FusedCfg& cfg,
                             hipStream_t st) {
  if (mode == 0) return launch_mhm_f32(a, recon, riemann, cfg, st);
  return muscl_launch::launch_mode<1>(a, recon, riemann, cfg, st);
}

template <int G, int RS>
static hipError_t launch_pred(const FusedArgs<float>& a, int grid, hipStream_t st) {
  auto k = vlpred::vl_predict_kernel<float, G, RS>;
  const size_t shm = (size_t)vlpred::lds_elems<G>() * sizeof(float);
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(vlpred::threads<G>()), shm, st>>>(a);
  return hipGetLastError();
}

template <int G>
static hipError_t launch_pred_g(const FusedArgs<float>& a, int riemann, int grid, hipStream_t st) {
  if (riemann == 0) return launch_pred<G, 0>(a, grid, st);
  if (riemann == 1) return launch_pred<G, 1>(a, grid, st);
  return launch_pred<G, 2>(a, grid, st);
}

// Input ghost width of the predictor: the scheme's (PPM 4, PLM 3) for
// ghosted groups, 1 when every segment is a periodic box (interiors only).
hipError_t launch_vlpred_f32(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.wstar_box) return launch_pred_g<1>(a, riemann, grid, st);
  if (recon == 1) return launch_pred_g<4>(a, riemann, grid, st);
  return launch_pred_g<3>(a, riemann, grid, st);
}

}  // namespace hy
