// Instantiations of the fused MHM / VL-second-stage kernel and the VL
// predictor for double.
#include "fused_muscl.hpp"
#include "fused_vlpred.hpp"

namespace hy {

template <int MODE, bool PPM, int RS, int WAVES, bool FAST>
static hipError_t launch_one(const FusedArgs<double>& a, int grid, hipStream_t st) {
  if (a.zrun != 1) return hipErrorInvalidValue;  // one group per work item in FP64
  auto k = muscl::muscl_kernel<double, PPM, RS, WAVES, MODE, FAST, 1>;
  const size_t shm = muscl::kLdsBytes(sizeof(double));
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(fz::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

template <int MODE, int WAVES, bool FAST>
static hipError_t launch_wf(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (recon == 1) {
    if (riemann == 0) return launch_one<MODE, true, 0, WAVES, FAST>(a, grid, st);
    if (riemann == 1) return launch_one<MODE, true, 1, WAVES, FAST>(a, grid, st);
    return launch_one<MODE, true, 2, WAVES, FAST>(a, grid, st);
  }
  if (riemann == 0) return launch_one<MODE, false, 0, WAVES, FAST>(a, grid, st);
  if (riemann == 1) return launch_one<MODE, false, 1, WAVES, FAST>(a, grid, st);
  return launch_one<MODE, false, 2, WAVES, FAST>(a, grid, st);
}

template <int MODE, int WAVES>
static hipError_t launch_w(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.limiter == 1 && a.charlim == 1) return launch_wf<MODE, WAVES, true>(a, recon, riemann, grid, st);
  return launch_wf<MODE, WAVES, false>(a, recon, riemann, grid, st);
}

hipError_t launch_muscl_f64(const FusedArgs<double>& a, int mode, int recon, int riemann, const FusedCfg& cfg,
                             hipStream_t st) {
  return mode == 0 ? launch_w<0, 2>(a, recon, riemann, cfg.grid, st) : launch_w<1, 2>(a, recon, riemann, cfg.grid, st);
}

template <int G, int RS>
static hipError_t launch_pred(const FusedArgs<double>& a, int grid, hipStream_t st) {
  auto k = vlpred::vl_predict_kernel<double, G, RS>;
  const size_t shm = (size_t)vlpred::lds_elems<G>() * sizeof(double);
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(vlpred::threads<G>()), shm, st>>>(a);
  return hipGetLastError();
}

template <int G>
static hipError_t launch_pred_g(const FusedArgs<double>& a, int riemann, int grid, hipStream_t st) {
  if (riemann == 0) return launch_pred<G, 0>(a, grid, st);
  if (riemann == 1) return launch_pred<G, 1>(a, grid, st);
  return launch_pred<G, 2>(a, grid, st);
}

// Input ghost width of the predictor: the scheme's (PPM 4, PLM 3) for
// ghosted groups, 1 when every segment is a periodic box (interiors only).
hipError_t launch_vlpred_f64(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.wstar_box) return launch_pred_g<1>(a, riemann, grid, st);
  if (recon == 1) return launch_pred_g<4>(a, riemann, grid, st);
  return launch_pred_g<3>(a, riemann, grid, st);
}

}  // namespace hy
