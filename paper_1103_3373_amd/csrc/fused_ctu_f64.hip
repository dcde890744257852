// Instantiations of the fused CTU kernel for double.
#include "fused_ctu.hpp"

namespace hy {

template <bool PPM, int RS, int WAVES, bool FAST>
static hipError_t launch_one(const FusedArgs<double>& a, int grid, hipStream_t st) {
  if (a.zrun != 1) return hipErrorInvalidValue;  // one tile depth in FP64
  auto k = ctu::ctu_fused_kernel<double, PPM, RS, WAVES, FAST, 1>;
  const size_t shm = ctu::kLdsBytes(sizeof(double));
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(ctu::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

template <int WAVES, bool FAST>
static hipError_t launch_wf(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (recon == 1) {
    if (riemann == 0) return launch_one<true, 0, WAVES, FAST>(a, grid, st);
    if (riemann == 1) return launch_one<true, 1, WAVES, FAST>(a, grid, st);
    return launch_one<true, 2, WAVES, FAST>(a, grid, st);
  }
  if (riemann == 0) return launch_one<false, 0, WAVES, FAST>(a, grid, st);
  if (riemann == 1) return launch_one<false, 1, WAVES, FAST>(a, grid, st);
  return launch_one<false, 2, WAVES, FAST>(a, grid, st);
}

template <int WAVES>
static hipError_t launch_w(const FusedArgs<double>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.limiter == 1 && a.charlim == 1) return launch_wf<WAVES, true>(a, recon, riemann, grid, st);
  return launch_wf<WAVES, false>(a, recon, riemann, grid, st);
}

hipError_t launch_ctu_f64(const FusedArgs<double>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st) {
  return launch_w<2>(a, recon, riemann, cfg.grid, st);
}

}  // namespace hy
