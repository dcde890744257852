// Instantiations of the fused CTU kernel for float.
#include "fused_ctu.hpp"

namespace hy {

template <bool PPM, int RS, int WAVES>
static hipError_t launch_one(const FusedArgs<float>& a, int grid, hipStream_t st) {
  auto k = ctu::ctu_fused_kernel<float, PPM, RS, WAVES>;
  const size_t shm = ctu::kLdsBytes(sizeof(float));
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr = true;
  }
  k<<<dim3(grid), dim3(ctu::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

template <int WAVES>
static hipError_t launch_w(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (recon == 1) {
    if (riemann == 0) return launch_one<true, 0, WAVES>(a, grid, st);
    if (riemann == 1) return launch_one<true, 1, WAVES>(a, grid, st);
    return launch_one<true, 2, WAVES>(a, grid, st);
  }
  if (riemann == 0) return launch_one<false, 0, WAVES>(a, grid, st);
  if (riemann == 1) return launch_one<false, 1, WAVES>(a, grid, st);
  return launch_one<false, 2, WAVES>(a, grid, st);
}

hipError_t launch_ctu_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st) {
  if (cfg.waves == 4) return launch_w<4>(a, recon, riemann, cfg.grid, st);
  return launch_w<2>(a, recon, riemann, cfg.grid, st);
}

}  // namespace hy
