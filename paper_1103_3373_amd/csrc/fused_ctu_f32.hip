// Instantiations of the fused CTU kernel for float with the HLLC and HLLE
// solvers (the Roe instantiations live in fused_ctu_f32_roe.hip, which is
// compiled with other scheduler options).
#include "fused_ctu.hpp"

namespace hy {

hipError_t launch_ctu_f32_roe(const FusedArgs<float>& a, int recon, int waves, bool fast, int grid, hipStream_t st);

template <bool PPM, int RS, int WAVES, bool FAST, int ZR>
static hipError_t launch_zr(const FusedArgs<float>& a, int grid, hipStream_t st) {
  auto k = ctu::ctu_fused_kernel<float, PPM, RS, WAVES, FAST, ZR>;
  const size_t shm = ctu::kLdsBytes(sizeof(float));
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(ctu::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

template <bool PPM, int RS, int WAVES, bool FAST>
static hipError_t launch_one(const FusedArgs<float>& a, int grid, hipStream_t st) {
  if constexpr (WAVES == 4 && FAST) {
    if (a.zrun == 2) return launch_zr<PPM, RS, WAVES, FAST, 2>(a, grid, st);
    if (a.zrun == 4) return launch_zr<PPM, RS, WAVES, FAST, 4>(a, grid, st);
  }
  if (a.zrun != 1) return hipErrorInvalidValue;
  return launch_zr<PPM, RS, WAVES, FAST, 1>(a, grid, st);
}

template <int WAVES, bool FAST>
static hipError_t launch_wf(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (riemann == 0) return launch_ctu_f32_roe(a, recon, WAVES, FAST, grid, st);
  if (recon == 1) {
    if (riemann == 1) return launch_one<true, 1, WAVES, FAST>(a, grid, st);
    return launch_one<true, 2, WAVES, FAST>(a, grid, st);
  }
  if (riemann == 1) return launch_one<false, 1, WAVES, FAST>(a, grid, st);
  return launch_one<false, 2, WAVES, FAST>(a, grid, st);
}

template <int WAVES>
static hipError_t launch_w(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.limiter == 1 && a.charlim == 1) return launch_wf<WAVES, true>(a, recon, riemann, grid, st);
  return launch_wf<WAVES, false>(a, recon, riemann, grid, st);
}

hipError_t launch_ctu_f32(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st) {
  if (cfg.waves == 4) return launch_w<4>(a, recon, riemann, cfg.grid, st);
  return launch_w<2>(a, recon, riemann, cfg.grid, st);
}

}  // namespace hy
