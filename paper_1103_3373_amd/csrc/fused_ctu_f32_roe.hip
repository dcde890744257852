// Instantiations of the fused CTU kernel for float with the Roe solver (its
// fallback included), in a file of their own so that they can be compiled
// with other scheduler options than the HLLC and HLLE instantiations.
#include "fused_ctu.hpp"

namespace hy {

template <bool PPM, int WAVES, bool FAST, int ZR>
static hipError_t launch_roe_zr(const FusedArgs<float>& a, int grid, hipStream_t st) {
  auto k = ctu::ctu_fused_kernel<float, PPM, 0, WAVES, FAST, ZR>;
  const size_t shm = ctu::kLdsBytes(sizeof(float));
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(ctu::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

template <bool PPM, int WAVES, bool FAST>
static hipError_t launch_roe(const FusedArgs<float>& a, int grid, hipStream_t st) {
  if constexpr (WAVES == 4 && FAST) {
    if (a.zrun == 2) return launch_roe_zr<PPM, WAVES, FAST, 2>(a, grid, st);
    if (a.zrun == 4) return launch_roe_zr<PPM, WAVES, FAST, 4>(a, grid, st);
  }
  if (a.zrun != 1) return hipErrorInvalidValue;
  return launch_roe_zr<PPM, WAVES, FAST, 1>(a, grid, st);
}

template <int WAVES>
static hipError_t launch_roe_w(const FusedArgs<float>& a, int recon, bool fast, int grid, hipStream_t st) {
  if (recon == 1) return fast ? launch_roe<true, WAVES, true>(a, grid, st) : launch_roe<true, WAVES, false>(a, grid, st);
  return fast ? launch_roe<false, WAVES, true>(a, grid, st) : launch_roe<false, WAVES, false>(a, grid, st);
}

hipError_t launch_ctu_f32_roe(const FusedArgs<float>& a, int recon, int waves, bool fast, int grid, hipStream_t st) {
  if (waves == 4) return launch_roe_w<4>(a, recon, fast, grid, st);
  return launch_roe_w<2>(a, recon, fast, grid, st);
}

}  // namespace hy
