// Launch helpers of the fused MHM / VL-second-stage kernel for float, shared
// by the two files that instantiate it (MHM and the VL second stage build
// with different scheduler options).
#pragma once

#include "fused_muscl.hpp"

namespace hy {
namespace muscl_launch {

template <int MODE, bool PPM, int RS, int WAVES, bool FAST, int ZR>
hipError_t launch_zr(const FusedArgs<float>& a, int grid, hipStream_t st) {
  auto k = muscl::muscl_kernel<float, PPM, RS, WAVES, MODE, FAST, ZR>;
  const size_t shm = muscl::kLdsBytes(sizeof(float));
  static std::atomic<unsigned long long> lds_set{0};
  const hipError_t e = raise_lds_limit((const void*)k, shm, lds_set);
  if (e != hipSuccess) return e;
  k<<<dim3(grid), dim3(fz::kThreads), shm, st>>>(a);
  return hipGetLastError();
}

// Tile depths 2 and 4 exist for the PPM van Leer / characteristic
// specialization with two workgroups per CU (zrun_built).
template <int MODE, bool PPM, int RS, int WAVES, bool FAST>
hipError_t launch_one(const FusedArgs<float>& a, int grid, hipStream_t st) {
  if constexpr (WAVES == 4 && FAST && PPM) {
    if (a.zrun == 2) return launch_zr<MODE, PPM, RS, WAVES, FAST, 2>(a, grid, st);
    if (a.zrun == 4) return launch_zr<MODE, PPM, RS, WAVES, FAST, 4>(a, grid, st);
  }
  if (a.zrun != 1) return hipErrorInvalidValue;
  return launch_zr<MODE, PPM, RS, WAVES, FAST, 1>(a, grid, st);
}

template <int MODE, int WAVES, bool FAST>
hipError_t launch_wf(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
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
hipError_t launch_w(const FusedArgs<float>& a, int recon, int riemann, int grid, hipStream_t st) {
  if (a.limiter == 1 && a.charlim == 1) return launch_wf<MODE, WAVES, true>(a, recon, riemann, grid, st);
  return launch_wf<MODE, WAVES, false>(a, recon, riemann, grid, st);
}

// Every specialization of one mode (0 MHM, 1 VL second stage).
template <int MODE>
hipError_t launch_mode(const FusedArgs<float>& a, int recon, int riemann, const FusedCfg& cfg, hipStream_t st) {
  if (cfg.waves == 4) return launch_w<MODE, 4>(a, recon, riemann, cfg.grid, st);
  return launch_w<MODE, 2>(a, recon, riemann, cfg.grid, st);
}

}  // namespace muscl_launch
}  // namespace hy
