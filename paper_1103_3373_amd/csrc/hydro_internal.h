// Internal interfaces between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "hydro_math.hpp"

namespace hy {

// Raises kernel fn's dynamic LDS limit to shm bytes on the current device,
// once per device (device ids 0..63 are remembered in done; others are set
// on every call).  done is one static per kernel instantiation.
inline hipError_t raise_lds_limit(const void* fn, size_t shm, std::atomic<unsigned long long>& done) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const unsigned long long bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0ull;
  if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_release);
  return e;
}

template <typename T>
struct PlainArgs {
  const T* in;     // [n][5][N][N][N]
  T* out;          // [n][5][16][16][16]
  T* flux;         // [n][3][nf][5][16][16] or null
  long n_groups;
  int g, N, nf;
  Phys<T> ph;
  T* ws;           // per-workgroup global temporaries
  long ws_stride;  // elements per workgroup (50 N^3)
  unsigned long long* diag;  // [0] Roe fallbacks, [1] floor activations
  int roe_fb_exact;          // Roe failures take the exact flux
};

hipError_t launch_plain(const PlainArgs<float>& a, int scheme, int recon, int riemann, int grid, hipStream_t st);
hipError_t launch_plain(const PlainArgs<double>& a, int scheme, int recon, int riemann, int grid, hipStream_t st);

// Segment of a batched launch: a run of groups sharing in/out/flux arrays,
// dh and a device time step (scaled per level).
struct Seg {
  const void* in;
  void* out;
  void* flux;
  const double* dt;
  double dt_scale;
  double dh;
  long long first;   // first global group index of this segment
  long long count;
  int ngx, ngy, ngz;  // box mode: groups per dimension of a periodic box
  int box;            // 1: `in` is the box [G][5][16][16][16]; ghosts are read from it
};

// Fused (optimized) solver.  groups are addressed through segments; a plain
// single-array call is one segment.
template <typename T>
struct FusedArgs {
  const Seg* segs;   // device table
  int n_segs;
  long long n_groups;
  int g, nf;
  T gamma, theta, floor;
  int limiter, charlim, roe_fb_hllc;
  unsigned long long* diag;
  // Single-segment launches pass their segment and time step by value
  // (segs == nullptr), so no table upload is needed.
  Seg seg0;
  double dt0;
  // VL: scratch for the half-step primitive state.  wstar_box == 0: ghosted
  // per group, [n_groups][5][N'^3]; wstar_box == 1 (every segment a periodic
  // box): interiors only, [n_groups][5][16^3], each segment's part a grouped
  // box of its own whose ghost cells the second stage reads from neighbours.
  T* wstar;
  int wstar_box;
  // CTU on one periodic box (seg0, no flux output): a workgroup marches
  // through zrun z-consecutive groups of one (gx, gy) column in one pass, so
  // the work items are n_groups / zrun runs (ngz a multiple of zrun).  1
  // everywhere else.
  int zrun;
};

// Tile depths (groups per z-run) built for the fused kernels: 1 always; 2
// and 4 for the FP32 specialization of the production configuration (van
// Leer limiter on characteristic variables) with two workgroups per CU, for
// CTU with PLM or PPM and for MHM / the VL second stage with PPM.
inline bool zrun_built(int scheme, bool f64, int waves, int recon, int limiter, int charlim, int zrun) {
  if (zrun == 1) return true;
  return !f64 && waves == 4 && limiter == 1 && charlim == 1 && (zrun == 2 || zrun == 4) &&
         (scheme == 2 || recon == 1);
}

struct FusedCfg {
  int grid;          // number of workgroups (persistent)
  int waves;         // register budget variant: minimum waves per SIMD (2 or 4)
  int grid_pred;     // VL predictor workgroups (0 = grid); it marches one group
                     // at a time whatever the second stage's tile depth
};

bool fused_supported(int scheme, int recon, int riemann, int charlim);
// Elements of T per group of the VL half-step scratch (0 for other schemes):
// the ghosted half-step region of a group, or with box_segs (every segment a
// periodic box) only its interior.
long long fused_scratch_per_group(int scheme, int recon, int box_segs);
hipError_t launch_fused(const FusedArgs<float>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st);
hipError_t launch_fused(const FusedArgs<double>& a, int scheme, int recon, int riemann, const FusedCfg& cfg,
                        hipStream_t st);
int fused_block_threads();

// Auxiliary kernels.
template <typename T>
hipError_t launch_fill_periodic(const T* box, int nx, int ny, int nz, int g, int grouped, T* out, hipStream_t st);
hipError_t launch_group_map(const int* layout, int n_groups, int ng0, int n_levels, long long map_len, int* map,
                            hipStream_t st);
template <typename T>
hipError_t launch_amr_correct(T* U, int n, const T* cflux, const T* fine, const int* flayout, int nf,
                              const int* fmap, const T* fflux, double dtdh, hipStream_t st);
template <typename T>
hipError_t launch_axpy(T* acc, const T* x, double w, long long n, hipStream_t st);
template <typename T>
hipError_t launch_fill_amr(const T* fine, const int* layout, int n_groups, const int* map, int ng0, int n_levels,
                           const T* c0, const T* c1, int cn, const double* alpha, int g, T* out, hipStream_t st);
template <typename T>
hipError_t launch_fill_interp(const T* coarse, int cn, const int* layout, long long n_groups, int g, double base_dh,
                              T* out, hipStream_t st);
template <typename T>
hipError_t launch_maxspeed(const T* U, long long n_blocks, long long cells, double gamma, double* partial,
                           int n_partial, hipStream_t st);
hipError_t launch_seg_dt(const Seg* segs, int n_segs, long long n_groups, double gamma, double cfl, int f64,
                         double* partial, hipStream_t st);
hipError_t launch_dt_finish(const double* partial, int n_partial, double dh, double cfl, double* dt_out,
                            hipStream_t st);
template <typename T>
hipError_t launch_sums(const T* U, long long n_blocks, long long cells, double dh, double* partial, int n_partial,
                       double* sums_out, hipStream_t st);
template <typename T>
hipError_t launch_dtsums(const T* U, long long n_blocks, double dh, double gamma, double cfl, double* partial,
                         int n_partial, double* dt_out, double* sums_out, hipStream_t st);

}  // namespace hy
