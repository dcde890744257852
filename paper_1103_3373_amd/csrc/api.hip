// Host side of the C ABI declared in include/hydro.h: argument validation,
// dispatch to the plain or fused kernels, library-owned workspaces, device
// diagnostics and the launch-shape autotuner.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hydro.h"
#include "hydro_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(HYDRO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const int kKnownFlags = HYDRO_F64 | HYDRO_CHAR | HYDRO_FLUX_MID | HYDRO_PLAIN | HYDRO_ROE_FB_HLLC | HYDRO_BOX_GROUPED |
                        HYDRO_BOX_SEGS | HYDRO_ROE_FB_EXACT;

int ghost_width(int scheme, int recon) {
  if (scheme < 0 || scheme > 2 || recon < 0 || recon > 1) return -1;
  int r = recon == HYDRO_PPM ? 2 : 1;
  return scheme == HYDRO_VL ? r + 2 : r + 1;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + nb && y < x + na;
}

// Library-owned device memory.  The plain path's temporaries are per
// (device, stream).  Reduction partials come from a per-device pool of slots
// allocated once, on the first call on that device, so a stream met later
// (for instance one that is capturing a graph) never allocates.
struct Workspace {
  void* plain = nullptr;
  size_t plain_bytes = 0;
  double* seg_partial = nullptr;  // per-group maxima of hydro_cfl_dt_batch
  long long seg_partial_n = 0;
  void* vl = nullptr;  // VL half-step scratch (fused path)
  size_t vl_bytes = 0;
  double* partial = nullptr;  // reduction partials, kPartials x 6 doubles (a pool slot or own memory)
  bool own_partial = false;
};
const int kPartialSlots = 64;
struct DeviceState {
  unsigned long long* diag = nullptr;
  double* partial_pool = nullptr;
  int partial_used = 0;
  std::map<hipStream_t, Workspace> ws;
};
std::mutex g_mu;
std::map<int, DeviceState> g_dev;

const int kPartials = 1024;   // reduction partials (fixed: deterministic order)
const int kPlainGridMax = 512; // plain path: workgroups (each owns 50 N^3 temporaries)

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return 0;
}

// Returns the device state (creating the diagnostics counters on first use).
int device_state(DeviceState** out) {
  int dev;
  if (int rc = current_device(&dev)) return rc;
  DeviceState& d = g_dev[dev];
  if (!d.diag) {
    hipError_t e = hipMalloc((void**)&d.diag, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(diag)");
    e = hipMemset(d.diag, 0, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) return hip_fail(e, "hipMemset(diag)");
    e = hipMalloc((void**)&d.partial_pool, (size_t)kPartialSlots * kPartials * 6 * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(partial pool)");
  }
  *out = &d;
  return 0;
}

int ensure_plain(Workspace& w, size_t bytes) {
  if (w.plain_bytes >= bytes) return 0;
  if (w.plain) {
    hipDeviceSynchronize();
    hipFree(w.plain);
    w.plain = nullptr;
    w.plain_bytes = 0;
  }
  hipError_t e = hipMalloc(&w.plain, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(plain workspace)");
  w.plain_bytes = bytes;
  return 0;
}
// VL scratch: grown on demand (an allocation, so the first VL call at a
// given batch size must not be inside a graph capture).
int ensure_vl(Workspace& w, size_t bytes) {
  if (w.vl_bytes >= bytes) return 0;
  if (w.vl) {
    hipDeviceSynchronize();
    hipFree(w.vl);
    w.vl = nullptr;
    w.vl_bytes = 0;
  }
  hipError_t e = hipMalloc(&w.vl, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(VL scratch)");
  w.vl_bytes = bytes;
  return 0;
}

int ensure_partial(DeviceState& d, Workspace& w) {
  if (w.partial) return 0;
  if (d.partial_used < kPartialSlots) {
    w.partial = d.partial_pool + (size_t)(d.partial_used++) * kPartials * 6;
    return 0;
  }
  hipError_t e = hipMalloc((void**)&w.partial, (size_t)kPartials * 6 * sizeof(double));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(partials)");
  w.own_partial = true;
  return 0;
}
template <typename T>
hy::Phys<T> make_phys(double dt, double dh, double gamma, int limiter, int flags) {
  hy::Phys<T> p;
  p.gamma = (T)gamma;
  p.gm1 = (T)(gamma - 1.0);
  p.inv_gm1 = (T)(1.0 / (gamma - 1.0));
  p.dtdh = (T)(dt / dh);
  p.hdtdh = (T)(0.5 * dt / dh);
  p.theta = (T)1.5;
  p.floor = (T)1e-10;
  p.limiter = limiter;
  p.charlim = (flags & HYDRO_CHAR) ? 1 : 0;
  p.roe_fb_hllc = (flags & HYDRO_ROE_FB_HLLC) ? 1 : 0;
  return p;
}

int check_options(int scheme, int recon, int riemann, int limiter, int flags) {
  if (ghost_width(scheme, recon) < 0) return fail(HYDRO_EINVAL, "bad scheme %d or reconstruction %d", scheme, recon);
  if (riemann < 0 || riemann > 3) return fail(HYDRO_EINVAL, "bad riemann %d", riemann);
  if (limiter < 0 || limiter > 3) return fail(HYDRO_EINVAL, "bad limiter %d", limiter);
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits 0x%x", flags & ~kKnownFlags);
  return 0;
}

// ---- launch-shape cache (autotuner) ----------------------------------------
// A launch shape is the persistent grid size and the register-budget variant
// (minimum waves per SIMD) of the fused kernel.
struct Tune {
  int grid;      // 0 = default (one resident wave of workgroups)
  int waves;     // 2 or 4
  int zrun;      // CTU box steps: groups per z-run (0 = default)
  int grid_box;  // CTU box steps: workgroups (0 = as grid)
};
std::map<std::string, Tune> g_tune;
bool g_tune_loaded = false;

std::string tune_key(int f64, int scheme, int recon, int riemann, int charlim) {
  char b[96];
  snprintf(b, sizeof(b), "gfx950/%s/s%d/r%d/rs%d/c%d", f64 ? "f64" : "f32", scheme, recon, riemann, charlim);
  return b;
}
void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("HYDRO_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[256], key[128];
  while (fgets(line, sizeof(line), f)) {
    int gr = 0, wv = 0, zr = 0, gb = 0;
    if (sscanf(line, "%127s %d %d %d %d", key, &gr, &wv, &zr, &gb) >= 3) g_tune[key] = Tune{gr, wv, zr, gb};
  }
  fclose(f);
}
int cu_count() {
  static std::map<int, int> cache;  // per device; read once (also safe under graph capture)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  cache[dev] = cus;
  return cus;
}
Tune tuned(int f64, int scheme, int recon, int riemann, int charlim, long long n_groups) {
  tune_load();
  auto it = g_tune.find(tune_key(f64, scheme, recon, riemann, charlim));
  // Untuned default: the two-workgroups-per-CU register variant with twelve
  // workgroups per CU over the persistent loop (about the autotuner's choice
  // for CTU on MI355X: more, shorter workgroups even out the tail); FP64 has
  // one variant only.
  Tune t = (it != g_tune.end()) ? it->second : Tune{0, 4, 0, 0};
  if (f64) t.waves = 2;
  if (t.grid <= 0) t.grid = cu_count() * (t.waves == 4 ? 12 : 1);
  if (t.grid > n_groups) t.grid = (int)n_groups;
  if (t.grid < 1) t.grid = 1;
  return t;
}

// Launch shape of a step over one periodic box of ngz groups in z
// (n_groups in all) without flux output: the z-run length (the tuned one,
// or the largest of 4, 2 that divides ngz and still leaves two runs per
// resident workgroup slot; in any case the largest built length, not above
// it, that divides ngz) and the grid over the runs.
Tune tuned_box(int f64, int scheme, int recon, int riemann, int limiter, int charlim, long long n_groups, int ngz) {
  Tune t = tuned(f64, scheme, recon, riemann, charlim, n_groups);
  int K = t.zrun;
  if (K <= 0) {
    const long long slots = (long long)cu_count() * (t.waves == 4 ? 2 : 1);
    K = 1;
    for (int k : {4, 2})
      if (ngz % k == 0 && n_groups / k >= 2 * slots) { K = k; break; }
  }
  while (K > 1 && (ngz % K || !hy::zrun_built(scheme, f64, t.waves, recon, limiter, charlim, K))) --K;
  t.zrun = K;
  if (t.grid_box > 0) t.grid = t.grid_box;
  const long long items = n_groups / K;
  if (t.grid > items) t.grid = (int)items;
  if (t.grid < 1) t.grid = 1;
  return t;
}

template <typename T>
int run_fused(const hy::Seg* segs_dev, int n_segs, long long n_groups, int g, int scheme, int recon, int riemann,
              int limiter, int flags, double gamma, unsigned long long* diag, int grid, int waves, hipStream_t st,
              void* wstar, const hy::Seg* seg0 = nullptr, double dt0 = 0.0, int wstar_box = 0, int zrun = 1) {
  hy::FusedArgs<T> a;
  a.segs = segs_dev;
  a.n_segs = n_segs;
  a.n_groups = n_groups;
  a.g = g;
  a.nf = (flags & HYDRO_FLUX_MID) ? 3 : 2;
  a.gamma = (T)gamma;
  a.theta = (T)1.5;
  a.floor = (T)1e-10;
  a.limiter = limiter;
  a.charlim = (flags & HYDRO_CHAR) ? 1 : 0;
  a.roe_fb_hllc = (flags & HYDRO_ROE_FB_HLLC) ? 1 : 0;
  a.diag = diag;
  if (seg0) a.seg0 = *seg0;
  else memset(&a.seg0, 0, sizeof(a.seg0));
  a.dt0 = dt0;
  a.wstar = reinterpret_cast<T*>(wstar);
  a.wstar_box = wstar_box;
  a.zrun = zrun;
  hy::FusedCfg cfg;
  cfg.grid = grid;
  cfg.waves = waves;
  // The VL predictor takes one group per work item: as many workgroups as
  // the second stage has groups in flight.
  cfg.grid_pred = (int)std::min<long long>(n_groups, (long long)grid * zrun);
  hipError_t e = hy::launch_fused(a, scheme, recon, riemann, cfg, st);
  if (e != hipSuccess) return hip_fail(e, "fused solver launch");
  return 0;
}

}  // namespace

// Per-group maxima of hydro_cfl_dt_batch_noalloc: a static device array, one
// copy per device.  In host code its name is only a host-side stand-in, so
// host code never passes it to a kernel or a copy; it uses the address that
// hipGetSymbolAddress returns on each device, resolved once per device.
static __device__ __align__(256) double scratch[HYDRO_NOALLOC_MAX_GROUPS];

namespace {

std::map<int, double*> g_scratch;  // device -> address of `scratch` there (guarded by g_mu)

// Address of `scratch` on the current device; resolves it on the first call
// there (no allocation: the array is part of the library's code object).
int scratch_on_device(double** out) {
  int dev;
  if (int rc = current_device(&dev)) return rc;
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(HYDRO_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    it = g_scratch.emplace(dev, static_cast<double*>(ptr)).first;
  }
  *out = it->second;
  return 0;
}

}  // namespace

extern "C" {

int hydro_ghost_width(int scheme, int reconstruction) { return ghost_width(scheme, reconstruction); }

const char* hydro_last_error(void) { return g_err; }

int hydro_solve_groups(const void* in, void* out, void* flux_out, int n_groups, double dt, double dh, double gamma,
                       int scheme, int reconstruction, int riemann, int limiter, int flags, void* stream) {
  g_err[0] = 0;
  if (int rc = check_options(scheme, reconstruction, riemann, limiter, flags)) return rc;
  if (n_groups < 0) return fail(HYDRO_EINVAL, "n_groups %d < 0", n_groups);
  if (!(dt > 0.0) || !isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be positive and finite");
  if (!(dh > 0.0) || !isfinite(dh)) return fail(HYDRO_EINVAL, "dh must be positive and finite");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(HYDRO_EINVAL, "gamma must exceed 1");
  if (n_groups == 0) return 0;
  if (!in || !out) return fail(HYDRO_EINVAL, "null in/out with n_groups > 0");
  const int g = ghost_width(scheme, reconstruction);
  const int N = 16 + 2 * g;
  const bool f64 = (flags & HYDRO_F64) != 0;
  const size_t esz = f64 ? 8 : 4;
  const int nf = (flags & HYDRO_FLUX_MID) ? 3 : 2;
  const size_t in_b = (size_t)n_groups * 5 * N * N * N * esz;
  const size_t out_b = (size_t)n_groups * 5 * 4096 * esz;
  const size_t fl_b = (size_t)n_groups * 3 * nf * 5 * 256 * esz;
  if (overlap(in, in_b, out, out_b)) return fail(HYDRO_EALIAS, "in and out overlap");
  if (flux_out && (overlap(flux_out, fl_b, out, out_b) || overlap(flux_out, fl_b, in, in_b)))
    return fail(HYDRO_EALIAS, "flux_out overlaps in or out");
  hipStream_t st = (hipStream_t)stream;

  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  Workspace& w = ds->ws[st];

  // The exact solver (riemann 3) and the Roe -> exact fallback run on the
  // plain path only.
  const bool plain = (flags & (HYDRO_PLAIN | HYDRO_ROE_FB_EXACT)) ||
                     !hy::fused_supported(scheme, reconstruction, riemann, (flags & HYDRO_CHAR) ? 1 : 0);
  if (plain) {
    int grid = n_groups < kPlainGridMax ? n_groups : kPlainGridMax;
    const long stride = 50L * N * N * N;
    if (int rc = ensure_plain(w, (size_t)grid * stride * esz)) return rc;
    hipError_t e;
    if (f64) {
      hy::PlainArgs<double> a{(const double*)in, (double*)out, (double*)flux_out, n_groups, g, N, nf,
                              make_phys<double>(dt, dh, gamma, limiter, flags), (double*)w.plain, stride, ds->diag,
                              (flags & HYDRO_ROE_FB_EXACT) ? 1 : 0};
      e = hy::launch_plain(a, scheme, reconstruction, riemann, grid, st);
    } else {
      hy::PlainArgs<float> a{(const float*)in, (float*)out, (float*)flux_out, n_groups, g, N, nf,
                             make_phys<float>(dt, dh, gamma, limiter, flags), (float*)w.plain, stride, ds->diag,
                             (flags & HYDRO_ROE_FB_EXACT) ? 1 : 0};
      e = hy::launch_plain(a, scheme, reconstruction, riemann, grid, st);
    }
    if (e != hipSuccess) return hip_fail(e, "plain solver launch");
    return 0;
  }
  // Fused path: a single segment passed by value, host dt included.
  hy::Seg seg{in, out, flux_out, nullptr, 1.0, dh, 0, n_groups, 0, 0, 0, 0};
  const Tune tu = tuned(f64, scheme, reconstruction, riemann, (flags & HYDRO_CHAR) ? 1 : 0, n_groups);
  if (int rc = ensure_vl(w, (size_t)n_groups * hy::fused_scratch_per_group(scheme, reconstruction, 0) * esz)) return rc;
  if (f64)
    return run_fused<double>(nullptr, 1, n_groups, g, scheme, reconstruction, riemann, limiter, flags, gamma,
                             ds->diag, tu.grid, tu.waves, st, w.vl, &seg, dt);
  return run_fused<float>(nullptr, 1, n_groups, g, scheme, reconstruction, riemann, limiter, flags, gamma, ds->diag,
                          tu.grid, tu.waves, st, w.vl, &seg, dt);
}

int hydro_solve_batch(const struct hydro_seg* segs, int n_segs, long long n_groups_total,
                      const struct hydro_spec* spec, void* stream) {
  g_err[0] = 0;
  if (!spec) return fail(HYDRO_EINVAL, "null spec");
  if (int rc = check_options(spec->scheme, spec->reconstruction, spec->riemann, spec->limiter, spec->flags)) return rc;
  if (spec->flags & HYDRO_PLAIN) return fail(HYDRO_EINVAL, "HYDRO_PLAIN is not a batched path");
  if (spec->flags & HYDRO_ROE_FB_EXACT) return fail(HYDRO_EUNSUPPORTED, "the exact fallback runs on the plain path only");
  if (!(spec->gamma > 1.0) || !isfinite(spec->gamma)) return fail(HYDRO_EINVAL, "gamma must exceed 1");
  if (n_groups_total < 0 || n_segs < 0) return fail(HYDRO_EINVAL, "negative sizes");
  if (n_groups_total == 0) return 0;
  if (!segs || n_segs == 0) return fail(HYDRO_EINVAL, "null segment table");
  const int charlim = (spec->flags & HYDRO_CHAR) ? 1 : 0;
  if (!hy::fused_supported(spec->scheme, spec->reconstruction, spec->riemann, charlim))
    return fail(HYDRO_EUNSUPPORTED, "fused path not built for this combination");
  static_assert(sizeof(hydro_seg) == sizeof(hy::Seg), "segment layout");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  const bool f64 = (spec->flags & HYDRO_F64) != 0;
  const int g = ghost_width(spec->scheme, spec->reconstruction);
  const Tune tu = tuned(f64, spec->scheme, spec->reconstruction, spec->riemann, charlim, n_groups_total);
  Workspace& w = ds->ws[st];
  const int box_segs = (spec->flags & HYDRO_BOX_SEGS) ? 1 : 0;
  if (int rc = ensure_vl(w, (size_t)n_groups_total *
                                hy::fused_scratch_per_group(spec->scheme, spec->reconstruction, box_segs) *
                                (f64 ? 8 : 4)))
    return rc;
  const hy::Seg* sd = (const hy::Seg*)segs;
  if (f64)
    return run_fused<double>(sd, n_segs, n_groups_total, g, spec->scheme, spec->reconstruction, spec->riemann,
                             spec->limiter, spec->flags, spec->gamma, ds->diag, tu.grid, tu.waves, st, w.vl, nullptr,
                             0.0, box_segs);
  return run_fused<float>(sd, n_segs, n_groups_total, g, spec->scheme, spec->reconstruction, spec->riemann,
                          spec->limiter, spec->flags, spec->gamma, ds->diag, tu.grid, tu.waves, st, w.vl, nullptr, 0.0,
                          box_segs);
}

int hydro_step_box(const void* box_in, void* box_out, void* flux_out, int nx, int ny, int nz, const double* dt_dev,
                   double dt_scale, double dh, double gamma, int scheme, int reconstruction, int riemann, int limiter,
                   int flags, void* stream) {
  g_err[0] = 0;
  if (int rc = check_options(scheme, reconstruction, riemann, limiter, flags)) return rc;
  if (flags & HYDRO_PLAIN) return fail(HYDRO_EINVAL, "HYDRO_PLAIN is not a box path");
  if (flags & HYDRO_ROE_FB_EXACT) return fail(HYDRO_EUNSUPPORTED, "the exact fallback runs on the plain path only");
  if (!box_in || !box_out || !dt_dev) return fail(HYDRO_EINVAL, "null pointer");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 16 || ny % 16 || nz % 16)
    return fail(HYDRO_EINVAL, "box sizes must be positive multiples of 16");
  if (!(dh > 0.0) || !isfinite(dh) || !(dt_scale > 0.0) || !isfinite(dt_scale))
    return fail(HYDRO_EINVAL, "dh and dt_scale must be positive and finite");
  if (!(gamma > 1.0) || !isfinite(gamma)) return fail(HYDRO_EINVAL, "gamma must exceed 1");
  const int charlim = (flags & HYDRO_CHAR) ? 1 : 0;
  if (!hy::fused_supported(scheme, reconstruction, riemann, charlim))
    return fail(HYDRO_EUNSUPPORTED, "box path not built for this combination");
  const bool f64 = (flags & HYDRO_F64) != 0;
  const size_t esz = f64 ? 8 : 4;
  if ((long long)(nx / 16) * (ny / 16) * 5 * 4096 * (long long)esz >= (1LL << 32))
    return fail(HYDRO_EINVAL, "a z-slab of groups ((nx/16)(ny/16) groups) must hold less than 4 GiB");
  const long long G = (long long)(nx / 16) * (ny / 16) * (nz / 16);
  const int nf = (flags & HYDRO_FLUX_MID) ? 3 : 2;
  const size_t bb = (size_t)G * 5 * 4096 * esz, fb = (size_t)G * 3 * nf * 5 * 256 * esz;
  if (overlap(box_in, bb, box_out, bb)) return fail(HYDRO_EALIAS, "box_in and box_out overlap");
  if (flux_out && (overlap(flux_out, fb, box_in, bb) || overlap(flux_out, fb, box_out, bb)))
    return fail(HYDRO_EALIAS, "flux_out overlaps a box");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  hy::Seg seg{box_in, box_out, flux_out, dt_dev, dt_scale, dh, 0, G, nx / 16, ny / 16, nz / 16, 1};
  const int g = ghost_width(scheme, reconstruction);
  // CTU without flux output marches through runs of z-consecutive groups.
  // Without flux output the workgroups march through runs of z-consecutive
  // groups.
  const Tune tu = !flux_out ? tuned_box(f64, scheme, reconstruction, riemann, limiter, charlim, G, nz / 16)
                            : tuned(f64, scheme, reconstruction, riemann, charlim, G);
  const int zrun = !flux_out ? tu.zrun : 1;
  Workspace& w = ds->ws[st];
  if (int rc = ensure_vl(w, (size_t)G * hy::fused_scratch_per_group(scheme, reconstruction, 1) * esz)) return rc;
  // Passed by value: the kernel reads dt through seg.dt (segs == nullptr and
  // a device dt pointer in seg0).
  // VL: the half step is computed once per cell of the box (wstar_box).
  if (f64)
    return run_fused<double>(nullptr, 1, G, g, scheme, reconstruction, riemann, limiter, flags, gamma, ds->diag,
                             tu.grid, tu.waves, st, w.vl, &seg, -1.0, 1, zrun);
  return run_fused<float>(nullptr, 1, G, g, scheme, reconstruction, riemann, limiter, flags, gamma, ds->diag, tu.grid,
                          tu.waves, st, w.vl, &seg, -1.0, 1, zrun);
}

int hydro_cfl_dt(const void* U, int n_groups, double dh, double gamma, double cfl, int flags, double* dt_out,
                 void* stream) {
  g_err[0] = 0;
  if (n_groups <= 0) return fail(HYDRO_EINVAL, "n_groups must be positive");
  if (!U || !dt_out) return fail(HYDRO_EINVAL, "null pointer");
  if (!(dh > 0.0) || !(gamma > 1.0) || !(cfl > 0.0)) return fail(HYDRO_EINVAL, "dh, cfl > 0 and gamma > 1 required");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  Workspace& w = ds->ws[st];
  if (int rc = ensure_partial(*ds, w)) return rc;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_maxspeed((const double*)U, n_groups, 4096, gamma, w.partial, kPartials, st)
                     : hy::launch_maxspeed((const float*)U, n_groups, 4096, gamma, w.partial, kPartials, st);
  if (e != hipSuccess) return hip_fail(e, "max speed");
  e = hy::launch_dt_finish(w.partial, kPartials, dh, cfl, dt_out, st);
  if (e != hipSuccess) return hip_fail(e, "dt finish");
  return 0;
}

int hydro_cfl_dt_sums(const void* U, int n_groups, double dh, double gamma, double cfl, int flags, double* dt_out,
                      double* sums_out, void* stream) {
  g_err[0] = 0;
  if (n_groups <= 0) return fail(HYDRO_EINVAL, "n_groups must be positive");
  if (!U || !dt_out || !sums_out) return fail(HYDRO_EINVAL, "null pointer");
  if (!(dh > 0.0) || !(gamma > 1.0) || !(cfl > 0.0)) return fail(HYDRO_EINVAL, "dh, cfl > 0 and gamma > 1 required");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  if (overlap(dt_out, sizeof(double), sums_out, 5 * sizeof(double))) return fail(HYDRO_EALIAS, "dt_out overlaps sums_out");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  Workspace& w = ds->ws[st];
  if (int rc = ensure_partial(*ds, w)) return rc;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_dtsums((const double*)U, n_groups, dh, gamma, cfl, w.partial, kPartials, dt_out,
                                         sums_out, st)
                     : hy::launch_dtsums((const float*)U, n_groups, dh, gamma, cfl, w.partial, kPartials, dt_out,
                                         sums_out, st);
  if (e != hipSuccess) return hip_fail(e, "dt and sums");
  return 0;
}

int hydro_cfl_dt_batch(const struct hydro_seg* segs, int n_segs, long long n_groups_total, double gamma, double cfl,
                       int flags, void* stream) {
  g_err[0] = 0;
  if (n_segs < 0 || n_groups_total < 0) return fail(HYDRO_EINVAL, "negative sizes");
  if (n_groups_total == 0) return 0;
  if (!segs || n_segs == 0) return fail(HYDRO_EINVAL, "null segment table");
  if (!(gamma > 1.0) || !(cfl > 0.0)) return fail(HYDRO_EINVAL, "cfl > 0 and gamma > 1 required");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  Workspace& w = ds->ws[st];
  if (w.seg_partial_n < n_groups_total) {
    if (w.seg_partial) {
      hipDeviceSynchronize();
      hipFree(w.seg_partial);
      w.seg_partial = nullptr;
      w.seg_partial_n = 0;
    }
    hipError_t e = hipMalloc((void**)&w.seg_partial, (size_t)n_groups_total * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(dt partials)");
    w.seg_partial_n = n_groups_total;
  }
  hipError_t e = hy::launch_seg_dt((const hy::Seg*)segs, n_segs, n_groups_total, gamma, cfl, (flags & HYDRO_F64) ? 1 : 0,
                                   w.seg_partial, st);
  if (e != hipSuccess) return hip_fail(e, "batched dt");
  return 0;
}

int hydro_cfl_dt_batch_noalloc(const struct hydro_seg* segs, int n_segs, long long n_groups_total, double gamma,
                               double cfl, int flags, void* stream) {
  g_err[0] = 0;
  if (n_segs < 0 || n_groups_total < 0) return fail(HYDRO_EINVAL, "negative sizes");
  if (n_groups_total > HYDRO_NOALLOC_MAX_GROUPS)
    return fail(HYDRO_EINVAL, "n_groups_total %lld exceeds the static scratch of %d groups", n_groups_total,
                HYDRO_NOALLOC_MAX_GROUPS);
  if (n_groups_total == 0) return 0;
  if (!segs || n_segs == 0) return fail(HYDRO_EINVAL, "null segment table");
  if (!(gamma > 1.0) || !(cfl > 0.0)) return fail(HYDRO_EINVAL, "cfl > 0 and gamma > 1 required");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  double* partial;
  if (int rc = scratch_on_device(&partial)) return rc;
  hipError_t e = hy::launch_seg_dt((const hy::Seg*)segs, n_segs, n_groups_total, gamma, cfl, (flags & HYDRO_F64) ? 1 : 0,
                                   partial, st);
  if (e != hipSuccess) return hip_fail(e, "batched dt (static scratch)");
  return 0;
}

int hydro_conserved_sums(const void* U, int n_groups, double dh, int flags, double* sums_out, void* stream) {
  g_err[0] = 0;
  if (n_groups < 0) return fail(HYDRO_EINVAL, "n_groups < 0");
  if (!U || !sums_out) return fail(HYDRO_EINVAL, "null pointer");
  if (!(dh > 0.0)) return fail(HYDRO_EINVAL, "dh must be positive");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  Workspace& w = ds->ws[st];
  if (int rc = ensure_partial(*ds, w)) return rc;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_sums((const double*)U, n_groups, 4096, dh, w.partial, kPartials, sums_out, st)
                     : hy::launch_sums((const float*)U, n_groups, 4096, dh, w.partial, kPartials, sums_out, st);
  if (e != hipSuccess) return hip_fail(e, "conserved sums");
  return 0;
}

int hydro_fill_ghosts_periodic(const void* box, int nx, int ny, int nz, int g, int flags, void* groups_out,
                               void* stream) {
  g_err[0] = 0;
  if (!box || !groups_out) return fail(HYDRO_EINVAL, "null pointer");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 16 || ny % 16 || nz % 16)
    return fail(HYDRO_EINVAL, "box sizes must be positive multiples of 16");
  if (g < 0 || g > 16) return fail(HYDRO_EINVAL, "ghost width out of range");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  if ((long long)(nx / 16) * (ny / 16) * (nz / 16) >= (1LL << 31)) return fail(HYDRO_EINVAL, "2^31 or more groups");
  const size_t esz = (flags & HYDRO_F64) ? 8 : 4;
  const size_t N = 16 + 2 * g;
  const size_t nb = (size_t)nx * ny * nz * 5 * esz;
  const size_t ng = (size_t)(nx / 16) * (ny / 16) * (nz / 16) * 5 * N * N * N * esz;
  if (overlap(box, nb, groups_out, ng)) return fail(HYDRO_EALIAS, "box and groups overlap");
  const int grouped = (flags & HYDRO_BOX_GROUPED) ? 1 : 0;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_fill_periodic((const double*)box, nx, ny, nz, g, grouped, (double*)groups_out, st)
                     : hy::launch_fill_periodic((const float*)box, nx, ny, nz, g, grouped, (float*)groups_out, st);
  if (e != hipSuccess) return hip_fail(e, "ghost fill");
  return 0;
}

int hydro_fill_groups_interp(const void* coarse, int cn, const int* layout, int n_groups, int g, double base_dh,
                             int flags, void* groups_out, void* stream) {
  g_err[0] = 0;
  if (n_groups < 0) return fail(HYDRO_EINVAL, "n_groups < 0");
  if (n_groups == 0) return 0;
  if (!coarse || !layout || !groups_out) return fail(HYDRO_EINVAL, "null pointer");
  if (cn <= 0 || g < 0 || g > 16 || !(base_dh > 0.0)) return fail(HYDRO_EINVAL, "bad sizes");
  if (flags & ~kKnownFlags) return fail(HYDRO_EINVAL, "unknown flag bits");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_fill_interp((const double*)coarse, cn, layout, n_groups, g, base_dh,
                                              (double*)groups_out, st)
                     : hy::launch_fill_interp((const float*)coarse, cn, layout, n_groups, g, base_dh,
                                              (float*)groups_out, st);
  if (e != hipSuccess) return hip_fail(e, "interpolating fill");
  return 0;
}

long long hydro_group_map_len(int ng0, int n_levels) {
  if (ng0 <= 0 || n_levels < 1 || n_levels > HYDRO_MAX_LEVELS) return -1;
  long long len = 0;
  for (int l = 0; l < n_levels; ++l) {
    const long long q = (long long)ng0 << l;
    if (q > (1LL << 20)) return -1;
    len += q * q * q;
    if (len >= (1LL << 31)) return -1;
  }
  return len;
}

int hydro_build_group_map(const int* layout, int n_groups, int ng0, int n_levels, int* map_out, void* stream) {
  g_err[0] = 0;
  const long long len = hydro_group_map_len(ng0, n_levels);
  if (len < 0) return fail(HYDRO_EINVAL, "ng0 > 0 and 1 <= n_levels <= %d with fewer than 2^31 map entries",
                           HYDRO_MAX_LEVELS);
  if (n_groups < 0) return fail(HYDRO_EINVAL, "n_groups < 0");
  if (!map_out || (n_groups > 0 && !layout)) return fail(HYDRO_EINVAL, "null pointer");
  hipError_t e = hy::launch_group_map(layout, n_groups, ng0, n_levels, len, map_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "group map");
  return 0;
}

int hydro_fill_groups_amr(const void* fine, const int* layout, int n_groups, const int* map, int ng0, int n_levels,
                          const void* coarse0, const void* coarse1, int cn, const double* alpha, int g, int flags,
                          void* groups_out, void* stream) {
  g_err[0] = 0;
  if (n_groups < 0) return fail(HYDRO_EINVAL, "n_groups < 0");
  if (hydro_group_map_len(ng0, n_levels) < 0)
    return fail(HYDRO_EINVAL, "ng0 > 0 and 1 <= n_levels <= %d with fewer than 2^31 map entries", HYDRO_MAX_LEVELS);
  if (g < 0 || g > 4) return fail(HYDRO_EINVAL, "ghost width must be 0..4");
  if (cn <= 0 || cn > 4096) return fail(HYDRO_EINVAL, "coarse size out of range");
  if (flags & ~HYDRO_F64) return fail(HYDRO_EINVAL, "only HYDRO_F64 is accepted");
  if (!alpha) return fail(HYDRO_EINVAL, "null alpha");
  for (int l = 0; l < n_levels; ++l)
    if (!(alpha[l] >= 0.0 && alpha[l] <= 1.0)) return fail(HYDRO_EINVAL, "alpha[%d] outside [0, 1]", l);
  if (n_groups == 0) return 0;
  if (!fine || !layout || !map || !coarse0 || !coarse1 || !groups_out) return fail(HYDRO_EINVAL, "null pointer");
  const size_t esz = (flags & HYDRO_F64) ? 8 : 4;
  const size_t N = 16 + 2 * g;
  const size_t ob = (size_t)n_groups * 5 * N * N * N * esz, fb = (size_t)n_groups * 5 * 4096 * esz;
  const size_t cb = (size_t)5 * cn * cn * cn * esz;
  if (overlap(groups_out, ob, fine, fb) || overlap(groups_out, ob, coarse0, cb) || overlap(groups_out, ob, coarse1, cb))
    return fail(HYDRO_EALIAS, "groups_out overlaps an input");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_fill_amr((const double*)fine, layout, n_groups, map, ng0, n_levels,
                                           (const double*)coarse0, (const double*)coarse1, cn, alpha, g,
                                           (double*)groups_out, st)
                     : hy::launch_fill_amr((const float*)fine, layout, n_groups, map, ng0, n_levels,
                                           (const float*)coarse0, (const float*)coarse1, cn, alpha, g,
                                           (float*)groups_out, st);
  if (e != hipSuccess) return hip_fail(e, "AMR preparation");
  return 0;
}

int hydro_amr_correct(void* coarse, int n, const void* coarse_flux, const void* fine, const int* fine_layout,
                      int n_fine, const int* fine_map, const void* fine_flux, double dt, double dh, int flags,
                      void* stream) {
  g_err[0] = 0;
  if (n <= 0 || n % 16 || n > 8192) return fail(HYDRO_EINVAL, "coarse box size must be a positive multiple of 16");
  if (n_fine < 0 || n_fine > (1 << 28)) return fail(HYDRO_EINVAL, "n_fine must be in [0, 2^28]");
  if (!(dt > 0.0) || !isfinite(dt) || !(dh > 0.0) || !isfinite(dh))
    return fail(HYDRO_EINVAL, "dt and dh must be positive and finite");
  if (flags & ~HYDRO_F64) return fail(HYDRO_EINVAL, "only HYDRO_F64 is accepted");
  if (n_fine == 0) return 0;
  if (!coarse || !coarse_flux || !fine || !fine_layout || !fine_map || !fine_flux)
    return fail(HYDRO_EINVAL, "null pointer");
  const size_t esz = (flags & HYDRO_F64) ? 8 : 4;
  const size_t gc = (size_t)(n / 16) * (n / 16) * (n / 16);
  const size_t ub = gc * 5 * 4096 * esz, cfb = gc * 3 * 3 * 5 * 256 * esz;
  const size_t fb = (size_t)n_fine * 5 * 4096 * esz, ffb = (size_t)n_fine * 3 * 2 * 5 * 256 * esz;
  if (overlap(coarse, ub, coarse_flux, cfb) || overlap(coarse, ub, fine, fb) || overlap(coarse, ub, fine_flux, ffb))
    return fail(HYDRO_EALIAS, "the coarse box overlaps an input");
  hipStream_t st = (hipStream_t)stream;
  const double dtdh = dt / dh;
  hipError_t e = (flags & HYDRO_F64)
                     ? hy::launch_amr_correct((double*)coarse, n, (const double*)coarse_flux, (const double*)fine,
                                              fine_layout, n_fine, fine_map, (const double*)fine_flux, dtdh, st)
                     : hy::launch_amr_correct((float*)coarse, n, (const float*)coarse_flux, (const float*)fine,
                                              fine_layout, n_fine, fine_map, (const float*)fine_flux, dtdh, st);
  if (e != hipSuccess) return hip_fail(e, "coarse-grid correction");
  return 0;
}

int hydro_accumulate(void* acc, const void* x, double w, long long n, int flags, void* stream) {
  g_err[0] = 0;
  if (n < 0) return fail(HYDRO_EINVAL, "n < 0");
  if (!isfinite(w)) return fail(HYDRO_EINVAL, "weight must be finite");
  if (flags & ~HYDRO_F64) return fail(HYDRO_EINVAL, "only HYDRO_F64 is accepted");
  if (n == 0) return 0;
  if (!acc || !x) return fail(HYDRO_EINVAL, "null pointer");
  const size_t b = (size_t)n * ((flags & HYDRO_F64) ? 8 : 4);
  if (acc != x && overlap(acc, b, x, b)) return fail(HYDRO_EALIAS, "acc and x overlap partially");
  hipError_t e = (flags & HYDRO_F64) ? hy::launch_axpy((double*)acc, (const double*)x, w, n, (hipStream_t)stream)
                                     : hy::launch_axpy((float*)acc, (const float*)x, w, n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "accumulate");
  return 0;
}

int hydro_get_diag(struct hydro_diag* out, int reset, void* stream) {
  g_err[0] = 0;
  if (!out) return fail(HYDRO_EINVAL, "null output");
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState* ds;
  if (int rc = device_state(&ds)) return rc;
  unsigned long long h[2];
  hipError_t e = hipMemcpyAsync(h, ds->diag, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "diag readback");
  out->roe_fallbacks = h[0];
  out->floor_hits = h[1];
  if (reset) {
    e = hipMemsetAsync(ds->diag, 0, sizeof(h), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "diag reset");
  }
  return 0;
}

int hydro_set_launch_shape(const struct hydro_spec* spec, int grid, int variant, int zrun) {
  g_err[0] = 0;
  if (!spec) return fail(HYDRO_EINVAL, "null spec");
  if (int rc = check_options(spec->scheme, spec->reconstruction, spec->riemann, spec->limiter, spec->flags)) return rc;
  const bool f64 = (spec->flags & HYDRO_F64) != 0;
  if (grid < 0) return fail(HYDRO_EINVAL, "grid %d < 0", grid);
  if (variant != 2 && variant != 4) return fail(HYDRO_EINVAL, "variant %d not in {2, 4}", variant);
  if (f64 && variant != 2) return fail(HYDRO_EINVAL, "FP64 kernels have variant 2 only");
  if (zrun < 0 || zrun > 64) return fail(HYDRO_EINVAL, "zrun %d not in 0..64", zrun);
  const int charlim = (spec->flags & HYDRO_CHAR) ? 1 : 0;
  std::lock_guard<std::mutex> lock(g_mu);
  tune_load();
  g_tune[tune_key(f64, spec->scheme, spec->reconstruction, spec->riemann, charlim)] = Tune{grid, variant, zrun, grid};
  return 0;
}

int hydro_get_launch_shape(const struct hydro_spec* spec, int nx, int ny, int nz, int* grid, int* variant,
                           int* zrun) {
  g_err[0] = 0;
  if (!spec || !grid || !variant || !zrun) return fail(HYDRO_EINVAL, "null pointer");
  if (int rc = check_options(spec->scheme, spec->reconstruction, spec->riemann, spec->limiter, spec->flags)) return rc;
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx % 16 || ny % 16 || nz % 16)
    return fail(HYDRO_EINVAL, "box sizes must be positive multiples of 16");
  const bool f64 = (spec->flags & HYDRO_F64) != 0;
  const int charlim = (spec->flags & HYDRO_CHAR) ? 1 : 0;
  const long long G = (long long)(nx / 16) * (ny / 16) * (nz / 16);
  std::lock_guard<std::mutex> lock(g_mu);
  const Tune t = tuned_box(f64, spec->scheme, spec->reconstruction, spec->riemann, spec->limiter, charlim, G, nz / 16);
  *grid = t.grid;
  *variant = t.waves;
  *zrun = t.zrun;
  return 0;
}

int hydro_autotune(const struct hydro_spec* spec, int n_groups_hint, void* stream) {
  g_err[0] = 0;
  if (!spec) return fail(HYDRO_EINVAL, "null spec");
  if (int rc = check_options(spec->scheme, spec->reconstruction, spec->riemann, spec->limiter, spec->flags)) return rc;
  const int charlim = (spec->flags & HYDRO_CHAR) ? 1 : 0;
  if (!hy::fused_supported(spec->scheme, spec->reconstruction, spec->riemann, charlim))
    return fail(HYDRO_EUNSUPPORTED, "fused path not built for this combination");
  if (n_groups_hint <= 0) return fail(HYDRO_EINVAL, "n_groups_hint must be positive");
  const bool f64 = (spec->flags & HYDRO_F64) != 0;
  const int g = ghost_width(spec->scheme, spec->reconstruction);
  const size_t N = 16 + 2 * g;
  const size_t esz = f64 ? 8 : 4;
  const long long n = n_groups_hint;
  hipStream_t st = (hipStream_t)stream;
  // Synthetic uniform state at rest (rho = 1, p = 1): every path is taken
  // with the same instruction mix, so timings compare launch shapes only.
  void *in = nullptr, *out = nullptr;
  double* dtd = nullptr;
  hy::Seg* sd = nullptr;
  hipError_t e = hipMalloc(&in, (size_t)n * 5 * N * N * N * esz);
  if (e == hipSuccess) e = hipMalloc(&out, (size_t)n * 5 * 4096 * esz);
  if (e == hipSuccess) e = hipMalloc((void**)&dtd, sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&sd, sizeof(hy::Seg));
  if (e != hipSuccess) {
    hipFree(in); hipFree(out); hipFree(dtd); hipFree(sd);
    return hip_fail(e, "autotune buffers");
  }
  {
    const size_t nc = N * N * N;
    std::vector<char> host(5 * nc * esz);
    for (size_t q = 0; q < nc; ++q) {
      double v[5] = {1.0, 0.0, 0.0, 0.0, 1.0 / (spec->gamma - 1.0)};
      for (int k = 0; k < 5; ++k) {
        if (f64) ((double*)host.data())[k * nc + q] = v[k];
        else ((float*)host.data())[k * nc + q] = (float)v[k];
      }
    }
    for (long long q = 0; q < n && e == hipSuccess; ++q)
      e = hipMemcpyAsync((char*)in + q * host.size(), host.data(), host.size(), hipMemcpyHostToDevice, st);
    double dt = 1e-4;
    hy::Seg s{in, out, nullptr, dtd, 1.0, 1.0 / 256, 0, n, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(dtd, &dt, sizeof(dt), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sd, &s, sizeof(s), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  const int cus = cu_count();
  DeviceState* ds = nullptr;
  void* vl = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (int rc = device_state(&ds)) { hipFree(in); hipFree(out); hipFree(dtd); hipFree(sd); return rc; }
    Workspace& w = ds->ws[st];
    if (int rc = ensure_vl(w, (size_t)n * hy::fused_scratch_per_group(spec->scheme, spec->reconstruction, 0) * esz)) {
      hipFree(in); hipFree(out); hipFree(dtd); hipFree(sd);
      return rc;
    }
    vl = w.vl;
  }
  // Candidates: register variant x persistent grid (multiples of the CU count).
  const int mults[] = {1, 2, 3, 4, 6, 8, 12, 16};
  const int variants[] = {2, 4};
  Tune best{-1, 2, 0, 0};
  float best_ms = 1e30f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int wv : variants) {
    if (f64 && wv != 2) continue;
    for (int m : mults) {
      if (e != hipSuccess) break;
      long long grid = (long long)cus * m;
      if (grid > n) grid = n;
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        int rc = f64 ? run_fused<double>(sd, 1, n, g, spec->scheme, spec->reconstruction, spec->riemann,
                                         spec->limiter, spec->flags, spec->gamma, ds->diag, (int)grid, wv, st, vl)
                     : run_fused<float>(sd, 1, n, g, spec->scheme, spec->reconstruction, spec->riemann,
                                        spec->limiter, spec->flags, spec->gamma, ds->diag, (int)grid, wv, st, vl);
        if (rc) { e = hipErrorLaunchFailure; break; }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && ms < ms_min) ms_min = ms;  // the first launch is a warm-up
      }
      if (ms_min < best_ms) { best_ms = ms_min; best = Tune{(int)grid, wv, 0, 0}; }
      if (grid == n) break;
    }
  }
  // Box steps: tile depth (z-run length) x grid, with the register variant
  // just chosen, on a synthetic periodic box of the same number of groups
  // (ngz and ngy the largest powers of two up to 16 that divide it).
  if (e == hipSuccess && best.grid > 0) {
    int ngz = 1, ngy = 1;
    while (ngz < 16 && n % (2 * ngz) == 0) ngz *= 2;
    while (ngy < 16 && (n / ngz) % (2 * ngy) == 0) ngy *= 2;
    const long long ngx = n / ngz / ngy;
    {
      std::vector<char> host((size_t)5 * 4096 * esz);
      for (size_t q = 0; q < 4096; ++q) {
        double v[5] = {1.0, 0.0, 0.0, 0.0, 1.0 / (spec->gamma - 1.0)};
        for (int k = 0; k < 5; ++k) {
          if (f64) ((double*)host.data())[k * 4096 + q] = v[k];
          else ((float*)host.data())[k * 4096 + q] = (float)v[k];
        }
      }
      for (long long q = 0; q < n && e == hipSuccess; ++q)
        e = hipMemcpyAsync((char*)in + q * host.size(), host.data(), host.size(), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    hy::Seg bs{in, out, nullptr, dtd, 1.0, 1.0 / 256, 0, n, (int)ngx, ngy, ngz, 1};
    float best_box = 1e30f;
    for (int zr : {1, 2, 4}) {
      if (ngz % zr || e != hipSuccess) continue;
      if (!hy::zrun_built(spec->scheme, f64, best.waves, spec->reconstruction, spec->limiter, charlim, zr)) continue;
      const long long items = n / zr;
      for (int m : mults) {
        long long grid = (long long)cus * m;
        if (grid > items) grid = items;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, st);
          int rc = f64 ? run_fused<double>(nullptr, 1, n, g, spec->scheme, spec->reconstruction, spec->riemann,
                                           spec->limiter, spec->flags, spec->gamma, ds->diag, (int)grid, best.waves,
                                           st, vl, &bs, -1.0, 1, zr)
                       : run_fused<float>(nullptr, 1, n, g, spec->scheme, spec->reconstruction, spec->riemann,
                                          spec->limiter, spec->flags, spec->gamma, ds->diag, (int)grid, best.waves,
                                          st, vl, &bs, -1.0, 1, zr);
          if (rc) { e = hipErrorLaunchFailure; break; }
          if (e == hipSuccess) e = hipEventRecord(e1, st);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0 && ms < ms_min) ms_min = ms;
        }
        if (ms_min < best_box) { best_box = ms_min; best.zrun = zr; best.grid_box = (int)grid; }
        if (grid == items) break;
      }
    }
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(in); hipFree(out); hipFree(dtd); hipFree(sd);
  if (e != hipSuccess || best.grid < 0) return hip_fail(e == hipSuccess ? hipErrorUnknown : e, "autotune");
  std::lock_guard<std::mutex> lock(g_mu);
  tune_load();
  const std::string key = tune_key(f64, spec->scheme, spec->reconstruction, spec->riemann, charlim);
  g_tune[key] = best;
  if (const char* path = getenv("HYDRO_TUNE_CACHE")) {
    if (FILE* f = fopen(path, "a")) {
      fprintf(f, "%s %d %d %d %d\n", key.c_str(), best.grid, best.waves, best.zrun, best.grid_box);
      fclose(f);
    }
  }
  return best.grid;
}

void hydro_shutdown(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  hipDeviceSynchronize();
  for (auto& kv : g_dev) {
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(kv.first);
    for (auto& w : kv.second.ws) {
      if (w.second.plain) hipFree(w.second.plain);
      if (w.second.vl) hipFree(w.second.vl);
      if (w.second.seg_partial) hipFree(w.second.seg_partial);
      if (w.second.partial && w.second.own_partial) hipFree(w.second.partial);
    }
    if (kv.second.diag) hipFree(kv.second.diag);
    if (kv.second.partial_pool) hipFree(kv.second.partial_pool);
    hipSetDevice(prev);
  }
  g_dev.clear();
  g_tune.clear();
  g_tune_loaded = false;
}

}  // extern "C"
