// Auxiliary kernels around the solver:
//  * preparation step (paper Sec. 4.2): periodic ghost fill of patch groups
//    from a resident box, and trilinear fill of AMR-shaped groups from a
//    coarse field (spatial interpolation at coarse-fine boundaries);
//  * FP64 CFL time step: max signal speed per block (wave64 shuffles), then a
//    single-block finish, dt = cfl * dh / max (max is order-free, so the
//    result is deterministic and equals a serial evaluation bit for bit);
//  * FP64 conserved sums with a fixed two-level reduction order.
#include <limits.h>

#include "hydro_internal.h"

namespace hy {

// ---------------------------------------------------------------------------
// Periodic ghost fill.  Output groups [G][5][N][N][N], G = (gz*ngy+gy)*ngx+gx.
// Source either a plain box [5][nz][ny][nx] or the grouped interior layout
// [G][5][16][16][16] (grouped != 0).  One thread per output cell, x fastest.
// ---------------------------------------------------------------------------
// GC > 0: the ghost width fixed at compile time (no run-time integer
// division per cell); GC == 0: g taken at run time.
template <typename T, int GC>
__global__ void __launch_bounds__(512) fill_periodic_kernel(const T* __restrict__ box, int nx, int ny, int nz, int g_rt,
                                                            int grouped, T* __restrict__ out, long long g_off) {
  // blockIdx.x = k in 0 .. N/2-1: the workgroup fills planes k and k + N/2
  // of the padded group (N = 16 + 2g is even), all ten loads of a thread
  // issued before its stores; blockIdx.y = group; threads cover the N x N
  // plane, x fastest (coalesced writes).  Group counts stay below 2^31 (the
  // caller checks), so the group coordinates use 32-bit division.
  const int g = GC > 0 ? GC : g_rt;
  const int N = 16 + 2 * g;
  const long long nc = (long long)N * N * N;
  const int H = N / 2;
  const int k = blockIdx.x;
  const unsigned G = (unsigned)(g_off + blockIdx.y);
  const unsigned ngx = (unsigned)nx >> 4, ngy = (unsigned)ny >> 4;
  const long long boxc = (long long)nx * ny * nz;
  const int gx = (int)(G % ngx), gy = (int)((G / ngx) % ngy), gz = (int)(G / ngx / ngy);
  int sz0 = gz * 16 + k - g, sz1 = sz0 + H;
  sz0 += (sz0 < 0) ? nz : 0;
  sz0 -= (sz0 >= nz) ? nz : 0;
  sz1 += (sz1 < 0) ? nz : 0;
  sz1 -= (sz1 >= nz) ? nz : 0;
  T* o = out + (long long)G * 5 * nc + (long long)k * N * N;
  const long long oH = (long long)H * N * N;
  for (int r = threadIdx.x; r < N * N; r += blockDim.x) {
    const int i = r % N, j = r / N;
    int sx = gx * 16 + i - g, sy = gy * 16 + j - g;
    sx += (sx < 0) ? nx : 0; sx -= (sx >= nx) ? nx : 0;
    sy += (sy < 0) ? ny : 0; sy -= (sy >= ny) ? ny : 0;
    T v0[5], v1[5];
    if (grouped) {
      const long long base = ((long long)(sy >> 4) * ngx + (sx >> 4));
      const long long sg0 = (long long)(sz0 >> 4) * ngy * ngx + base, sg1 = (long long)(sz1 >> 4) * ngy * ngx + base;
      const int in = ((sy & 15) * 16 + (sx & 15));
      const T* s0 = box + sg0 * 5 * 4096 + (sz0 & 15) * 256 + in;
      const T* s1 = box + sg1 * 5 * 4096 + (sz1 & 15) * 256 + in;
#pragma unroll
      for (int n = 0; n < 5; ++n) { v0[n] = s0[n * 4096]; v1[n] = s1[n * 4096]; }
    } else {
      const T* s0 = box + ((long long)sz0 * ny + sy) * nx + sx;
      const T* s1 = box + ((long long)sz1 * ny + sy) * nx + sx;
#pragma unroll
      for (int n = 0; n < 5; ++n) { v0[n] = s0[n * boxc]; v1[n] = s1[n * boxc]; }
    }
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      o[n * nc + r] = v0[n];
      o[n * nc + oH + r] = v1[n];
    }
  }
}

template <typename T>
hipError_t launch_fill_periodic(const T* box, int nx, int ny, int nz, int g, int grouped, T* out, hipStream_t st) {
  const int N = 16 + 2 * g;
  const long long groups = (long long)(nx / 16) * (ny / 16) * (nz / 16);
  if (groups == 0) return hipSuccess;
  // grid.y is limited to 65535 groups per launch.
  for (long long g0 = 0; g0 < groups; g0 += 65535) {
    const long long cnt = groups - g0 < 65535 ? groups - g0 : 65535;
    const dim3 grid(N / 2, (unsigned)cnt);
    switch (g) {
      case 2: fill_periodic_kernel<T, 2><<<grid, dim3(512), 0, st>>>(box, nx, ny, nz, g, grouped, out, g0); break;
      case 3: fill_periodic_kernel<T, 3><<<grid, dim3(512), 0, st>>>(box, nx, ny, nz, g, grouped, out, g0); break;
      case 4: fill_periodic_kernel<T, 4><<<grid, dim3(512), 0, st>>>(box, nx, ny, nz, g, grouped, out, g0); break;
      default: fill_periodic_kernel<T, 0><<<grid, dim3(512), 0, st>>>(box, nx, ny, nz, g, grouped, out, g0); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
template hipError_t launch_fill_periodic<float>(const float*, int, int, int, int, int, float*, hipStream_t);
template hipError_t launch_fill_periodic<double>(const double*, int, int, int, int, int, double*, hipStream_t);

// ---------------------------------------------------------------------------
// AMR-shaped preparation: every cell of every padded group is the trilinear
// interpolation, at its centre, of a periodic coarse field [5][cn][cn][cn]
// on the unit box.  layout[G] = (level, ox, oy, oz): the group's first
// interior cell on the level-l grid of spacing base_dh / 2^l.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) fill_interp_kernel(const T* __restrict__ coarse, int cn,
                                                          const int4* __restrict__ layout, int g, double base_dh,
                                                          T* __restrict__ out, long long total) {
  const int N = 16 + 2 * g;
  const long long nc = (long long)N * N * N;
  const long long cc = (long long)cn * cn * cn;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const long long G = t / nc;
    const int r = (int)(t - G * nc);
    const int i = r % N, j = (r / N) % N, k = r / (N * N);
    const int4 L = layout[G];
    const double dh = base_dh / (double)(1 << L.x);
    // Coarse-index coordinates of the fine cell centre.
    const double X = ((double)(L.y + i - g) + 0.5) * dh * cn - 0.5;
    const double Y = ((double)(L.z + j - g) + 0.5) * dh * cn - 0.5;
    const double Z = ((double)(L.w + k - g) + 0.5) * dh * cn - 0.5;
    const double fx0 = floor(X), fy0 = floor(Y), fz0 = floor(Z);
    const double ax = X - fx0, ay = Y - fy0, az = Z - fz0;
    int x0 = (int)fx0, y0 = (int)fy0, z0 = (int)fz0;
    x0 = ((x0 % cn) + cn) % cn; y0 = ((y0 % cn) + cn) % cn; z0 = ((z0 % cn) + cn) % cn;
    const int x1 = (x0 + 1) % cn, y1 = (y0 + 1) % cn, z1 = (z0 + 1) % cn;
    const long long c000 = ((long long)z0 * cn + y0) * cn + x0, c001 = ((long long)z0 * cn + y0) * cn + x1;
    const long long c010 = ((long long)z0 * cn + y1) * cn + x0, c011 = ((long long)z0 * cn + y1) * cn + x1;
    const long long c100 = ((long long)z1 * cn + y0) * cn + x0, c101 = ((long long)z1 * cn + y0) * cn + x1;
    const long long c110 = ((long long)z1 * cn + y1) * cn + x0, c111 = ((long long)z1 * cn + y1) * cn + x1;
    T* o = out + G * 5 * nc + r;
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      const T* f = coarse + n * cc;
      const double v00 = (1.0 - ax) * (double)f[c000] + ax * (double)f[c001];
      const double v01 = (1.0 - ax) * (double)f[c010] + ax * (double)f[c011];
      const double v10 = (1.0 - ax) * (double)f[c100] + ax * (double)f[c101];
      const double v11 = (1.0 - ax) * (double)f[c110] + ax * (double)f[c111];
      const double v0 = (1.0 - ay) * v00 + ay * v01;
      const double v1 = (1.0 - ay) * v10 + ay * v11;
      o[n * nc] = (T)((1.0 - az) * v0 + az * v1);
    }
  }
}

// The same interpolation with one workgroup per group and one thread per
// (x, y) column of its padded region, the ghost width fixed at compile time.
// A column's x and y weights and coarse indices are formed once.  Along z,
// the value of a fine cell is the z blend of the x-y interpolations at the
// two coarse layers that bracket it.  Where the fine level is finer than the
// coarse field, the pair stays the same over several consecutive fine planes
// and moves by one layer at a time, so each thread keeps both layers' x-y
// values in registers and reads the coarse field only for a new layer.
// Every value is formed by the expressions of fill_interp_kernel, in the
// same order and without contraction, so the results are those of a plain
// FP64 evaluation.
__device__ __forceinline__ int wrap_index(long long v, int n) {
  if (v < 0 || v >= n) {  // ghost cells across the periodic boundary
    v %= n;
    if (v < 0) v += n;
  }
  return (int)v;
}
template <int G> constexpr int interp_threads() { return ((16 + 2 * G) * (16 + 2 * G) + 63) / 64 * 64; }

template <typename T, int G>
__global__ void __launch_bounds__(interp_threads<G>()) fill_interp_group_kernel(const T* __restrict__ coarse, int cn,
                                                                               const int4* __restrict__ layout,
                                                                               double base_dh, T* __restrict__ out) {
#pragma clang fp contract(off)
  constexpr int N = 16 + 2 * G;
  constexpr long long nc = (long long)N * N * N;
  const long long cc = (long long)cn * cn * cn;
  const long long grp = blockIdx.x;
  const int4 L = layout[grp];
  const double dh = base_dh / (double)(1 << L.x);
  const int r = threadIdx.x;
  if (r >= N * N) return;  // no barrier below
  const int i = r % N, j = r / N;
  const double X = ((double)(L.y + i - G) + 0.5) * dh * cn - 0.5;
  const double Y = ((double)(L.z + j - G) + 0.5) * dh * cn - 0.5;
  const double fx0 = floor(X), fy0 = floor(Y);
  const double ax = X - fx0, ay = Y - fy0;
  const int x0 = wrap_index((long long)fx0, cn), y0 = wrap_index((long long)fy0, cn);
  const int x1 = x0 + 1 == cn ? 0 : x0 + 1, y1 = y0 + 1 == cn ? 0 : y0 + 1;
  // x-y interpolation of layer z of variable n at this column.
  auto layer = [&](int z, int n) -> double {
    const T* f = coarse + n * cc + (long long)z * cn * cn;
    const double v00 = (1.0 - ax) * (double)f[y0 * cn + x0] + ax * (double)f[y0 * cn + x1];
    const double v01 = (1.0 - ax) * (double)f[y1 * cn + x0] + ax * (double)f[y1 * cn + x1];
    return (1.0 - ay) * v00 + ay * v01;
  };
  T* o = out + grp * 5 * nc + r;
  double v0[5], v1[5];
  int zc = -1;  // coarse layer of v0 (none yet)
  for (int k = 0; k < N; ++k) {
    const double Z = ((double)(L.w + k - G) + 0.5) * dh * cn - 0.5;
    const double fz0 = floor(Z);
    const double az = Z - fz0;
    const int z0 = wrap_index((long long)fz0, cn), z1 = z0 + 1 == cn ? 0 : z0 + 1;
    if (z0 != zc) {  // uniform over the workgroup
      const bool shift = zc >= 0 && z0 == (zc + 1 == cn ? 0 : zc + 1);
#pragma unroll
      for (int n = 0; n < 5; ++n) {
        v0[n] = shift ? v1[n] : layer(z0, n);
        v1[n] = layer(z1, n);
      }
      zc = z0;
    }
#pragma unroll
    for (int n = 0; n < 5; ++n) o[n * nc + (long long)k * N * N] = (T)((1.0 - az) * v0[n] + az * v1[n]);
  }
}

template <typename T, int G>
static hipError_t launch_interp_groups(const T* coarse, int cn, const int* layout, long long n_groups, double base_dh,
                                       T* out, hipStream_t st) {
  fill_interp_group_kernel<T, G><<<dim3((unsigned)n_groups), dim3(interp_threads<G>()), 0, st>>>(
      coarse, cn, (const int4*)layout, base_dh, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AMR preparation step for groups next to coarse-fine boundaries (Sec. 4.2:
// ghost data by spatial and temporal interpolation).  Level l spans the
// periodic unit box with ng_l = ng0 << l groups (16 ng_l cells) per side;
// the group map holds, per level, the index of the group at each group
// position or -1: map[off_l + (gz ng_l + gy) ng_l + gx], off_l = sum over
// m < l of ng_m^3.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) fill_int_kernel(int* __restrict__ p, long long n, int v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}
// Group origins off the level's 16-cell grid or outside it, and levels out of
// range, are left out; where two groups share a position the higher index
// wins (atomicMax), so the map does not depend on scheduling.
__global__ void __launch_bounds__(256) group_map_kernel(const int4* __restrict__ layout, int n_groups, int ng0,
                                                        int n_levels, int* __restrict__ map) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= n_groups) return;
  const int4 L = layout[G];
  if (L.x < 0 || L.x >= n_levels) return;
  const long long ng = (long long)ng0 << L.x, nl = 16 * ng;
  if (L.y < 0 || L.z < 0 || L.w < 0 || L.y >= nl || L.z >= nl || L.w >= nl || ((L.y | L.z | L.w) & 15)) return;
  long long off = 0;
  for (int m = 0; m < L.x; ++m) {
    const long long q = (long long)ng0 << m;
    off += q * q * q;
  }
  atomicMax(&map[off + ((long long)(L.w >> 4) * ng + (L.z >> 4)) * ng + (L.y >> 4)], G);
}

hipError_t launch_group_map(const int* layout, int n_groups, int ng0, int n_levels, long long map_len, int* map,
                            hipStream_t st) {
  long long blocks = (map_len + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  fill_int_kernel<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(map, map_len, -1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_groups == 0) return e;
  group_map_kernel<<<dim3((unsigned)((n_groups + 255) / 256)), dim3(256), 0, st>>>((const int4*)layout, n_groups, ng0,
                                                                                  n_levels, map);
  return hipGetLastError();
}

// One workgroup per group, one thread per (x, y) column of its padded
// region, marching along z.  A cell is the group's own interior value, else
// the value of the same-level group that the map places at its (periodic)
// position, else the coarse state blended in time, (1 - alpha_l) coarse0 +
// alpha_l coarse1 at the four coarse points of a layer, interpolated in x
// and y and then in z between the two layers that bracket the cell; a
// thread keeps both layers' values and recomputes them only when the pair
// moves.  When the coarse points that the group's padded region touches fit
// in kFoot^3 (levels at least about 4x finer than the coarse field), the
// workgroup first blends them once into LDS and the columns interpolate
// from there; otherwise every column blends from global memory.  Both give
// the same values.  No contraction: a plain FP64 evaluation of that
// expression.  Map entries outside [0, n_groups) count as empty, and levels
// are clamped into range, so every access stays inside the arrays whatever
// the layout holds.
template <typename T>
struct AmrArgs {
  const T* fine;       // [n][5][16][16][16]
  const int4* layout;  // [n] (level, ox, oy, oz)
  const int* map;
  const T* c0;         // [5][cn][cn][cn]
  const T* c1;
  T* out;              // [n][5][N][N][N]
  int n_groups, ng0, n_levels, cn;
  double alpha[8];
};

constexpr int kFoot = 8;  // coarse points per axis staged in LDS

template <typename T, int G>
__global__ void __launch_bounds__(interp_threads<G>()) fill_amr_group_kernel(AmrArgs<T> a) {
#pragma clang fp contract(off)
  constexpr int N = 16 + 2 * G;
  constexpr long long nc = (long long)N * N * N;
  __shared__ double sB[5][kFoot * kFoot * kFoot];  // blended coarse footprint, [n][z][y][x]
  const int cn = a.cn;
  const long long cc = (long long)cn * cn * cn;
  const long long grp = blockIdx.x;
  const int4 L = a.layout[grp];
  const int r = threadIdx.x;
  const int lev = L.x < 0 ? 0 : (L.x >= a.n_levels ? a.n_levels - 1 : L.x);
  const long long ng = (long long)a.ng0 << lev;
  const int nl = (int)(16 * ng);
  long long moff = 0;
  for (int m = 0; m < lev; ++m) {
    const long long q = (long long)a.ng0 << m;
    moff += q * q * q;
  }
  const double dh = 1.0 / (double)nl;
  const double al = a.alpha[lev];
  // Coarse-index coordinate of the centre of padded-region cell c (-G .. 15+G)
  // along an axis whose group origin is o.
  auto coord = [&](int o, int c) -> double { return (((double)o + c) + 0.5) * dh * cn - 0.5; };
  // Footprint: unwrapped coarse indices lo .. lo + W - 1 per axis.
  const int lox = (int)floor(coord(L.y, -G)), loy = (int)floor(coord(L.z, -G)), loz = (int)floor(coord(L.w, -G));
  const int wx = (int)floor(coord(L.y, 15 + G)) + 2 - lox, wy = (int)floor(coord(L.z, 15 + G)) + 2 - loy,
            wz = (int)floor(coord(L.w, 15 + G)) + 2 - loz;
  // Uniform over the workgroup.  Origins outside the level take the direct
  // path, whose indices all wrap.
  const bool staged = L.y >= 0 && L.y < nl && L.z >= 0 && L.z < nl && L.w >= 0 && L.w < nl && wx <= kFoot &&
                      wy <= kFoot && wz <= kFoot;
  if (staged) {
    for (int q = r; q < 5 * kFoot * kFoot * kFoot; q += blockDim.x) {
      const int n = q / (kFoot * kFoot * kFoot), p = q % (kFoot * kFoot * kFoot);
      const int ix = p % kFoot, iy = (p / kFoot) % kFoot, iz = p / (kFoot * kFoot);
      if (ix < wx && iy < wy && iz < wz) {
        const long long g = (long long)n * cc +
                            ((long long)wrap_index((long long)loz + iz, cn) * cn + wrap_index((long long)loy + iy, cn)) *
                                cn +
                            wrap_index((long long)lox + ix, cn);
        sB[n][p] = (1.0 - al) * (double)a.c0[g] + al * (double)a.c1[g];
      }
    }
    __syncthreads();
  }
  if (r >= N * N) return;  // no barrier below
  const int ci = r % N - G, cj = r / N - G;
  const bool in_xy = ci >= 0 && ci < 16 && cj >= 0 && cj < 16;
  const int px = wrap_index((long long)L.y + ci, nl), py = wrap_index((long long)L.z + cj, nl);
  const double X = coord(L.y, ci), Y = coord(L.z, cj);
  const double fx0 = floor(X), fy0 = floor(Y);
  const double ax = X - fx0, ay = Y - fy0;
  const int x0 = wrap_index((long long)fx0, cn), y0 = wrap_index((long long)fy0, cn);
  const int x1 = x0 + 1 == cn ? 0 : x0 + 1, y1 = y0 + 1 == cn ? 0 : y0 + 1;
  const int sx = (int)fx0 - lox, sy = (int)fy0 - loy;  // staged footprint indices
  // x-y interpolation of layer z (unwrapped coarse index) of variable n.
  auto layer = [&](int zu, int n) -> double {
    if (staged) {
      const double* f = sB[n] + (zu - loz) * kFoot * kFoot;
      const double v00 = (1.0 - ax) * f[sy * kFoot + sx] + ax * f[sy * kFoot + sx + 1];
      const double v01 = (1.0 - ax) * f[(sy + 1) * kFoot + sx] + ax * f[(sy + 1) * kFoot + sx + 1];
      return (1.0 - ay) * v00 + ay * v01;
    }
    const long long base = (long long)n * cc + (long long)wrap_index(zu, cn) * cn * cn;
    const T* f0 = a.c0 + base;
    const T* f1 = a.c1 + base;
    auto b = [&](int q) -> double { return (1.0 - al) * (double)f0[q] + al * (double)f1[q]; };
    const double v00 = (1.0 - ax) * b(y0 * cn + x0) + ax * b(y0 * cn + x1);
    const double v01 = (1.0 - ax) * b(y1 * cn + x0) + ax * b(y1 * cn + x1);
    return (1.0 - ay) * v00 + ay * v01;
  };
  const T* own = a.fine + grp * 5 * 4096;
  T* o = a.out + grp * 5 * nc + r;
  // The column meets three group positions along z (below, its own, above;
  // G < 16): their map entries are read once, before the march.
  int owner3[3];
  {
    const long long gzc = wrap_index((long long)L.w, nl) >> 4;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      long long gz = gzc + t - 1;
      gz += gz < 0 ? ng : 0;
      gz -= gz >= ng ? ng : 0;
      const int ow = a.map[moff + (gz * ng + (py >> 4)) * ng + (px >> 4)];
      owner3[t] = (ow >= 0 && ow < a.n_groups) ? ow : -1;
    }
  }
  double v0[5], v1[5];
  long long zc = LLONG_MIN;  // unwrapped coarse layer of v0 (none yet)
  for (int k = 0; k < N; ++k) {
    const int ck = k - G;
    T val[5];
    if (in_xy && ck >= 0 && ck < 16) {
#pragma unroll
      for (int n = 0; n < 5; ++n) val[n] = own[n * 4096 + (ck * 16 + cj) * 16 + ci];
    } else {
      const int pz = wrap_index((long long)L.w + ck, nl);
      const int owner = owner3[ck < 0 ? 0 : (ck < 16 ? 1 : 2)];
      if (owner >= 0) {
        const T* s = a.fine + (long long)owner * 5 * 4096 + ((pz & 15) * 16 + (py & 15)) * 16 + (px & 15);
#pragma unroll
        for (int n = 0; n < 5; ++n) val[n] = s[n * 4096];
      } else {
        const double Z = coord(L.w, ck);
        const double fz0 = floor(Z);
        const double az = Z - fz0;
        const long long z0 = (long long)fz0;
        if (z0 != zc) {
          const bool shift = z0 == zc + 1;
#pragma unroll
          for (int n = 0; n < 5; ++n) {
            v0[n] = shift ? v1[n] : layer((int)z0, n);
            v1[n] = layer((int)z0 + 1, n);
          }
          zc = z0;
        }
#pragma unroll
        for (int n = 0; n < 5; ++n) val[n] = (T)((1.0 - az) * v0[n] + az * v1[n]);
      }
    }
#pragma unroll
    for (int n = 0; n < 5; ++n) o[n * nc + (long long)k * N * N] = val[n];
  }
}

template <typename T, int G>
static hipError_t launch_amr_g(const AmrArgs<T>& a, hipStream_t st) {
  fill_amr_group_kernel<T, G><<<dim3((unsigned)a.n_groups), dim3(interp_threads<G>()), 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_amr(const T* fine, const int* layout, int n_groups, const int* map, int ng0, int n_levels,
                           const T* c0, const T* c1, int cn, const double* alpha, int g, T* out, hipStream_t st) {
  if (n_groups == 0) return hipSuccess;
  AmrArgs<T> a;
  a.fine = fine;
  a.layout = (const int4*)layout;
  a.map = map;
  a.c0 = c0;
  a.c1 = c1;
  a.out = out;
  a.n_groups = n_groups;
  a.ng0 = ng0;
  a.n_levels = n_levels;
  a.cn = cn;
  for (int l = 0; l < 8; ++l) a.alpha[l] = l < n_levels ? alpha[l] : 0.0;
  switch (g) {
    case 0: return launch_amr_g<T, 0>(a, st);
    case 1: return launch_amr_g<T, 1>(a, st);
    case 2: return launch_amr_g<T, 2>(a, st);
    case 3: return launch_amr_g<T, 3>(a, st);
    case 4: return launch_amr_g<T, 4>(a, st);
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_fill_amr<float>(const float*, const int*, int, const int*, int, int, const float*,
                                           const float*, int, const double*, int, float*, hipStream_t);
template hipError_t launch_fill_amr<double>(const double*, const int*, int, const int*, int, int, const double*,
                                            const double*, int, const double*, int, double*, hipStream_t);

// ---------------------------------------------------------------------------
// Coarse-grid correction after a coarse step (Sec. 2 step 5, Sec. 4.3): the
// coarse level is a periodic n^3 box in patch-group order, the fine level
// has ratio 2 and its groups (fine-grid origins on the 16-cell grid) each
// cover one 8^3 coarse patch; fmap is the fine level's group map (n / 8
// groups per side).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fine_owner(const int* fmap, int nf, int ngf, int cx, int cy, int cz) {
  const int o = fmap[((long long)(cz >> 3) * ngf + (cy >> 3)) * ngf + (cx >> 3)];
  return (o >= 0 && o < nf) ? o : -1;
}

// Refluxing.  An uncovered coarse cell next to a covered one across a face
// replaces the coarse flux of that face (stored by the coarse step on the
// patch faces: group faces -, + and the mid plane) by the mean of the four
// fine fluxes on it: U -= dt/dh (Ff - Fc) when the fine cell lies on its +
// side, += on its - side, in the order x, y, z and -, +.  No contraction:
// the same FP64 expression as a plain evaluation.
//
// One 64-thread workgroup per face of a fine group, one thread per coarse
// cell just outside that face (8 x 8).  A cell next to several refined
// patches is visited from several faces; only the face of its first covered
// neighbour in the order above processes it, applying all of its
// corrections in that order, so every cell is written by one thread.
template <typename T>
__global__ void __launch_bounds__(64) reflux_kernel(T* __restrict__ U, int n, const T* __restrict__ cflux,
                                                    const int* __restrict__ fmap, int nf, const T* __restrict__ fflux,
                                                    const int4* __restrict__ flayout, double dtdh) {
#pragma clang fp contract(off)
  const int F0 = blockIdx.x / 6, face = blockIdx.x % 6;
  const int dF = face >> 1, sF = (face & 1) ? 1 : -1;  // the fine group's face: axis and side
  const int4 o0 = flayout[F0];
  const int nfine = 2 * n, ng = n >> 4, ngf = n >> 3;
  if (o0.y < 0 || o0.z < 0 || o0.w < 0 || o0.y >= nfine || o0.z >= nfine || o0.w >= nfine ||
      ((o0.y | o0.z | o0.w) & 15))
    return;
  const int c0[3] = {o0.y >> 1, o0.z >> 1, o0.w >> 1};
  if (fine_owner(fmap, nf, ngf, c0[0], c0[1], c0[2]) != F0) return;
  // The coarse cell a outside this face; from a, the refined patch lies on
  // side -sF along dF.
  const int e1 = dF == 0 ? 1 : 0, e2 = dF == 2 ? 1 : 2;
  int c[3];
  c[dF] = sF < 0 ? c0[dF] - 1 : c0[dF] + 8;
  c[dF] += c[dF] < 0 ? n : 0;
  c[dF] -= c[dF] >= n ? n : 0;
  c[e1] = c0[e1] + (threadIdx.x & 7);
  c[e2] = c0[e2] + (threadIdx.x >> 3);
  if (fine_owner(fmap, nf, ngf, c[0], c[1], c[2]) >= 0) return;  // covered: restriction sets it
  int owners[6];
  int first = -1;
  for (int q = 0; q < 6; ++q) {
    const int d = q >> 1, side = (q & 1) ? 1 : -1;
    int b[3] = {c[0], c[1], c[2]};
    b[d] += side;
    b[d] += b[d] < 0 ? n : 0;
    b[d] -= b[d] >= n ? n : 0;
    owners[q] = fine_owner(fmap, nf, ngf, b[0], b[1], b[2]);
    if (owners[q] >= 0 && first < 0) first = q;
  }
  if (first != dF * 2 + (sF < 0 ? 1 : 0)) return;  // another face processes this cell
  const long long G = ((long long)(c[2] >> 4) * ng + (c[1] >> 4)) * ng + (c[0] >> 4);
  const int l = ((c[2] & 15) * 16 + (c[1] & 15)) * 16 + (c[0] & 15);
  const int loc[3] = {c[0] & 15, c[1] & 15, c[2] & 15};
  double u[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = (double)U[(G * 5 + v) * 4096 + l];
  for (int q = 0; q < 6; ++q) {
    const int F = owners[q];
    if (F < 0) continue;
    const int d = q >> 1, side = (q & 1) ? 1 : -1;
    // transverse coordinates (slow, fast) of a d-face: x (z, y), y (z, x), z (y, x)
    const int ts = d == 2 ? 1 : 2, tf = d == 0 ? 1 : 0;
    const int slot = side > 0 ? (loc[d] == 15 ? 1 : (loc[d] == 7 ? 2 : -1)) : (loc[d] == 0 ? 0 : (loc[d] == 8 ? 2 : -1));
    if (slot < 0) continue;  // cannot happen: fine groups cover whole coarse patches
    const int4 o = flayout[F];
    const int fo[3] = {o.y, o.z, o.w};
    const int fs0 = 2 * (c[ts] - (fo[ts] >> 1)), ff0 = 2 * (c[tf] - (fo[tf] >> 1));
    if (fs0 < 0 || fs0 > 14 || ff0 < 0 || ff0 > 14) continue;  // layout disagrees with the map
    const int fslot = side > 0 ? 0 : 1;  // F's face towards this cell
    const double sg = side > 0 ? -1.0 : 1.0;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double Fc = (double)cflux[((((G * 3 + d) * 3 + slot) * 5 + v) * 16 + loc[ts]) * 16 + loc[tf]];
      const T* f = fflux + ((((long long)F * 3 + d) * 2 + fslot) * 5 + v) * 256;
      double Ff = 0.0;
      Ff += (double)f[fs0 * 16 + ff0];
      Ff += (double)f[fs0 * 16 + ff0 + 1];
      Ff += (double)f[(fs0 + 1) * 16 + ff0];
      Ff += (double)f[(fs0 + 1) * 16 + ff0 + 1];
      Ff *= 0.25;
      u[v] += sg * dtdh * (Ff - Fc);
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) U[(G * 5 + v) * 4096 + l] = (T)u[v];
}

// Restriction: one workgroup per fine group, one thread per covered coarse
// cell (8^3); only the group that the map names at its position writes.
template <typename T>
__global__ void __launch_bounds__(512) restrict_kernel(T* __restrict__ U, int n, const T* __restrict__ fine,
                                                       const int4* __restrict__ flayout, const int* __restrict__ fmap,
                                                       int nf) {
#pragma clang fp contract(off)
  const int F = blockIdx.x;
  const int4 o = flayout[F];
  const int nfine = 2 * n;
  if (o.y < 0 || o.z < 0 || o.w < 0 || o.y >= nfine || o.z >= nfine || o.w >= nfine || ((o.y | o.z | o.w) & 15))
    return;
  const int cx0 = o.y >> 1, cy0 = o.z >> 1, cz0 = o.w >> 1;
  if (fine_owner(fmap, nf, n >> 3, cx0, cy0, cz0) != F) return;
  const int i = threadIdx.x & 7, j = (threadIdx.x >> 3) & 7, k = threadIdx.x >> 6;
  const int cx = cx0 + i, cy = cy0 + j, cz = cz0 + k;
  const int ng = n >> 4;
  const long long G = ((long long)(cz >> 4) * ng + (cy >> 4)) * ng + (cx >> 4);
  const int l = ((cz & 15) * 16 + (cy & 15)) * 16 + (cx & 15);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T* f = fine + ((long long)F * 5 + v) * 4096;
    double s = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) s += (double)f[((2 * k + dz) * 16 + 2 * j + dy) * 16 + 2 * i + dx];
    U[(G * 5 + v) * 4096 + l] = (T)(0.125 * s);
  }
}

template <typename T>
hipError_t launch_amr_correct(T* U, int n, const T* cflux, const T* fine, const int* flayout, int nf,
                              const int* fmap, const T* fflux, double dtdh, hipStream_t st) {
  if (nf == 0) return hipSuccess;
  reflux_kernel<T><<<dim3((unsigned)(6 * (long long)nf)), dim3(64), 0, st>>>(U, n, cflux, fmap, nf, fflux,
                                                                             (const int4*)flayout, dtdh);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  restrict_kernel<T><<<dim3((unsigned)nf), dim3(512), 0, st>>>(U, n, fine, (const int4*)flayout, fmap, nf);
  return hipGetLastError();
}
template hipError_t launch_amr_correct<float>(float*, int, const float*, const float*, const int*, int, const int*,
                                              const float*, double, hipStream_t);
template hipError_t launch_amr_correct<double>(double*, int, const double*, const double*, const int*, int,
                                               const int*, const double*, double, hipStream_t);

// acc += w * x, elementwise (the weighted sum of fine fluxes over sub-steps).
template <typename T>
__global__ void __launch_bounds__(256) axpy_kernel(T* __restrict__ acc, const T* __restrict__ x, double w, long long n) {
#pragma clang fp contract(off)
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    acc[t] = (T)((double)acc[t] + w * (double)x[t]);
}
template <typename T>
hipError_t launch_axpy(T* acc, const T* x, double w, long long n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  axpy_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(acc, x, w, n);
  return hipGetLastError();
}
template hipError_t launch_axpy<float>(float*, const float*, double, long long, hipStream_t);
template hipError_t launch_axpy<double>(double*, const double*, double, long long, hipStream_t);

template <typename T>
hipError_t launch_fill_interp(const T* coarse, int cn, const int* layout, long long n_groups, int g, double base_dh,
                              T* out, hipStream_t st) {
  const int N = 16 + 2 * g;
  const long long total = n_groups * N * N * N;
  if (total == 0) return hipSuccess;
  switch (g) {
    case 2: return launch_interp_groups<T, 2>(coarse, cn, layout, n_groups, base_dh, out, st);
    case 3: return launch_interp_groups<T, 3>(coarse, cn, layout, n_groups, base_dh, out, st);
    case 4: return launch_interp_groups<T, 4>(coarse, cn, layout, n_groups, base_dh, out, st);
    default: break;
  }
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  fill_interp_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(coarse, cn, (const int4*)layout, g, base_dh,
                                                                      out, total);
  return hipGetLastError();
}
template hipError_t launch_fill_interp<float>(const float*, int, const int*, long long, int, double, float*,
                                              hipStream_t);
template hipError_t launch_fill_interp<double>(const double*, int, const int*, long long, int, double, double*,
                                               hipStream_t);

// ---------------------------------------------------------------------------
// FP64 signal speed and time step.  The per-cell expression is evaluated in
// double without contraction, in a fixed order, so that the maximum (and
// hence dt) is bit-identical to a serial FP64 evaluation on the same data.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// U: n_blocks blocks of [5][4096]; one partial max per workgroup.  The
// per-cell expression is written out in a fixed order with contraction off.
template <typename T>
__global__ void __launch_bounds__(256) maxspeed_kernel(const T* __restrict__ U, long long n_blocks, double gamma,
                                                       double* __restrict__ partial) {
#pragma clang fp contract(off)
  __shared__ double red[4];
  double m = 0.0;
  const long long total = n_blocks << 12;
#pragma unroll 4
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const T* u = U + ((t >> 12) * 5 << 12) + (t & 4095);
    const double rho = (double)u[0];
    const double mx = (double)u[4096], my = (double)u[2 * 4096], mz = (double)u[3 * 4096];
    const double vx = mx / rho, vy = my / rho, vz = mz / rho;
    const double ke = 0.5 * (mx * vx + my * vy + mz * vz);
    const double p = (gamma - 1.0) * ((double)u[4 * 4096] - ke);
    const double cs = __builtin_sqrt(gamma * p / rho);
    double av = __builtin_fabs(vx);
    if (__builtin_fabs(vy) > av) av = __builtin_fabs(vy);
    if (__builtin_fabs(vz) > av) av = __builtin_fabs(vz);
    const double s = av + cs;
    m = s > m ? s : m;
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Batched time step: one workgroup per group of a segment table computes the
// group's maximum signal speed (same expression as above); one workgroup per
// segment then writes dt = cfl * dh / max to the segment's dt pointer.
template <typename T>
__global__ void __launch_bounds__(256) seg_maxspeed_kernel(const Seg* __restrict__ segs, int n_segs, double gamma,
                                                           double* __restrict__ partial) {
#pragma clang fp contract(off)
  __shared__ double red[4];
  const long long gidx = blockIdx.x;
  int lo = 0, hi = n_segs - 1;  // last segment with first <= gidx
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first <= gidx) lo = mid;
    else hi = mid - 1;
  }
  const Seg& S = segs[lo];
  const T* U = reinterpret_cast<const T*>(S.out) + (gidx - S.first) * 5 * 4096;
  double m = 0.0;
  for (int q = threadIdx.x; q < 4096; q += blockDim.x) {
    const T* u = U + q;
    const double rho = (double)u[0];
    const double mx = (double)u[4096], my = (double)u[2 * 4096], mz = (double)u[3 * 4096];
    const double vx = mx / rho, vy = my / rho, vz = mz / rho;
    const double ke = 0.5 * (mx * vx + my * vy + mz * vz);
    const double p = (gamma - 1.0) * ((double)u[4 * 4096] - ke);
    const double cs = __builtin_sqrt(gamma * p / rho);
    double av = __builtin_fabs(vx);
    if (__builtin_fabs(vy) > av) av = __builtin_fabs(vy);
    if (__builtin_fabs(vz) > av) av = __builtin_fabs(vz);
    const double sp = av + cs;
    m = sp > m ? sp : m;
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) partial[gidx] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ void __launch_bounds__(256) seg_dt_finish_kernel(const Seg* __restrict__ segs,
                                                            const double* __restrict__ partial, double cfl) {
#pragma clang fp contract(off)
  __shared__ double red[4];
  const Seg& S = segs[blockIdx.x];
  double m = 0.0;
  for (long long q = threadIdx.x; q < S.count; q += blockDim.x) m = fmax(m, partial[S.first + q]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    *const_cast<double*>(S.dt) = cfl * S.dh / mx;
  }
}

hipError_t launch_seg_dt(const Seg* segs, int n_segs, long long n_groups, double gamma, double cfl, int f64,
                         double* partial, hipStream_t st) {
  if (n_groups > 2147483647LL) return hipErrorInvalidValue;
  if (f64) seg_maxspeed_kernel<double><<<dim3((unsigned)n_groups), dim3(256), 0, st>>>(segs, n_segs, gamma, partial);
  else seg_maxspeed_kernel<float><<<dim3((unsigned)n_groups), dim3(256), 0, st>>>(segs, n_segs, gamma, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  seg_dt_finish_kernel<<<dim3(n_segs), dim3(256), 0, st>>>(segs, partial, cfl);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) dt_finish_kernel(const double* __restrict__ partial, int n, double dh,
                                                        double cfl, double* __restrict__ dt_out) {
#pragma clang fp contract(off)
  __shared__ double red[4];
  double m = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, partial[t]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    dt_out[0] = cfl * dh / mx;
  }
}

template <typename T>
hipError_t launch_maxspeed(const T* U, long long n_blocks, long long cells, double gamma, double* partial,
                           int n_partial, hipStream_t st) {
  if (cells != 4096) return hipErrorInvalidValue;
  maxspeed_kernel<T><<<dim3(n_partial), dim3(256), 0, st>>>(U, n_blocks, gamma, partial);
  return hipGetLastError();
}
template hipError_t launch_maxspeed<float>(const float*, long long, long long, double, double*, int, hipStream_t);
template hipError_t launch_maxspeed<double>(const double*, long long, long long, double, double*, int, hipStream_t);

hipError_t launch_dt_finish(const double* partial, int n_partial, double dh, double cfl, double* dt_out,
                            hipStream_t st) {
  dt_finish_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, n_partial, dh, cfl, dt_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 conserved sums.  Workgroup w sums a fixed contiguous slice of cells
// (lane-strided, then a fixed shuffle tree); a single workgroup then adds the
// partials in index order.  The order depends only on n_partial, never on
// timing, so repeated calls are bitwise identical.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) sums_kernel(const T* __restrict__ U, long long n_blocks,
                                                   double* __restrict__ partial) {
  __shared__ double red[5][4];
  const long long total = n_blocks << 12;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * per, hi = min(total, lo + per);
  double s[5] = {0, 0, 0, 0, 0};
  for (long long t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T* u = U + ((t >> 12) * 5 << 12) + (t & 4095);
#pragma unroll
    for (int n = 0; n < 5; ++n) s[n] += (double)u[n * 4096];
  }
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    double v = wave_sum(s[n]);
    if ((threadIdx.x & 63) == 0) red[n][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int n = threadIdx.x;
    partial[(long long)blockIdx.x * 5 + n] = (red[n][0] + red[n][1]) + (red[n][2] + red[n][3]);
  }
}

// Fixed-order finish: thread q adds partials q, q+256, ... in index order,
// then a fixed shuffle tree and a fixed cross-wave sum.
__global__ void __launch_bounds__(256) sums_finish_kernel(const double* __restrict__ partial, int n, double vol,
                                                         double* __restrict__ out) {
  __shared__ double red[5][4];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) s += partial[(long long)b * 5 + v];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[v][threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int v = threadIdx.x;
    out[v] = ((red[v][0] + red[v][1]) + (red[v][2] + red[v][3])) * vol;
  }
}

template <typename T>
hipError_t launch_sums(const T* U, long long n_blocks, long long cells, double dh, double* partial, int n_partial,
                       double* sums_out, hipStream_t st) {
  if (cells != 4096) return hipErrorInvalidValue;
  sums_kernel<T><<<dim3(n_partial), dim3(256), 0, st>>>(U, n_blocks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sums_finish_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, n_partial, dh * dh * dh, sums_out);
  return hipGetLastError();
}
template hipError_t launch_sums<float>(const float*, long long, long long, double, double*, int, double*, hipStream_t);
template hipError_t launch_sums<double>(const double*, long long, long long, double, double*, int, double*,
                                        hipStream_t);

// ---------------------------------------------------------------------------
// Time step and conserved sums in one pass over the state.  Workgroup w takes
// the same contiguous slice, lane order and shuffle trees as sums_kernel, and
// evaluates the signal speed with the same expression as maxspeed_kernel on
// the same cells; the finish repeats dt_finish_kernel and sums_finish_kernel.
// Both results are therefore bit-identical to the two separate reductions,
// while the state is read once.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) dtsums_kernel(const T* __restrict__ U, long long n_blocks, double gamma,
                                                     double* __restrict__ partial) {
#pragma clang fp contract(off)
  __shared__ double red[6][4];
  const long long total = n_blocks << 12;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long lo = blockIdx.x * per, hi = min(total, lo + per);
  double s[5] = {0, 0, 0, 0, 0};
  double m = 0.0;
  // Unrolled so that the FP64 division chains of several cells overlap; the
  // sums still take the cells of a lane in order.
#pragma unroll 4
  for (long long t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const T* u = U + ((t >> 12) * 5 << 12) + (t & 4095);
    double c[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) c[n] = (double)u[n * 4096];
#pragma unroll
    for (int n = 0; n < 5; ++n) s[n] += c[n];
    const double rho = c[0];
    const double mx = c[1], my = c[2], mz = c[3];
    const double vx = mx / rho, vy = my / rho, vz = mz / rho;
    const double ke = 0.5 * (mx * vx + my * vy + mz * vz);
    const double p = (gamma - 1.0) * (c[4] - ke);
    const double cs = __builtin_sqrt(gamma * p / rho);
    double av = __builtin_fabs(vx);
    if (__builtin_fabs(vy) > av) av = __builtin_fabs(vy);
    if (__builtin_fabs(vz) > av) av = __builtin_fabs(vz);
    const double sp = av + cs;
    m = sp > m ? sp : m;
  }
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    double v = wave_sum(s[n]);
    if ((threadIdx.x & 63) == 0) red[n][threadIdx.x >> 6] = v;
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[5][threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x < 5) {
    const int n = threadIdx.x;
    partial[(long long)blockIdx.x * 5 + n] = (red[n][0] + red[n][1]) + (red[n][2] + red[n][3]);
  } else if (threadIdx.x == 5) {
    partial[(long long)gridDim.x * 5 + blockIdx.x] = fmax(fmax(red[5][0], red[5][1]), fmax(red[5][2], red[5][3]));
  }
}

__global__ void __launch_bounds__(256) dtsums_finish_kernel(const double* __restrict__ partial, int n, double dh,
                                                           double cfl, double* __restrict__ dt_out,
                                                           double* __restrict__ sums_out) {
#pragma clang fp contract(off)
  __shared__ double red[6][4];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) s += partial[(long long)b * 5 + v];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[v][threadIdx.x >> 6] = s;
  }
  double m = 0.0;
  for (int t = threadIdx.x; t < n; t += blockDim.x) m = fmax(m, partial[(long long)n * 5 + t]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[5][threadIdx.x >> 6] = m;
  __syncthreads();
  const double vol = dh * dh * dh;
  if (threadIdx.x < 5) {
    const int v = threadIdx.x;
    sums_out[v] = ((red[v][0] + red[v][1]) + (red[v][2] + red[v][3])) * vol;
  } else if (threadIdx.x == 5) {
    const double mx = fmax(fmax(red[5][0], red[5][1]), fmax(red[5][2], red[5][3]));
    dt_out[0] = cfl * dh / mx;
  }
}

template <typename T>
hipError_t launch_dtsums(const T* U, long long n_blocks, double dh, double gamma, double cfl, double* partial,
                         int n_partial, double* dt_out, double* sums_out, hipStream_t st) {
  dtsums_kernel<T><<<dim3(n_partial), dim3(256), 0, st>>>(U, n_blocks, gamma, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dtsums_finish_kernel<<<dim3(1), dim3(256), 0, st>>>(partial, n_partial, dh, cfl, dt_out, sums_out);
  return hipGetLastError();
}
template hipError_t launch_dtsums<float>(const float*, long long, double, double, double, double*, int, double*,
                                         double*, hipStream_t);
template hipError_t launch_dtsums<double>(const double*, long long, double, double, double, double*, int, double*,
                                          double*, hipStream_t);

}  // namespace hy
