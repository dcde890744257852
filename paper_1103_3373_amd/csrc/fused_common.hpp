// Pieces shared by the fused z-marching kernels (CTU, MHM, VL): LDS
// helpers, the thread -> column map of a 512-thread workgroup over the 16x16
// interior plus rings, segment lookup, and loads of a group's cells either
// from a ghosted group array or, in box mode, from the periodic grouped box.
#pragma once

#include "hydro_internal.h"
#include "hydro_math.hpp"

namespace hy {
namespace fz {

constexpr int kThreads = 512;

template <typename T> HY_DEV V5<T> lds5(const T* s, int stride, int i) {
  V5<T> v;
#pragma unroll
  for (int n = 0; n < 5; ++n) v[n] = s[n * stride + i];
  return v;
}
template <typename T> HY_DEV void sts5(T* s, int stride, int i, const V5<T>& v) {
#pragma unroll
  for (int n = 0; n < 5; ++n) s[n * stride + i] = v[n];
}
template <typename T> HY_DEV V5<T> sub5(const V5<T>& a, const V5<T>& b) {
  V5<T> r;
#pragma unroll
  for (int n = 0; n < 5; ++n) r[n] = a[n] - b[n];
  return r;
}

// Face values of one cell from its neighbourhood along a direction (frame
// states), PLM or PPM, before tracing.  wm/wp are the neighbours, sm/s0/sp
// the limited slopes of the neighbours and the cell (PLM uses s0 only).
template <bool PPM, typename T>
HY_DEV void face_values(const V5<T>& wm, const V5<T>& w0, const V5<T>& wp, const V5<T>& sm, const V5<T>& s0,
                        const V5<T>& sp, const Phys<T>& ph, V5<T>& fl, V5<T>& fr) {
  if (PPM) {
    fl = ppm_edge(wm, w0, sm, s0);
    fr = ppm_edge(w0, wp, s0, sp);
    ppm_mono(w0, fl, fr);
  } else {
    plm_faces(wm, w0, wp, s0, ph, fl, fr);
  }
}

// Corrected state: U(W) - hdtdh * d, back to primitive with floors; the
// floor hits are counted for the whole wavefront (floor_wave).
template <typename T>
HY_DEV V5<T> correct(const V5<T>& W, const V5<T>& d, const Phys<T>& ph, unsigned& wave_floors) {
  V5<T> u = cons_of(W, ph);
#pragma unroll
  for (int n = 0; n < 5; ++n) u[n] -= ph.hdtdh * d[n];
  V5<T> w = prim_of(u, ph);
  wave_floors += floor_wave(w, ph);
  return w;
}

template <typename T> struct Column {
  int x, y;      // interior-relative coordinates
  int cross;     // 1 if the column needs z work (interior + 1-cell ring)
  int active;    // 1 if the column feeds the primitive plane
};

template <int G> HY_DEV Column<int> column_of(int tid) {
  Column<int> c{0, 0, 0, 0};
  if (tid < 256) {
    c.x = tid & 15; c.y = tid >> 4; c.cross = 1; c.active = 1;
  } else if (tid < 320) {
    int q = tid - 256, s = q & 15;
    switch (q >> 4) {
      case 0: c.x = -1; c.y = s; break;
      case 1: c.x = 16; c.y = s; break;
      case 2: c.x = s; c.y = -1; break;
      default: c.x = s; c.y = 16; break;
    }
    c.cross = 1; c.active = 1;
  } else if (tid < 324) {
    int q = tid - 320;
    c.x = (q & 1) ? 16 : -1; c.y = (q & 2) ? 16 : -1; c.active = 1;
  } else {
    // Outer columns: G-1 per side beyond the ring, 18 long, along both axes.
    const int w = G - 1;               // 2 for PPM, 1 for PLM
    const int per = 2 * w * 18;        // one orientation
    int q = tid - 324;
    if (q < 2 * per) {
      int o = q / per, r = q % per;
      int side = r / (w * 18), rr = r % (w * 18);
      int depth = rr / 18, along = rr % 18 - 1;   // along in -1..16
      int off = side ? (17 + depth) : (-2 - depth);
      if (o == 0) { c.x = off; c.y = along; }
      else { c.x = along; c.y = off; }
      c.active = 1;
    }
  }
  return c;
}


// Order in which a workgroup of the persistent grid visits the groups.
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b % 8), each XCD with its own L2.  XCD x takes the x-th contiguous
// eighth of the groups, so the workgroups resident on one XCD at a time work
// on neighbouring groups (x, then y, then z neighbours are close in group
// order) and the ghost cells they read from each other hit in that L2.  Any
// grid that is not a multiple of 8 uses the plain strided order.
struct GroupOrder {
  long long first, stride, end;  // visits first, first + stride, ... < end
};
HY_DEV GroupOrder group_order(long long n_groups) {
  const long long P = gridDim.x, b = blockIdx.x;
  if (P < 8 || P % 8 != 0) return GroupOrder{b, P, n_groups};
  const long long chunk = (n_groups + 7) / 8;
  const long long lo = (b % 8) * chunk;
  const long long hi = lo + chunk < n_groups ? lo + chunk : n_groups;
  return GroupOrder{lo + b / 8, P / 8, hi};
}

// Per-launch physics constants (dt/dh set per group from its segment).
template <typename T> HY_DEV Phys<T> make_phys(const FusedArgs<T>& a) {
  Phys<T> ph;
  ph.gamma = a.gamma;
  ph.gm1 = a.gamma - T(1);
  ph.inv_gm1 = T(1) / ph.gm1;
  ph.theta = a.theta;
  ph.floor = a.floor;
  ph.limiter = a.limiter;
  ph.charlim = a.charlim;
  ph.roe_fb_hllc = a.roe_fb_hllc;
  ph.dtdh = T(0);
  ph.hdtdh = T(0);
  return ph;
}

// Pointers qualified with the global address space.  A load through a
// generic pointer is a FLAT access: it counts against the LDS wait counter
// too, and the compiler must treat its result as possibly per-lane.
template <typename T> using gptr = __attribute__((address_space(1))) T*;

// Workgroup-uniform values: readfirstlane puts them in scalar registers, so
// the arithmetic on them is scalar and branches on them do not diverge.
HY_DEV int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
HY_DEV long long uni(long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
HY_DEV double uni(double v) { return __longlong_as_double(uni(__double_as_longlong(v))); }
template <typename P> HY_DEV P* uni(P* p) { return reinterpret_cast<P*>(uni((long long)(uintptr_t)p)); }

// Global store / load at a uniform base plus a per-lane byte offset (the
// base + 32-bit offset addressing form of the memory instructions).
template <typename T> HY_DEV void gstore(T* base, unsigned byte_off, T v) {
  *(gptr<T>)((gptr<char>)(gptr<T>)base + byte_off) = v;
}
template <typename T> HY_DEV T gload(const T* base, unsigned byte_off) {
  return *(gptr<const T>)((gptr<const char>)(gptr<const T>)base + byte_off);
}

// The segment a work item belongs to, as workgroup-uniform values.
struct USeg {
  const void* in;
  void* out;
  void* flux;
  double dh;
  long long first;
  int ngx, ngy, ngz;
  int box;
};

// Segment of global group grp (segments sorted by first group; `seg` is a
// cursor that only moves forward in a persistent loop) and its time step.
template <typename T>
HY_DEV USeg find_seg(const FusedArgs<T>& a, long long grp, int& seg, double& dt) {
  USeg u;
  if (a.segs) {
    const gptr<const Seg> segs = (gptr<const Seg>)a.segs;
    while (seg + 1 < a.n_segs && segs[seg + 1].first <= grp) ++seg;
    while (seg > 0 && segs[seg].first > grp) --seg;
    seg = uni(seg);
    const gptr<const Seg> S = segs + seg;
    u = USeg{S->in, S->out, S->flux, S->dh, S->first, S->ngx, S->ngy, S->ngz, S->box};
    dt = *(gptr<const double>)S->dt * S->dt_scale;
  } else {
    const Seg& S = a.seg0;
    u = USeg{S.in, S.out, S.flux, S.dh, S.first, S.ngx, S.ngy, S.ngz, S.box};
    dt = S.dt ? *(gptr<const double>)S.dt * S.dt_scale : a.dt0;
  }
  u.in = uni(u.in);
  u.out = uni(u.out);
  u.flux = uni(u.flux);
  u.dh = uni(u.dh);
  u.first = uni(u.first);
  u.ngx = uni(u.ngx);
  u.ngy = uni(u.ngy);
  u.ngz = uni(u.ngz);
  u.box = uni(u.box);
  dt = uni(dt);
  return u;
}

// Box segments address a cell by a 32-bit byte offset within a z-slab of
// groups (ngx * ngy groups), so a slab must hold less than 4 GiB; a segment
// beyond that gets NaN outputs.
template <typename T> HY_DEV bool slab_fits(const USeg& S) {
  return !S.box || (unsigned long long)S.ngx * (unsigned long long)S.ngy * (5ull * 4096ull * sizeof(T)) < (1ull << 32);
}

// Reader of the conserved cells of one column (x, y fixed, interior-relative)
// of one group: a ghosted group array of width G (N = 16 + 2G), or, in box
// mode, the periodic box stored as groups.  The address of a cell is a
// uniform base (the group or box, the z plane and the variable) plus the
// column's byte offset, formed once per group; box mode keeps that offset
// below 4 GiB (the host rejects boxes whose z-slab of groups is larger).
template <typename T, int G> struct ColumnReader {
  static constexpr int N = 16 + 2 * G;
  static constexpr long NC = (long)N * N * N;
  const char* base;  // uniform: box mode the box, else the group's array
  unsigned off;      // this column's byte offset from `base` (box: in z-group 0)
  int box;           // uniform
  int bz0, bnz;      // box mode, uniform: first z of the group, box size in z
  long zgs;          // box mode, uniform: elements between z-neighbouring groups
  HY_DEV void init(const USeg& S, long long lg, int x, int y) {
    box = S.box;
    if (box) {
      const int ngx = S.ngx, ngy = S.ngy, l = (int)lg;
      const int bnx = ngx * 16, bny = ngy * 16;
      bnz = S.ngz * 16;
      const int bx0 = (l % ngx) * 16, by0 = ((l / ngx) % ngy) * 16;
      bz0 = (l / (ngx * ngy)) * 16;
      int cx = bx0 + x, cy = by0 + y;
      cx += cx < 0 ? bnx : 0; cx -= cx >= bnx ? bnx : 0;
      cy += cy < 0 ? bny : 0; cy -= cy >= bny ? bny : 0;
      zgs = (long)ngx * ngy * 5 * 4096;
      base = reinterpret_cast<const char*>(S.in);
      off = (unsigned)(((cy >> 4) * ngx + (cx >> 4)) * 5 * 4096 + ((cy & 15) * 16 + (cx & 15))) * (unsigned)sizeof(T);
    } else {
      base = reinterpret_cast<const char*>(reinterpret_cast<const T*>(S.in) + lg * 5 * NC);
      off = (unsigned)(((y + G) * N + (x + G) + G * N * N) * (int)sizeof(T));
      bz0 = bnz = 0;
      zgs = 0;
    }
  }
  HY_DEV V5<T> load(int z) const {
    V5<T> u;
    long zo;
    if (box) {
      int cz = bz0 + z;
      cz += cz < 0 ? bnz : 0;
      cz -= cz >= bnz ? bnz : 0;
      zo = (cz >> 4) * zgs + (cz & 15) * 256;
    } else {
      zo = (long)z * N * N;
    }
    const long vs = box ? 4096 : NC;
#pragma unroll
    for (int n = 0; n < 5; ++n) u[n] = gload(reinterpret_cast<const T*>(base) + zo + n * vs, off);
    return u;
  }
};

template <typename T> HY_DEV void flush_diag(const FusedArgs<T>& a, int fails, int floors) {
  if (a.diag) {
    if (fails) atomicAdd(&a.diag[0], (unsigned long long)fails);
    if (floors) atomicAdd(&a.diag[1], (unsigned long long)floors);
  }
}

}  // namespace fz
}  // namespace hy
