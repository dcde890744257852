// Fused CTU solver for patch groups (arXiv:1103.3373, Sec. 2 steps (1)-(5)),
// designed for gfx950 rather than after the paper's Fermi kernel.
//
// One 512-thread workgroup owns one patch group at a time (persistent loop
// over groups) and marches through it plane by plane along z:
//
//  * Every thread owns an (x, y) column.  Threads 0-255 are the 16x16
//    interior columns, 256-319 the one-cell ring around it (the "cross" on
//    which transverse corrections are needed), 320-323 the ring corners and
//    324.. the outer columns that only feed x/y reconstruction.  Cross
//    threads keep a sliding window of primitive states, limited slopes and
//    PPM edges along z in registers, so the z reconstruction, the
//    characteristic tracing, the first z Riemann solve and later the second
//    one and the conservative update are done without any shared memory and
//    every slope is computed once.
//  * x and y work of the current plane goes through LDS: primitive plane,
//    limited slopes, traced face states, first-set fluxes and the
//    transverse z-flux differences (about 69 KB for FP32, so two
//    workgroups share a CU).
//  * Per plane: A columns (prims, z trace, H1, dH1) | B x/y slopes |
//    C x/y traces | D x/y Riemann set 1 | E corrected x/y Riemann set 2 and
//    z correction + z Riemann set 2 | F conservative update and flux store.
//    Five barriers per plane; the update of plane t-1 completes in plane t
//    once its upper z flux exists.
//  * The correction of a face state is done by the task that solves that
//    face, so each corrected state is formed exactly once.
// Global memory sees only the input (read once per cell), the output and
// the optional face fluxes.
#pragma once

#include "fused_common.hpp"

namespace hy {
namespace ctu {

using namespace fz;

// LDS layout (elements of T).  Sizes are those of PPM (g = 3); PLM uses a
// subset of the same layout.
constexpr int kNmax = 22;
constexpr int kP = kNmax * kNmax;   // primitive plane, full padded square
constexpr int kSX = 20 * 18;        // x slopes: x in -2..17, y in -1..16
constexpr int kSY = 18 * 20;        // y slopes: x in -1..16, y in -2..17
constexpr int kSQ = 18 * 18;        // x,y in -1..16
constexpr int kF1 = 17 * 18;        // x faces -1..15 (i+1/2), y in -1..16
constexpr int kG1 = 18 * 17;        // x in -1..16, y faces -1..15
constexpr int oP = 0;
constexpr int oSX = oP + 5 * kP;
constexpr int oSY = oSX + 5 * kSX;
constexpr int oWX = oSY + 5 * kSY;    // [2][5][kSQ]: 0 = left face, 1 = right face
constexpr int oWY = oWX + 10 * kSQ;
constexpr int oF1 = oWY + 10 * kSQ;
constexpr int oG1 = oF1 + 5 * kF1;
constexpr int oDH = oG1 + 5 * kG1;
constexpr int kLds = oDH + 5 * kSQ;
// After the T-typed area: addresses of the ring-corner and outer columns of
// the current group (column ids 320 .. 467), formed once per group.
constexpr int kOuterCols = 148;
constexpr size_t kLdsBytes(size_t elem) { return kLds * elem + kOuterCols * sizeof(void*); }
// Final in-plane fluxes reuse the slope area (dead after the traces).
constexpr int kF2 = 17 * 16;          // x faces -1..15, y in 0..15
constexpr int kG2 = 16 * 17;          // x in 0..15, y faces -1..15
constexpr int oF2 = oSX;
constexpr int oG2 = oSX + 5 * kF2;
static_assert(10 * kF2 <= 5 * (kSX + kSY), "F2/G2 alias");

// WAVES = minimum waves per SIMD the register allocation must allow: 2 gives
// one workgroup per CU without spills, 4 gives two workgroups per CU (with
// some spilling); the autotuner picks per specialization.
template <typename T, bool PPM, int RS, int WAVES>
__global__ void __launch_bounds__(kThreads, WAVES) ctu_fused_kernel(FusedArgs<T> a) {
  constexpr int NT = kThreads;
  constexpr int G = PPM ? 3 : 2;
  constexpr int N = 16 + 2 * G;
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  T* sP = sm + oP;
  T* sSX = sm + oSX;
  T* sSY = sm + oSY;
  T* sWX = sm + oWX;
  T* sWY = sm + oWY;
  T* sF1 = sm + oF1;
  T* sG1 = sm + oG1;
  T* sDH = sm + oDH;
  T* sF2 = sm + oF2;
  T* sG2 = sm + oG2;
  const T** sOC = reinterpret_cast<const T**>(smem_raw + kLds * sizeof(T));

  const int tid = threadIdx.x;
  const Column<int> col = column_of<G>(tid);
  const int pcol = (col.y + G) * N + (col.x + G);  // primitive plane index
  const int sqc = (col.y + 1) * 18 + (col.x + 1);  // 18x18 square index (cross columns)
  const bool interior = tid < 256;
  constexpr int nCols = 324 + 4 * (G - 1) * 18;  // columns that feed the primitive plane
  static_assert(nCols - 320 <= kOuterCols, "outer column table");
  int fails = 0, floors = 0;

  Phys<T> ph = make_phys(a);

  // Slope task counts (PLM needs slopes of the traced cells only).
  constexpr int wSX = PPM ? 20 : 18, x0SX = PPM ? -2 : -1;
  constexpr int nSX = wSX * 18;
  constexpr int hSY = PPM ? 20 : 18, y0SY = PPM ? -2 : -1;
  constexpr int nSY = 18 * hSY;

  int seg = 0;
  for (long long grp = blockIdx.x; grp < a.n_groups; grp += gridDim.x) {
    double dt;
    const Seg* S = find_seg(a, grp, seg, dt);
    const long long lg = grp - S->first;
    T* __restrict__ O = reinterpret_cast<T*>(S->out) + lg * 5 * 4096;
    T* __restrict__ FO = S->flux ? reinterpret_cast<T*>(S->flux) + lg * 3 * a.nf * 5 * 256 : nullptr;
    ph.dtdh = (T)(dt / S->dh);
    ph.hdtdh = (T)(0.5 * dt / S->dh);
    // The group's cells (ghosts included) come from the ghosted input or, in
    // box mode, straight from the periodic grouped box.
    ColumnReader<T, G> rd;
    rd.init(S, lg, col.x, col.y);
    if (!col.cross) {
      // Each thread reads back only the slots it writes: no barrier needed.
      for (int c = tid; c < nCols; c += NT - 320) {
        const Column<int> oc = column_of<G>(c);
        ColumnReader<T, G> orr;
        orr.init(S, lg, oc.x, oc.y);
        sOC[c - 320] = orr.col;
      }
    }
    auto load_cons = [&](int x, int y, int z) -> V5<T> { return rd.load(z); };
    auto zprim = [&](int z) -> V5<T> { return to_frame<2>(prim_of(load_cons(col.x, col.y, z), ph)); };

    // Register state of a cross column (frame z unless noted):
    V5<T> w0, w1, w2;   // W(t), W(t+1), W(t+2)   (PLM: w0, w1)
    V5<T> s1, e0;       // S(t+1), E(t+1/2)       (PPM)
    V5<T> ztm, ztp;     // traced states of plane t
    V5<T> h1m;          // H1(t-1/2)
    V5<T> zcp;          // corrected right state of plane t-1
    V5<T> hprev;        // final H below the plane being updated (lab)
    V5<T> accp;         // in-plane flux differences of the plane being updated (lab)

    // ---- prologue: window and traced states of plane -1 -------------------
    if (col.cross) {
      if (PPM) {
        V5<T> wa = zprim(-3), wb = zprim(-2);
        w0 = zprim(-1);
        w1 = zprim(0);
        w2 = zprim(1);
        V5<T> sa = slope(wa, wb, w0, ph), sb = slope(wb, w0, w1, ph);
        s1 = slope(w0, w1, w2, ph);
        ztm = ppm_edge(wb, w0, sa, sb);
        e0 = ppm_edge(w0, w1, sb, s1);
        ztp = e0;
        ppm_mono(w0, ztm, ztp);
        ctu_trace<true>(w0, ztm, ztp, ph);
      } else {
        V5<T> wb = zprim(-2);
        w0 = zprim(-1);
        w1 = zprim(0);
        V5<T> sb = slope(wb, w0, w1, ph);
        plm_faces(wb, w0, w1, sb, ph, ztm, ztp);
        ctu_trace<false>(w0, ztm, ztp, ph);
      }
      floors += floor_state(ztm, ph) + floor_state(ztp, ph);
    }

    for (int t = -1; t <= 16; ++t) {
      // ---- A: columns: primitive plane t; trace plane t+1; H1(t+1/2) -------
      V5<T> nzm, nzp;  // traced states of plane t+1
      if (col.cross) {
        sts5(sP, kP, pcol, from_frame<2>(w0));
        if (t <= 15) {
          if (PPM) {
            V5<T> w3 = zprim(t + 3);
            V5<T> s2 = slope(w1, w2, w3, ph);
            V5<T> e1 = ppm_edge(w1, w2, s1, s2);
            nzm = e0;
            nzp = e1;
            ppm_mono(w1, nzm, nzp);
            ctu_trace<true>(w1, nzm, nzp, ph);
            w0 = w1; w1 = w2; w2 = w3; s1 = s2; e0 = e1;
          } else {
            V5<T> w3 = zprim(t + 2);
            V5<T> sb = slope(w0, w1, w3, ph);
            plm_faces(w0, w1, w3, sb, ph, nzm, nzp);
            ctu_trace<false>(w1, nzm, nzp, ph);
            w0 = w1; w1 = w3;
          }
          floors += floor_state(nzm, ph) + floor_state(nzp, ph);
          V5<T> h1p = riemann<RS>(ztp, nzm, ph, &fails);  // H1(t+1/2)
          if (t >= 0) sts5(sDH, kSQ, sqc, from_frame<2>(sub5(h1p, h1m)));
          h1m = h1p;
        }
      } else {
        // Ring corners and outer columns (column ids 320 .. nCols-1), strided
        // over the threads that own no cross column.
        for (int c = tid; c < nCols; c += NT - 320) {
          const Column<int> oc = column_of<G>(c);
          ColumnReader<T, G> orr = rd;  // z part of the group
          orr.col = sOC[c - 320];
          sts5(sP, kP, (oc.y + G) * N + (oc.x + G), prim_of(orr.load(t), ph));
        }
      }
      __syncthreads();

      // ---- B: limited slopes along x and y of plane t ----------------------
      for (int q = tid; q < nSX + nSY; q += NT) {
        if (q < nSX) {
          const int x = q % wSX + x0SX, y = q / wSX - 1;
          const int c = (y + G) * N + (x + G);
          V5<T> s = slope(to_frame<0>(lds5(sP, kP, c - 1)), to_frame<0>(lds5(sP, kP, c)),
                          to_frame<0>(lds5(sP, kP, c + 1)), ph);
          sts5(sSX, kSX, (y + 1) * 20 + (x + 2), s);
        } else {
          const int r = q - nSX;
          const int x = r % 18 - 1, y = r / 18 + y0SY;
          const int c = (y + G) * N + (x + G);
          V5<T> s = slope(to_frame<1>(lds5(sP, kP, c - N)), to_frame<1>(lds5(sP, kP, c)),
                          to_frame<1>(lds5(sP, kP, c + N)), ph);
          sts5(sSY, kSY, (y + 2) * 18 + (x + 1), s);
        }
      }
      __syncthreads();

      // ---- C: traced x and y face states of plane t (frame order) ----------
      for (int q = tid; q < 2 * kSQ; q += NT) {
        const int r = q < kSQ ? q : q - kSQ;
        const int x = r % 18 - 1, y = r / 18 - 1;
        const int c = (y + G) * N + (x + G);
        V5<T> fl, fr;
        if (q < kSQ) {
          V5<T> wm = to_frame<0>(lds5(sP, kP, c - 1)), w = to_frame<0>(lds5(sP, kP, c)),
                wp = to_frame<0>(lds5(sP, kP, c + 1));
          const int si = (y + 1) * 20 + (x + 2);
          V5<T> s0 = lds5(sSX, kSX, si);
          V5<T> smn = PPM ? lds5(sSX, kSX, si - 1) : s0, spl = PPM ? lds5(sSX, kSX, si + 1) : s0;
          face_values<PPM>(wm, w, wp, smn, s0, spl, ph, fl, fr);
          ctu_trace<PPM>(w, fl, fr, ph);
          floors += floor_state(fl, ph) + floor_state(fr, ph);
          sts5(sWX, kSQ, r, fl);
          sts5(sWX + 5 * kSQ, kSQ, r, fr);
        } else {
          V5<T> wm = to_frame<1>(lds5(sP, kP, c - N)), w = to_frame<1>(lds5(sP, kP, c)),
                wp = to_frame<1>(lds5(sP, kP, c + N));
          const int si = (y + 2) * 18 + (x + 1);
          V5<T> s0 = lds5(sSY, kSY, si);
          V5<T> smn = PPM ? lds5(sSY, kSY, si - 18) : s0, spl = PPM ? lds5(sSY, kSY, si + 18) : s0;
          face_values<PPM>(wm, w, wp, smn, s0, spl, ph, fl, fr);
          ctu_trace<PPM>(w, fl, fr, ph);
          floors += floor_state(fl, ph) + floor_state(fr, ph);
          sts5(sWY, kSQ, r, fl);
          sts5(sWY + 5 * kSQ, kSQ, r, fr);
        }
      }
      __syncthreads();

      // ---- D: first-set Riemann solves in x and y (lab-order fluxes) -------
      for (int q = tid; q < kF1 + kG1; q += NT) {
        if (q < kF1) {
          const int i = q % 17 - 1, y = q / 17 - 1;  // face between x = i and i+1
          const int l = (y + 1) * 18 + (i + 1);
          V5<T> F = riemann<RS>(lds5(sWX + 5 * kSQ, kSQ, l), lds5(sWX, kSQ, l + 1), ph, &fails);
          sts5(sF1, kF1, q, from_frame<0>(F));
        } else {
          const int r = q - kF1;
          const int x = r % 18 - 1, j = r / 18 - 1;  // face between y = j and j+1
          const int l = (j + 1) * 18 + (x + 1);
          V5<T> F = riemann<RS>(lds5(sWY + 5 * kSQ, kSQ, l), lds5(sWY, kSQ, l + 18), ph, &fails);
          sts5(sG1, kG1, r, from_frame<1>(F));
        }
      }
      __syncthreads();

      // ---- E: corrected x/y faces and their final fluxes (planes 0..15);
      //         z correction of plane t and H(t-1/2) (interior columns) ----
      V5<T> hn;
      if (interior) {
        const int x = col.x, y = col.y;
        V5<T> dF = sub5(lds5(sF1, kF1, (y + 1) * 17 + x + 1), lds5(sF1, kF1, (y + 1) * 17 + x));
        V5<T> dG = sub5(lds5(sG1, kG1, (y + 1) * 18 + x + 1), lds5(sG1, kG1, y * 18 + x + 1));
        V5<T> d;
#pragma unroll
        for (int n = 0; n < 5; ++n) d[n] = dF[n] + dG[n];
        d = to_frame<2>(d);
        V5<T> cm = correct(ztm, d, ph, floors), cp = correct(ztp, d, ph, floors);
        if (t >= 0) hn = from_frame<2>(riemann<RS>(zcp, cm, ph, &fails));  // H(t-1/2)
        zcp = cp;
      }
      if (t >= 0 && t <= 15) {
        for (int q = NT - 1 - tid; q < kF2 + kG2; q += NT) {
          if (q < kF2) {
            const int i = q % 17 - 1, y = q / 17;  // x face between i and i+1, row y
            const int l = (y + 1) * 18 + (i + 1);
            V5<T> dl, dr;
            V5<T> gl = sub5(lds5(sG1, kG1, (y + 1) * 18 + i + 1), lds5(sG1, kG1, y * 18 + i + 1));
            V5<T> gr = sub5(lds5(sG1, kG1, (y + 1) * 18 + i + 2), lds5(sG1, kG1, y * 18 + i + 2));
            V5<T> hl = lds5(sDH, kSQ, l), hr = lds5(sDH, kSQ, l + 1);
#pragma unroll
            for (int n = 0; n < 5; ++n) { dl[n] = gl[n] + hl[n]; dr[n] = gr[n] + hr[n]; }
            V5<T> L = correct(lds5(sWX + 5 * kSQ, kSQ, l), to_frame<0>(dl), ph, floors);
            V5<T> R = correct(lds5(sWX, kSQ, l + 1), to_frame<0>(dr), ph, floors);
            sts5(sF2, kF2, q, from_frame<0>(riemann<RS>(L, R, ph, &fails)));
          } else {
            const int r = q - kF2;
            const int x = r % 16, j = r / 16 - 1;  // y face between j and j+1, column x
            const int l = (j + 1) * 18 + (x + 1);
            V5<T> dl, dr;
            V5<T> fl_ = sub5(lds5(sF1, kF1, (j + 1) * 17 + x + 1), lds5(sF1, kF1, (j + 1) * 17 + x));
            V5<T> fr_ = sub5(lds5(sF1, kF1, (j + 2) * 17 + x + 1), lds5(sF1, kF1, (j + 2) * 17 + x));
            V5<T> hl = lds5(sDH, kSQ, l), hr = lds5(sDH, kSQ, l + 18);
#pragma unroll
            for (int n = 0; n < 5; ++n) { dl[n] = hl[n] + fl_[n]; dr[n] = hr[n] + fr_[n]; }
            V5<T> L = correct(lds5(sWY + 5 * kSQ, kSQ, l), to_frame<1>(dl), ph, floors);
            V5<T> R = correct(lds5(sWY, kSQ, l + 18), to_frame<1>(dr), ph, floors);
            sts5(sG2, kG2, r, from_frame<1>(riemann<RS>(L, R, ph, &fails)));
          }
        }
      }
      __syncthreads();

      // ---- F: finish plane t-1; in-plane flux differences of plane t;
      //         boundary fluxes (Sec. 2 step 5) ------------------------------
      if (interior) {
        const int x = col.x, y = col.y;
        if (t >= 1) {
          V5<T> u = load_cons(x, y, t - 1);
          const int o = ((t - 1) * 16 + y) * 16 + x;
#pragma unroll
          for (int n = 0; n < 5; ++n) O[n * 4096 + o] = u[n] - ph.dtdh * (accp[n] + (hn[n] - hprev[n]));
        }
        if (t >= 0) hprev = hn;
        if (t >= 0 && t <= 15) {
          V5<T> fx = sub5(lds5(sF2, kF2, y * 17 + x + 1), lds5(sF2, kF2, y * 17 + x));
          V5<T> gy = sub5(lds5(sG2, kG2, (y + 1) * 16 + x), lds5(sG2, kG2, y * 16 + x));
#pragma unroll
          for (int n = 0; n < 5; ++n) accp[n] = fx[n] + gy[n];
        }
        if (FO) {
          const int f = (t == 0) ? 0 : (t == 16 ? 1 : (t == 8 && a.nf == 3 ? 2 : -1));
          if (f >= 0) {
#pragma unroll
            for (int n = 0; n < 5; ++n) FO[((2 * a.nf + f) * 5 + n) * 256 + y * 16 + x] = hn[n];
          }
        }
      } else if (FO && t >= 0 && t <= 15) {
        const int q = tid - 256;
        if (q < 2 * a.nf * 16) {
          const int d = q / (a.nf * 16), f = (q / 16) % a.nf, s = q % 16;
          const int fi = f == 0 ? -1 : (f == 1 ? 15 : 7);  // face index of offsets 0, 16, 8
          V5<T> v = d == 0 ? lds5(sF2, kF2, s * 17 + fi + 1) : lds5(sG2, kG2, (fi + 1) * 16 + s);
#pragma unroll
          for (int n = 0; n < 5; ++n) FO[((d * a.nf + f) * 5 + n) * 256 + t * 16 + s] = v[n];
        }
      }
      if (col.cross) {
        ztm = nzm;
        ztp = nzp;
      }
    }
    __syncthreads();
  }
  flush_diag(a, fails, floors);
}

}  // namespace ctu
}  // namespace hy
