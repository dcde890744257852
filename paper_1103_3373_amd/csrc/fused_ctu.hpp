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
//    limited slopes, face states, first-set fluxes and the transverse
//    z-flux differences (about 78 KB for FP32, so two workgroups share a
//    CU).  Every per-direction array is laid out in that direction's own
//    (along, across) coordinates with the components in its frame; the
//    primitive plane is kept twice, in lab order and transposed in y-frame
//    order.  An x task and a y task then differ only in base pointers, so
//    they share one code path and a wavefront that holds both does not
//    diverge.
//  * Per plane: A columns (prims, z trace, H1, dH1) | B x/y slopes |
//    C x/y face values (PPM: both edges of the cell), monotonization and
//    traces | D x/y Riemann set 1 | E corrected x/y Riemann set 2 and z correction
//    + z Riemann set 2 | F conservative update and flux store.  The update
//    of plane t-1 completes in plane t once its upper z flux exists.
//  * The correction of a face state is done by the task that solves that
//    face, so each corrected state is formed exactly once.
// Global memory sees the input (each group's cells plus, from the
// neighbouring groups, its ghost layers: about 2.4x the interior for g = 3,
// mostly served from L2), the output, the optional face fluxes, and the
// register spills of the two-workgroups-per-CU variant.
#pragma once

#include "fused_common.hpp"

namespace hy {
namespace ctu {

using namespace fz;

// LDS layout (elements of T).  Sizes are those of PPM (g = 3); PLM uses a
// subset of the same layout.  For direction d (0 = x, 1 = y) a cell has the
// along coordinate a and the across coordinate b: (a, b) = (x, y) for x and
// (y, x) for y.
constexpr int kNmax = 22;
constexpr int kP = kNmax * kNmax;    // primitive plane, full padded square
constexpr int kS = 18 * 20;          // slopes: b in -1..16, a in -2..17
constexpr int kSQ = 18 * 18;         // b, a in -1..16 (and the lab 18x18 square)
constexpr int kF1 = 18 * 17;         // first-set fluxes: b in -1..16, faces a+1/2, a in -1..15
constexpr int kF2 = 16 * 17;         // final fluxes: b in 0..15, faces a+1/2, a in -1..15
constexpr int oP = 0;                // [5][kP] lab order, (y+G) N + (x+G)
constexpr int oQ = oP + 5 * kP;      // [5][kP] y frame, transposed: (x+G) N + (y+G)
constexpr int oS = oQ + 5 * kP;      // [2][5][kS] frame of d, (b+1) 20 + (a+2)
constexpr int oW = oS + 10 * kS;     // [2][2][5][kSQ] frame of d, (b+1) 18 + (a+1); side 0 = left face
constexpr int oF1 = oW + 20 * kSQ;   // [2][5][kF1] frame of the OTHER direction, (b+1) 17 + (a+1)
constexpr int oDH = oF1 + 10 * kF1;  // [5][kSQ] lab order, (y+1) 18 + (x+1)
constexpr int kLds = oDH + 5 * kSQ;
constexpr int oF2 = oS;              // [2][5][kF2] frame of d, b 17 + (a+1): slopes are dead by then
static_assert(10 * kF2 <= 10 * kS, "final fluxes alias the slopes");
// After the T-typed area: byte offsets of the ring-corner and outer columns of
// the current group (column ids 320 .. 467), formed once per group, then the
// workgroup's two diagnostic counters (Roe fallbacks, floor hits).
constexpr int kOuterCols = 148;
constexpr size_t kLdsBytes(size_t elem) { return kLds * elem + kOuterCols * sizeof(unsigned) + 2 * sizeof(unsigned); }

// Diagnostic counts go straight to LDS counters (rare events), so no
// register carries them through the plane loop.
struct Tally {
  unsigned* c;  // [0] Roe fallbacks, [1] floor hits
  HY_DEV void fails(int v) const { if (v) atomicAdd(&c[0], (unsigned)v); }
  HY_DEV void floors(int v) const { if (v) atomicAdd(&c[1], (unsigned)v); }
  // A wavefront's floor hits (uniform): one atomic from its first active lane.
  HY_DEV void floors_wave(unsigned n) const {
    if (n) {
      const unsigned long long act = __builtin_amdgcn_ballot_w64(true);
      if ((unsigned long long)__lane_id() == (unsigned long long)__builtin_ctzll(act)) atomicAdd(&c[1], n);
    }
  }
};

// Frame changes for a direction d known per lane (0 = x, whose frame is the
// lab order, 1 = y, whose frame is (v, w, u)).
template <typename T> HY_DEV V5<T> to_frame_d(const V5<T>& v, bool d) {
  V5<T> r;
  r[0] = v[0]; r[1] = d ? v[2] : v[1]; r[2] = d ? v[3] : v[2]; r[3] = d ? v[1] : v[3]; r[4] = v[4];
  return r;
}
template <typename T> HY_DEV V5<T> from_frame_d(const V5<T>& v, bool d) {
  V5<T> r;
  r[0] = v[0]; r[1] = d ? v[3] : v[1]; r[2] = d ? v[1] : v[2]; r[3] = d ? v[2] : v[3]; r[4] = v[4];
  return r;
}
// Frame of d -> frame of the other direction.
template <typename T> HY_DEV V5<T> other_frame_d(const V5<T>& v, bool d) {
  V5<T> r;
  r[0] = v[0]; r[1] = d ? v[3] : v[2]; r[2] = d ? v[1] : v[3]; r[3] = d ? v[2] : v[1]; r[4] = v[4];
  return r;
}

// WAVES = minimum waves per SIMD the register allocation must allow: 2 gives
// one workgroup per CU without spills, 4 gives two workgroups per CU (with
// some spilling); the autotuner picks per specialization.
//
// FAST: the configuration of every production workload (van Leer limiter on
// characteristic variables) is compiled with those two choices fixed, so the
// limiter takes no run-time branch per component (about 10% of the kernel);
// every other combination runs the same code with run-time choices.
//
// ZR: groups per work item (tile depth 16 * ZR): ZR > 1 only for a single
// periodic box without flux output (a.zrun == ZR).
template <typename T, bool PPM, int RS, int WAVES, bool FAST, int ZR>
__global__ void __launch_bounds__(kThreads, WAVES) ctu_fused_kernel(FusedArgs<T> a) {
  constexpr int NT = kThreads;
  constexpr int G = PPM ? 3 : 2;
  constexpr int N = 16 + 2 * G;
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  T* sP = sm + oP;
  T* sQ = sm + oQ;
  T* sS = sm + oS;
  T* sW = sm + oW;
  T* sF1 = sm + oF1;
  T* sDH = sm + oDH;
  T* sF2 = sm + oF2;
  unsigned* sOC = reinterpret_cast<unsigned*>(smem_raw + kLds * sizeof(T));
  const Tally tally{reinterpret_cast<unsigned*>(smem_raw + kLds * sizeof(T) + kOuterCols * sizeof(unsigned))};

  const int tid = threadIdx.x;
  const Column<int> col = column_of<G>(tid);
  const int pcol = (col.y + G) * N + (col.x + G);  // primitive plane index, lab
  const int qcol = (col.x + G) * N + (col.y + G);  // the same cell in the transposed plane
  const int sqc = (col.y + 1) * 18 + (col.x + 1);  // 18x18 square index (cross columns)
  // Column classes are whole wavefronts (interior: waves 0-3, cross: 0-4),
  // so the tests are made on a wave-uniform value and do not diverge.
  const int wtid = uni(tid & ~63);
  const bool interior = wtid < 256;
  const bool cross = wtid < 320;
  constexpr int nCols = 324 + 4 * (G - 1) * 18;  // columns that feed the primitive plane
  static_assert(nCols - 320 <= kOuterCols, "outer column table");
  if (tid < 2) tally.c[tid] = 0u;
  __syncthreads();

  Phys<T> ph = make_phys(a);
  if (FAST) {
    ph.limiter = 1;  // van Leer
    ph.charlim = 1;
  }

  // Task counts per direction.  Slopes: PPM needs a in -2..17 (edges of the
  // traced cells), PLM a in -1..16.
  constexpr int wS = PPM ? 20 : 18, a0S = PPM ? -2 : -1;
  constexpr int nS = wS * 18;

  // Work items: single groups, or runs of ZR z-consecutive groups of one
  // periodic box (flux output off), marched through in one pass: the z
  // prologue and the two planes beyond each end are paid once per run.
  constexpr int nzt = 16 * ZR;  // interior planes of an item
  int seg = 0;
  const GroupOrder order = group_order(a.n_groups / ZR);
  for (long long item = order.first; item < order.end; item += order.stride) {
    double dt;
    const USeg S = find_seg(a, item * ZR, seg, dt);
    long long lg = item * ZR - S.first;  // the item's first group (local)
    int gzs = 0;                           // groups between z neighbours
    if constexpr (ZR > 1) {
      // item -> (column c, run r) of the box; group (r ZR + j) nxy + c
      const int nxy = S.ngx * S.ngy, li = (int)(item - S.first / ZR);
      lg = (long long)(li / nxy) * ZR * nxy + li % nxy;
      gzs = nxy;
    }
    T* __restrict__ O = reinterpret_cast<T*>(S.out) + lg * 5 * 4096;
    T* __restrict__ FO = (ZR == 1 && S.flux) ? reinterpret_cast<T*>(S.flux) + lg * 3 * a.nf * 5 * 256 : nullptr;
    // A box segment beyond the addressing limit gets NaN outputs: a NaN dt/dh
    // makes every updated cell NaN, and the face fluxes get NaN added.
    const T poison = slab_fits<T>(S) ? T(0) : T(__builtin_nan(""));
    ph.dtdh = (T)(dt / S.dh) + poison;
    ph.hdtdh = (T)(0.5 * dt / S.dh) + poison;
    // The group's cells (ghosts included) come from the ghosted input or, in
    // box mode, straight from the periodic grouped box.
    ColumnReader<T, G> rd;
    rd.init(S, lg, col.x, col.y);
    if (!cross) {
      // Each thread reads back only the slots it writes: no barrier needed.
      for (int c = tid; c < nCols; c += NT - 320) {
        const Column<int> oc = column_of<G>(c);
        ColumnReader<T, G> orr;
        orr.init(S, lg, oc.x, oc.y);
        sOC[c - 320] = orr.off;
      }
    }
    auto load_cons = [&](int z) -> V5<T> { return rd.load(z); };
    auto zprim = [&](int z) -> V5<T> { return to_frame<2>(prim_of(load_cons(z), ph)); };

    // Register state of a cross column (frame z unless noted):
    V5<T> w0, w1, w2;   // W(t), W(t+1), W(t+2)   (PLM: w0, w1)
    V5<T> s1, e0;       // S(t+1), E(t+1/2)       (PPM)
    V5<T> ztm, ztp;     // traced states of plane t
    V5<T> h1m;          // H1(t-1/2)
    V5<T> zcp;          // corrected right state of plane t-1
    V5<T> acc;          // flux differences of the plane being updated, all but its upper z face (lab)
    // The plane that enters the window next (t + ahead in iteration t) is
    // requested one plane early, so its load overlaps a whole iteration; the
    // last plane a column reads is zlast (the last iteration repeats it).
    V5<T> unext;        // conserved state of that plane
    constexpr int ahead = PPM ? 3 : 2;
    const int zlast = nzt + ahead - 1;

    // ---- prologue: window and traced states of plane -1 -------------------
    if (cross) {
      if (PPM) {
        V5<T> wa = zprim(-3), wb = zprim(-2);
        w0 = zprim(-1);
        w1 = zprim(0);
        w2 = zprim(1);
        unext = load_cons(-1 + ahead);
        V5<T> sa = slope<PPM>(wa, wb, w0, ph), sb = slope<PPM>(wb, w0, w1, ph);
        s1 = slope<PPM>(w0, w1, w2, ph);
        ztm = ppm_edge(wb, w0, sa, sb);
        e0 = ppm_edge(w0, w1, sb, s1);
        ztp = e0;
        ppm_mono(w0, ztm, ztp);
        ctu_trace<true>(w0, ztm, ztp, ph);
      } else {
        V5<T> wb = zprim(-2);
        w0 = zprim(-1);
        w1 = zprim(0);
        unext = load_cons(-1 + ahead);
        V5<T> sb = slope<PPM>(wb, w0, w1, ph);
        plm_faces(wb, w0, w1, sb, ph, ztm, ztp);
        ctu_trace<false>(w0, ztm, ztp, ph);
      }
      tally.floors_wave(floor_wave(ztm, ph) + floor_wave(ztp, ph));
    }

    for (int t = -1; t <= nzt; ++t) {
      // ---- A: columns: primitive plane t; trace plane t+1; H1(t+1/2) -------
      V5<T> nzm, nzp;  // traced states of plane t+1
      if (cross) {
        const V5<T> wl = from_frame<2>(w0);
        sts5(sP, kP, pcol, wl);
        sts5(sQ, kP, qcol, to_frame<1>(wl));
        // The last plane (t == nzt) needs nothing above it.  The work is done
        // anyway, on a clamped plane index, so that the column's register
        // window advances the same way on every iteration (no copies at a
        // join); its diagnostics are not counted and its results are unused.
        const bool live = t < nzt;
        const V5<T> w3 = to_frame<2>(prim_of(unext, ph));  // plane min(t + ahead, zlast)
        unext = load_cons(t + 1 + ahead < zlast ? t + 1 + ahead : zlast);
        if (PPM) {
          V5<T> s2 = slope<PPM>(w1, w2, w3, ph);
          V5<T> e1 = ppm_edge(w1, w2, s1, s2);
          nzm = e0;
          nzp = e1;
          ppm_mono(w1, nzm, nzp);
          ctu_trace<true>(w1, nzm, nzp, ph);
          w0 = w1; w1 = w2; w2 = w3; s1 = s2; e0 = e1;
        } else {
          V5<T> sb = slope<PPM>(w0, w1, w3, ph);
          plm_faces(w0, w1, w3, sb, ph, nzm, nzp);
          ctu_trace<false>(w1, nzm, nzp, ph);
          w0 = w1; w1 = w3;
        }
        const unsigned fl = floor_wave(nzm, ph) + floor_wave(nzp, ph);
        int nf = 0;
        V5<T> h1p = riemann<RS>(ztp, nzm, ph, &nf);  // H1(t+1/2)
        if (live) {
          tally.floors_wave(fl);
          tally.fails(nf);
        }
        if (t >= 0) sts5(sDH, kSQ, sqc, from_frame<2>(sub5(h1p, h1m)));
        h1m = h1p;
      } else {
        // Ring corners and outer columns (column ids 320 .. nCols-1), strided
        // over the threads that own no cross column.
        for (int c = tid; c < nCols; c += NT - 320) {
          const Column<int> oc = column_of<G>(c);
          ColumnReader<T, G> orr = rd;  // z part of the group
          orr.off = sOC[c - 320];
          const V5<T> wl = prim_of(orr.load(t), ph);
          sts5(sP, kP, (oc.y + G) * N + (oc.x + G), wl);
          sts5(sQ, kP, (oc.x + G) * N + (oc.y + G), to_frame<1>(wl));
        }
      }
      __syncthreads();

      // ---- B: limited slopes along x and y of plane t ----------------------
      for (int q = tid; q < 2 * nS; q += NT) {
        const bool d = q >= nS;
        const int r = d ? q - nS : q;
        const int aa = r % wS + a0S, b = r / wS - 1;
        const T* pl = d ? sQ : sP;
        const int c = (b + G) * N + (aa + G);
        V5<T> s = slope<PPM>(lds5(pl, kP, c - 1), lds5(pl, kP, c), lds5(pl, kP, c + 1), ph);
        sts5(sS + (d ? 5 * kS : 0), kS, (b + 1) * 20 + (aa + 2), s);
      }
      __syncthreads();

      // ---- C: traced x and y face states of plane t (frame of d) -----------
      for (int q = tid; q < 2 * kSQ; q += NT) {
        const bool d = q >= kSQ;
        const int r = d ? q - kSQ : q;
        const int aa = r % 18 - 1, b = r / 18 - 1;
        const T* pl = d ? sQ : sP;
        const int c = (b + G) * N + (aa + G);
        T* w = sW + (d ? 10 * kSQ : 0);
        const V5<T> wc = lds5(pl, kP, c);
        V5<T> fl, fr;
        if (PPM) {
          // Both PPM edges of the cell.  An edge shared by two cells is
          // evaluated by each of them, with the same operands in the same
          // order, so both get the same value; that costs less than a phase
          // of its own (index math, a barrier, a partly filled wavefront).
          const T* ss = sS + (d ? 5 * kS : 0);
          const int si = (b + 1) * 20 + (aa + 2);
          const V5<T> s0 = lds5(ss, kS, si);
          fl = ppm_edge(lds5(pl, kP, c - 1), wc, lds5(ss, kS, si - 1), s0);
          fr = ppm_edge(wc, lds5(pl, kP, c + 1), s0, lds5(ss, kS, si + 1));
          ppm_mono(wc, fl, fr);
        } else {
          const T* ss = sS + (d ? 5 * kS : 0);
          plm_faces(lds5(pl, kP, c - 1), wc, lds5(pl, kP, c + 1), lds5(ss, kS, (b + 1) * 20 + (aa + 2)), ph, fl,
                    fr);
        }
        ctu_trace<PPM>(wc, fl, fr, ph);
        tally.floors_wave(floor_wave(fl, ph) + floor_wave(fr, ph));
        sts5(w, kSQ, r, fl);
        sts5(w + 5 * kSQ, kSQ, r, fr);
      }
      __syncthreads();

      // ---- D: first-set Riemann solves in x and y, stored in the other
      //         direction's frame (where they are used) ----------------------
      for (int q = tid; q < 2 * kF1; q += NT) {
        const bool d = q >= kF1;
        const int r = d ? q - kF1 : q;
        const int i = r % 17 - 1, b = r / 17 - 1;  // face between cells i and i+1 of row b
        const T* w = sW + (d ? 10 * kSQ : 0);
        const int l = (b + 1) * 18 + (i + 1);
        int nf = 0;
        V5<T> F = riemann<RS>(lds5(w + 5 * kSQ, kSQ, l), lds5(w, kSQ, l + 1), ph, &nf);
        tally.fails(nf);
        sts5(sF1 + (d ? 5 * kF1 : 0), kF1, r, other_frame_d(F, d));
      }
      __syncthreads();

      // ---- E: corrected x/y faces and their final fluxes (planes 0..15);
      //         z correction of plane t and H(t-1/2) (interior columns) ----
      V5<T> hn;
      if (interior) {
        const int x = col.x, y = col.y;
        // x fluxes (stored in the y frame) at x -+ 1/2, y fluxes (stored in
        // the lab order) at y -+ 1/2.
        V5<T> dF = sub5(lds5(sF1, kF1, (y + 1) * 17 + x + 1), lds5(sF1, kF1, (y + 1) * 17 + x));
        V5<T> dG = sub5(lds5(sF1 + 5 * kF1, kF1, (x + 1) * 17 + y + 1), lds5(sF1 + 5 * kF1, kF1, (x + 1) * 17 + y));
        const V5<T> fz_ = to_frame<2>(from_frame<1>(dF)), gz_ = to_frame<2>(dG);
        V5<T> d;
#pragma unroll
        for (int n = 0; n < 5; ++n) d[n] = fz_[n] + gz_[n];
        unsigned nfl = 0;
        int nf = 0;
        V5<T> cm = correct(ztm, d, ph, nfl), cp = correct(ztp, d, ph, nfl);
        if (t >= 0) hn = from_frame<2>(riemann<RS>(zcp, cm, ph, &nf));  // H(t-1/2)
        tally.floors_wave(nfl);
        tally.fails(nf);
        zcp = cp;
      }
      if (t >= 0 && t < nzt) {
        for (int q = NT - 1 - tid; q < 2 * kF2; q += NT) {
          const bool d = q >= kF2;
          const int r = d ? q - kF2 : q;
          const int i = r % 17 - 1, b = r / 17;  // face between cells i and i+1 of row b
          const T* w = sW + (d ? 10 * kSQ : 0);
          // The other direction's first-set fluxes, already in this frame:
          // its rows are this direction's cells, its faces run along b.
          const T* fo = sF1 + (d ? 0 : 5 * kF1);
          V5<T> ol = sub5(lds5(fo, kF1, (i + 1) * 17 + b + 1), lds5(fo, kF1, (i + 1) * 17 + b));
          V5<T> orr = sub5(lds5(fo, kF1, (i + 2) * 17 + b + 1), lds5(fo, kF1, (i + 2) * 17 + b));
          // z-flux differences of the two cells, lab order -> this frame.
          const int hl = d ? (i + 1) * 18 + (b + 1) : (b + 1) * 18 + (i + 1);
          const int hr = hl + (d ? 18 : 1);
          const V5<T> Hl = to_frame_d(lds5(sDH, kSQ, hl), d), Hr = to_frame_d(lds5(sDH, kSQ, hr), d);
          V5<T> dl, dr;
#pragma unroll
          for (int n = 0; n < 5; ++n) { dl[n] = ol[n] + Hl[n]; dr[n] = orr[n] + Hr[n]; }
          const int l = (b + 1) * 18 + (i + 1);
          unsigned nfl = 0;
          int nf = 0;
          V5<T> L = correct(lds5(w + 5 * kSQ, kSQ, l), dl, ph, nfl);
          V5<T> R = correct(lds5(w, kSQ, l + 1), dr, ph, nfl);
          sts5(sF2 + (d ? 5 * kF2 : 0), kF2, r, riemann<RS>(L, R, ph, &nf));
          tally.floors_wave(nfl);
          tally.fails(nf);
        }
      }
      __syncthreads();

      // ---- F: finish plane t-1; in-plane flux differences of plane t;
      //         boundary fluxes (Sec. 2 step 5) ------------------------------
      if (interior) {
        const int x = col.x, y = col.y;
        if (t >= 1) {
          V5<T> u = load_cons(t - 1);
          // plane t-1 lies in the item's group (t-1)/16, at its z = (t-1)%16
          T* Og = O;
          if constexpr (ZR > 1) Og += (long)((t - 1) >> 4) * gzs * (5 * 4096);
          const int o = (((t - 1) & 15) * 16 + y) * 16 + x;
#pragma unroll
          for (int n = 0; n < 5; ++n) gstore(Og + n * 4096, (unsigned)o * (unsigned)sizeof(T), u[n] - ph.dtdh * (acc[n] + hn[n]));
        }
        if (t >= 0 && t < nzt) {
          V5<T> fx = sub5(lds5(sF2, kF2, y * 17 + x + 1), lds5(sF2, kF2, y * 17 + x));
          V5<T> gy = from_frame<1>(sub5(lds5(sF2 + 5 * kF2, kF2, x * 17 + y + 1), lds5(sF2 + 5 * kF2, kF2, x * 17 + y)));
#pragma unroll
          for (int n = 0; n < 5; ++n) acc[n] = (fx[n] + gy[n]) - hn[n];  // hn is the lower z face of plane t
        }
        if (FO) {
          const int f = (t == 0) ? 0 : (t == 16 ? 1 : (t == 8 && a.nf == 3 ? 2 : -1));
          if (f >= 0) {
#pragma unroll
            for (int n = 0; n < 5; ++n) gstore(FO + ((2 * a.nf + f) * 5 + n) * 256, (unsigned)(y * 16 + x) * (unsigned)sizeof(T), hn[n] + poison);
          }
        }
      } else if (FO && t >= 0 && t < nzt) {
        const int q = tid - 256;
        if (q < 2 * a.nf * 16) {
          const bool d = q >= a.nf * 16;
          const int f = (q / 16) % a.nf, s = q % 16;
          const int fi = f == 0 ? -1 : (f == 1 ? 15 : 7);  // face index of offsets 0, 16, 8
          const V5<T> v = from_frame_d(lds5(sF2 + (d ? 5 * kF2 : 0), kF2, s * 17 + fi + 1), d);
#pragma unroll
          for (int n = 0; n < 5; ++n) gstore(FO + (((d ? 1 : 0) * a.nf + f) * 5 + n) * 256, (unsigned)(t * 16 + s) * (unsigned)sizeof(T), v[n] + poison);
        }
      }
      if (cross) {
        ztm = nzm;
        ztp = nzp;
      }
    }
    __syncthreads();
  }
  if (tid < 2 && a.diag && tally.c[tid]) atomicAdd(&a.diag[tid], (unsigned long long)tally.c[tid]);
}

}  // namespace ctu
}  // namespace hy
