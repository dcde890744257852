// Fused MUSCL-Hancock (MHM) solver and the second stage of the VL scheme
// for patch groups (arXiv:1103.3373, Sec. 2), in the z-marching layout of
// the fused CTU kernel (one 512-thread workgroup per group, column threads
// with z windows in registers, x/y work of the current plane in LDS).
//
// MODE 0 (MHM): reconstruct the six face states of a cell from U^n, advance
//   all of them by one cell-centred dU = -dt/(2dh) sum_d [F_d(U_{d+}) -
//   F_d(U_{d-})] (no Riemann solver), then one Riemann solve per face and
//   the conservative update.
// MODE 1 (VL, second stage): the input is the half-step primitive state W*
//   produced by the VL predictor kernel; reconstruct it (no predictor), one
//   Riemann solve per face, and update U^n (read from the segment) with the
//   full dt.
//
// Per plane t (t = -1 .. 16): A columns (primitive plane t, z face states of
// plane t) | B x/y slopes | C x/y face states (PPM: both edges of the cell
// and monotonization) | D (MHM) Hancock half step of the cross cells by their column
// threads | E x/y Riemann faces of plane t and the z Riemann face below it |
// F update of plane t-1 and boundary fluxes.  As in the CTU kernel, every
// per-direction LDS array is laid out in the direction's own (along,
// across) coordinates and frame, with the primitive plane also kept
// transposed in y-frame order, so x and y tasks share one code path.
#pragma once

#include "fused_ctu.hpp"

namespace hy {
namespace muscl {

using namespace fz;
using ctu::kP;
using ctu::kS;
using ctu::kSQ;
using ctu::kF2;
using ctu::Tally;
using ctu::to_frame_d;
using ctu::from_frame_d;

constexpr int oP = 0;               // [5][kP] lab order, (y+G) N + (x+G)
constexpr int oQ = oP + 5 * kP;     // [5][kP] y frame, transposed: (x+G) N + (y+G)
constexpr int oS = oQ + 5 * kP;     // [2][5][kS] frame of d, (b+1) 20 + (a+2)
constexpr int oW = oS + 10 * kS;    // [2][2][5][kSQ] frame of d, (b+1) 18 + (a+1); side 0 = left face
constexpr int kLds = oW + 20 * kSQ;
constexpr int oF2 = oS;             // [2][5][kF2] frame of d, b 17 + (a+1): slopes are dead by then
static_assert(10 * kF2 <= 10 * kS, "final fluxes alias the slopes");
constexpr size_t kLdsBytes(size_t elem) { return kLds * elem + 2 * sizeof(unsigned); }

// FAST as in the CTU kernel: van Leer on characteristic variables fixed at
// compile time.  ZR as in the CTU kernel: groups per work item (tile depth
// 16 * ZR), ZR > 1 only for a single periodic box without flux output.
template <typename T, bool PPM, int RS, int WAVES, int MODE, bool FAST, int ZR>
__global__ void __launch_bounds__(kThreads, WAVES) muscl_kernel(FusedArgs<T> a) {
  constexpr int NT = kThreads;
  constexpr int G = PPM ? 3 : 2;
  constexpr int N = 16 + 2 * G;
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  T* sP = sm + oP;
  T* sQ = sm + oQ;
  T* sS = sm + oS;
  T* sW = sm + oW;
  T* sF2 = sm + oF2;
  const Tally tally{reinterpret_cast<unsigned*>(smem_raw + kLds * sizeof(T))};

  const int tid = threadIdx.x;
  const Column<int> col = column_of<G>(tid);
  const int pcol = (col.y + G) * N + (col.x + G);
  const int qcol = (col.x + G) * N + (col.y + G);
  const int sqx = (col.y + 1) * 18 + (col.x + 1);  // the cross cell in the x arrays
  const int sqy = (col.x + 1) * 18 + (col.y + 1);  // ... and in the (transposed) y arrays
  // Column classes are whole wavefronts (interior: waves 0-3, cross: 0-4),
  // so the tests are made on a wave-uniform value and do not diverge.
  const int wtid = uni(tid & ~63);
  const bool interior = wtid < 256;
  const bool cross = wtid < 320;
  if (tid < 2) tally.c[tid] = 0u;
  __syncthreads();
  Phys<T> ph = make_phys(a);
  if (FAST) {
    ph.limiter = 1;  // van Leer
    ph.charlim = 1;
  }

  constexpr int wS = PPM ? 20 : 18, a0S = PPM ? -2 : -1;
  constexpr int nS = wS * 18;

  // Work items: single groups, or runs of ZR z-consecutive groups of one
  // periodic box, marched through in one pass (the z prologue and the
  // planes beyond each end are paid once per run).
  constexpr int nzt = 16 * ZR;  // interior planes of an item
  int seg = 0;
  const GroupOrder order = group_order(a.n_groups / ZR);
  for (long long item = order.first; item < order.end; item += order.stride) {
    double dt;
    const USeg S = find_seg(a, item * ZR, seg, dt);
    long long lg = item * ZR - S.first;  // the item's first group (local)
    int gzs = 0;                          // groups between z neighbours
    if constexpr (ZR > 1) {
      // item -> (column c, run r) of the box; group (r ZR + j) nxy + c
      const int nxy = S.ngx * S.ngy, li = (int)(item - S.first / ZR);
      lg = (long long)(li / nxy) * ZR * nxy + li % nxy;
      gzs = nxy;
    }
    const long long grp = S.first + lg;
    T* __restrict__ O = reinterpret_cast<T*>(S.out) + lg * 5 * 4096;
    T* __restrict__ FO = (ZR == 1 && S.flux) ? reinterpret_cast<T*>(S.flux) + lg * 3 * a.nf * 5 * 256 : nullptr;
    ph.dtdh = (T)(dt / S.dh);
    ph.hdtdh = (T)(0.5 * dt / S.dh);
    // A segment that is no box in a launch that declared boxes only (its
    // half step was not computed for it), or a box whose z-slab of groups
    // exceeds 4 GiB: its output is made NaN.
    const T poison = ((MODE == 1 && a.wstar_box && !S.box) || !slab_fits<T>(S)) ? T(__builtin_nan("")) : T(0);

    // Sources: MHM reads U^n (ghost width G) and converts; VL reads the
    // half-step primitive W* from the predictor's scratch (ghost width G)
    // and U^n for the update from the segment (ghost width G + 1).
    ColumnReader<T, G> src;
    ColumnReader<T, G + 1> upd;
    if (MODE == 0) {
      src.init(S, lg, col.x, col.y);
    } else {
      if (a.wstar_box) {
        // W* of this segment is a grouped periodic box of the segment's
        // shape: ghost cells come from the neighbouring groups.
        USeg w = S;
        w.in = a.wstar + S.first * 5 * 4096;
        src.init(w, lg, col.x, col.y);
      } else {
        USeg w{};
        w.in = a.wstar;
        src.init(w, grp, col.x, col.y);
      }
      upd.init(S, lg, col.x, col.y);
    }
    auto wprim = [&](int z) -> V5<T> {
      V5<T> v = src.load(z);
      return MODE == 0 ? prim_of(v, ph) : v;
    };
    auto ucons = [&](int z) -> V5<T> { return MODE == 0 ? src.load(z) : upd.load(z); };
    auto zprim = [&](int z) -> V5<T> { return to_frame<2>(wprim(z)); };
    auto put_plane = [&](int idx_p, int idx_q, const V5<T>& wl) {
      sts5(sP, kP, idx_p, wl);
      sts5(sQ, kP, idx_q, to_frame<1>(wl));
    };

    // Column state (frame z):
    //   PPM: wa = W(t), wb = W(t+1), st = S(t), em = E(t-1/2)
    //   PLM: wa = W(t-1), wb = W(t)
    V5<T> wa, wb, st, em;
    V5<T> zfm, zfp;   // z face states of plane t (half-stepped in MHM)
    V5<T> zhp;        // right z state of plane t-1
    V5<T> acc;        // flux differences of the plane being updated, all but its upper z face (lab)
    V5<T> wnext;      // the column's newest z plane, loaded one plane ahead (prims)
    constexpr int zAhead = PPM ? 2 : 1;
    if (cross) {
      if (PPM) {
        V5<T> w3 = zprim(-3), w2 = zprim(-2);
        wa = zprim(-1);
        wb = zprim(0);
        V5<T> s2 = slope<PPM>(w3, w2, wa, ph);
        st = slope<PPM>(w2, wa, wb, ph);
        em = ppm_edge(w2, wa, s2, st);
      } else {
        wa = zprim(-2);
        wb = zprim(-1);
      }
      wnext = src.load(-1 + zAhead);
    }

    for (int t = -1; t <= nzt; ++t) {
      // ---- A: primitive planes t; z face states of plane t -----------------
      if (cross) {
        if (PPM) {
          put_plane(pcol, qcol, from_frame<2>(wa));
          V5<T> wc = to_frame<2>(MODE == 0 ? prim_of(wnext, ph) : wnext);  // plane t + 2
          wnext = src.load(t + 1 + zAhead <= nzt + zAhead ? t + 1 + zAhead : nzt + zAhead);
          V5<T> sn = slope<PPM>(wa, wb, wc, ph);
          V5<T> ep = ppm_edge(wa, wb, st, sn);
          zfm = em;
          zfp = ep;
          ppm_mono(wa, zfm, zfp);
          wa = wb; wb = wc; st = sn; em = ep;
        } else {
          put_plane(pcol, qcol, from_frame<2>(wb));
          V5<T> wc = to_frame<2>(MODE == 0 ? prim_of(wnext, ph) : wnext);  // plane t + 1
          wnext = src.load(t + 1 + zAhead <= nzt + zAhead ? t + 1 + zAhead : nzt + zAhead);
          V5<T> s0 = slope<PPM>(wa, wb, wc, ph);
          plm_faces(wa, wb, wc, s0, ph, zfm, zfp);
          wa = wb; wb = wc;
        }
        tally.floors_wave(floor_wave(zfm, ph) + floor_wave(zfp, ph));
      } else if (col.active) {
        put_plane(pcol, qcol, wprim(t));
      }
      __syncthreads();

      // ---- B: limited slopes along x and y ---------------------------------
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

      // ---- C: x and y face states (frame of d) -----------------------------
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
        tally.floors_wave(floor_wave(fl, ph) + floor_wave(fr, ph));
        sts5(w, kSQ, r, fl);
        sts5(w + 5 * kSQ, kSQ, r, fr);
      }
      __syncthreads();

      // ---- D (MHM): Hancock half step of every cross cell ------------------
      if (MODE == 0) {
        if (cross) {
          T* wx = sW;
          T* wy = sW + 10 * kSQ;
          V5<T> xm = lds5(wx, kSQ, sqx), xp = lds5(wx + 5 * kSQ, kSQ, sqx);
          V5<T> ym = lds5(wy, kSQ, sqy), yp = lds5(wy + 5 * kSQ, kSQ, sqy);
          V5<T> dU;
          {
            V5<T> fp = from_frame<0>(flux_of(xp, ph)), fm = from_frame<0>(flux_of(xm, ph));
#pragma unroll
            for (int n = 0; n < 5; ++n) dU[n] = fp[n] - fm[n];
          }
          {
            V5<T> fp = from_frame<1>(flux_of(yp, ph)), fm = from_frame<1>(flux_of(ym, ph));
#pragma unroll
            for (int n = 0; n < 5; ++n) dU[n] += fp[n] - fm[n];
          }
          {
            V5<T> fp = from_frame<2>(flux_of(zfp, ph)), fm = from_frame<2>(flux_of(zfm, ph));
#pragma unroll
            for (int n = 0; n < 5; ++n) dU[n] += fp[n] - fm[n];
          }
          V5<T> dx = to_frame<0>(dU), dy = to_frame<1>(dU), dz = to_frame<2>(dU);
          unsigned nfl = 0;
          sts5(wx, kSQ, sqx, correct(xm, dx, ph, nfl));
          sts5(wx + 5 * kSQ, kSQ, sqx, correct(xp, dx, ph, nfl));
          sts5(wy, kSQ, sqy, correct(ym, dy, ph, nfl));
          sts5(wy + 5 * kSQ, kSQ, sqy, correct(yp, dy, ph, nfl));
          zfm = correct(zfm, dz, ph, nfl);
          zfp = correct(zfp, dz, ph, nfl);
          tally.floors_wave(nfl);
        }
        __syncthreads();
      }

      // ---- E: Riemann solves: x/y faces of plane t, z face below it --------
      V5<T> hn;
      if (interior) {
        int nf = 0;
        if (t >= 0) hn = from_frame<2>(riemann<RS>(zhp, zfm, ph, &nf));  // H(t-1/2)
        tally.fails(nf);
        zhp = zfp;
      }
      if (t >= 0 && t < nzt) {
        for (int q = NT - 1 - tid; q < 2 * kF2; q += NT) {
          const bool d = q >= kF2;
          const int r = d ? q - kF2 : q;
          const int i = r % 17 - 1, b = r / 17;  // face between cells i and i+1 of row b
          const T* w = sW + (d ? 10 * kSQ : 0);
          const int l = (b + 1) * 18 + (i + 1);
          int nf = 0;
          V5<T> F = riemann<RS>(lds5(w + 5 * kSQ, kSQ, l), lds5(w, kSQ, l + 1), ph, &nf);
          tally.fails(nf);
          sts5(sF2 + (d ? 5 * kF2 : 0), kF2, r, F);
        }
      }
      __syncthreads();

      // ---- F: update plane t-1; flux differences of plane t; face fluxes ---
      if (interior) {
        const int x = col.x, y = col.y;
        if (t >= 1) {
          V5<T> u = ucons(t - 1);
          // plane t-1 lies in the item's group (t-1)/16, at its z = (t-1)%16
          T* Og = O;
          if constexpr (ZR > 1) Og += (long)((t - 1) >> 4) * gzs * (5 * 4096);
          const int o = (((t - 1) & 15) * 16 + y) * 16 + x;
#pragma unroll
          for (int n = 0; n < 5; ++n) gstore(Og + n * 4096, (unsigned)o * (unsigned)sizeof(T), u[n] - ph.dtdh * (acc[n] + hn[n]) + poison);
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
          const int fi = f == 0 ? -1 : (f == 1 ? 15 : 7);
          const V5<T> v = from_frame_d(lds5(sF2 + (d ? 5 * kF2 : 0), kF2, s * 17 + fi + 1), d);
#pragma unroll
          for (int n = 0; n < 5; ++n) gstore(FO + (((d ? 1 : 0) * a.nf + f) * 5 + n) * 256, (unsigned)(t * 16 + s) * (unsigned)sizeof(T), v[n] + poison);
        }
      }
    }
    __syncthreads();
  }
  if (tid < 2 && a.diag && tally.c[tid]) atomicAdd(&a.diag[tid], (unsigned long long)tally.c[tid]);
}

}  // namespace muscl
}  // namespace hy
