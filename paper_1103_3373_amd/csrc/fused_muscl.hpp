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
// plane t) | B x/y slopes | C x/y face states | D (MHM) Hancock half step of
// the cross cells by their column threads | E x/y Riemann faces of plane t
// and the z Riemann face below it | F update of plane t-1 and boundary
// fluxes.  Four (VL) or five (MHM) barriers per plane.
#pragma once

#include "fused_common.hpp"

namespace hy {
namespace muscl {

using namespace fz;

constexpr int kNmax = 22;
constexpr int kP = kNmax * kNmax;
constexpr int kSX = 20 * 18;
constexpr int kSY = 18 * 20;
constexpr int kSQ = 18 * 18;
constexpr int oP = 0;
constexpr int oSX = oP + 5 * kP;
constexpr int oSY = oSX + 5 * kSX;
constexpr int oWX = oSY + 5 * kSY;
constexpr int oWY = oWX + 10 * kSQ;
constexpr int kLds = oWY + 10 * kSQ;
constexpr int kF2 = 17 * 16;
constexpr int kG2 = 16 * 17;
constexpr int oF2 = oSX;
constexpr int oG2 = oSX + 5 * kF2;
static_assert(10 * kF2 <= 5 * (kSX + kSY), "F2/G2 alias");

template <typename T, bool PPM, int RS, int WAVES, int MODE>
__global__ void __launch_bounds__(kThreads, WAVES) muscl_kernel(FusedArgs<T> a) {
  constexpr int G = PPM ? 3 : 2;
  constexpr int N = 16 + 2 * G;
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  T* sP = sm + oP;
  T* sSX = sm + oSX;
  T* sSY = sm + oSY;
  T* sWX = sm + oWX;
  T* sWY = sm + oWY;
  T* sF2 = sm + oF2;
  T* sG2 = sm + oG2;

  const int tid = threadIdx.x;
  const Column<int> col = column_of<G>(tid);
  const int pcol = (col.y + G) * N + (col.x + G);
  const int sqc = (col.y + 1) * 18 + (col.x + 1);
  const bool interior = tid < 256;
  int fails = 0, floors = 0;
  Phys<T> ph = make_phys(a);

  constexpr int wSX = PPM ? 20 : 18, x0SX = PPM ? -2 : -1;
  constexpr int nSX = wSX * 18;
  constexpr int hSY = PPM ? 20 : 18, y0SY = PPM ? -2 : -1;
  constexpr int nSY = 18 * hSY;

  int seg = 0;
  const GroupOrder order = group_order(a.n_groups);
  for (long long grp = order.first; grp < order.end; grp += order.stride) {
    double dt;
    const Seg* S = find_seg(a, grp, seg, dt);
    const long long lg = grp - S->first;
    T* __restrict__ O = reinterpret_cast<T*>(S->out) + lg * 5 * 4096;
    T* __restrict__ FO = S->flux ? reinterpret_cast<T*>(S->flux) + lg * 3 * a.nf * 5 * 256 : nullptr;
    ph.dtdh = (T)(dt / S->dh);
    ph.hdtdh = (T)(0.5 * dt / S->dh);

    // Sources: MHM reads U^n (ghost width G) and converts; VL reads the
    // half-step primitive W* from the predictor's scratch (ghost width G)
    // and U^n for the update from the segment (ghost width G + 1).
    ColumnReader<T, G> src;
    ColumnReader<T, G + 1> upd;
    if (MODE == 0) {
      src.init(S, lg, col.x, col.y);
    } else {
      Seg w{};
      w.in = a.wstar;
      src.init(&w, grp, col.x, col.y);
      upd.init(S, lg, col.x, col.y);
    }
    auto wprim = [&](int z) -> V5<T> {
      V5<T> v = src.load(z);
      return MODE == 0 ? prim_of(v, ph) : v;
    };
    auto ucons = [&](int z) -> V5<T> { return MODE == 0 ? src.load(z) : upd.load(z); };
    auto zprim = [&](int z) -> V5<T> { return to_frame<2>(wprim(z)); };

    // Column state (frame z):
    //   PPM: wa = W(t), wb = W(t+1), st = S(t), em = E(t-1/2)
    //   PLM: wa = W(t-1), wb = W(t)
    V5<T> wa, wb, st, em;
    V5<T> zfm, zfp;   // z face states of plane t (half-stepped in MHM)
    V5<T> zhp;        // right z state of plane t-1
    V5<T> hprev, accp;
    if (col.cross) {
      if (PPM) {
        V5<T> w3 = zprim(-3), w2 = zprim(-2);
        wa = zprim(-1);
        wb = zprim(0);
        V5<T> s2 = slope(w3, w2, wa, ph);
        st = slope(w2, wa, wb, ph);
        em = ppm_edge(w2, wa, s2, st);
      } else {
        wa = zprim(-2);
        wb = zprim(-1);
      }
    }

    for (int t = -1; t <= 16; ++t) {
      // ---- A: primitive plane t; z face states of plane t ------------------
      if (col.cross) {
        if (PPM) {
          sts5(sP, kP, pcol, from_frame<2>(wa));
          V5<T> wc = zprim(t + 2);
          V5<T> sn = slope(wa, wb, wc, ph);
          V5<T> ep = ppm_edge(wa, wb, st, sn);
          zfm = em;
          zfp = ep;
          ppm_mono(wa, zfm, zfp);
          wa = wb; wb = wc; st = sn; em = ep;
        } else {
          sts5(sP, kP, pcol, from_frame<2>(wb));
          V5<T> wc = zprim(t + 1);
          V5<T> s0 = slope(wa, wb, wc, ph);
          plm_faces(wa, wb, wc, s0, ph, zfm, zfp);
          wa = wb; wb = wc;
        }
        floors += floor_state(zfm, ph) + floor_state(zfp, ph);
      } else if (col.active) {
        sts5(sP, kP, pcol, wprim(t));
      }
      __syncthreads();

      // ---- B: limited slopes along x and y ---------------------------------
      for (int q = tid; q < nSX + nSY; q += kThreads) {
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

      // ---- C: x and y face states (frame order) ----------------------------
      for (int q = tid; q < 2 * kSQ; q += kThreads) {
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
          floors += floor_state(fl, ph) + floor_state(fr, ph);
          sts5(sWY, kSQ, r, fl);
          sts5(sWY + 5 * kSQ, kSQ, r, fr);
        }
      }
      __syncthreads();

      // ---- D (MHM): Hancock half step of every cross cell ------------------
      if (MODE == 0) {
        if (col.cross) {
          V5<T> xm = lds5(sWX, kSQ, sqc), xp = lds5(sWX + 5 * kSQ, kSQ, sqc);
          V5<T> ym = lds5(sWY, kSQ, sqc), yp = lds5(sWY + 5 * kSQ, kSQ, sqc);
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
          sts5(sWX, kSQ, sqc, correct(xm, dx, ph, floors));
          sts5(sWX + 5 * kSQ, kSQ, sqc, correct(xp, dx, ph, floors));
          sts5(sWY, kSQ, sqc, correct(ym, dy, ph, floors));
          sts5(sWY + 5 * kSQ, kSQ, sqc, correct(yp, dy, ph, floors));
          zfm = correct(zfm, dz, ph, floors);
          zfp = correct(zfp, dz, ph, floors);
        }
        __syncthreads();
      }

      // ---- E: Riemann solves: x/y faces of plane t, z face below it --------
      V5<T> hn;
      if (interior) {
        if (t >= 0) hn = from_frame<2>(riemann<RS>(zhp, zfm, ph, &fails));  // H(t-1/2)
        zhp = zfp;
      }
      if (t >= 0 && t <= 15) {
        for (int q = kThreads - 1 - tid; q < kF2 + kG2; q += kThreads) {
          if (q < kF2) {
            const int i = q % 17 - 1, y = q / 17;
            const int l = (y + 1) * 18 + (i + 1);
            V5<T> F = riemann<RS>(lds5(sWX + 5 * kSQ, kSQ, l), lds5(sWX, kSQ, l + 1), ph, &fails);
            sts5(sF2, kF2, q, from_frame<0>(F));
          } else {
            const int r = q - kF2;
            const int x = r % 16, j = r / 16 - 1;
            const int l = (j + 1) * 18 + (x + 1);
            V5<T> F = riemann<RS>(lds5(sWY + 5 * kSQ, kSQ, l), lds5(sWY, kSQ, l + 18), ph, &fails);
            sts5(sG2, kG2, r, from_frame<1>(F));
          }
        }
      }
      __syncthreads();

      // ---- F: update plane t-1; flux differences of plane t; face fluxes ---
      if (interior) {
        const int x = col.x, y = col.y;
        if (t >= 1) {
          V5<T> u = ucons(t - 1);
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
          const int fi = f == 0 ? -1 : (f == 1 ? 15 : 7);
          V5<T> v = d == 0 ? lds5(sF2, kF2, s * 17 + fi + 1) : lds5(sG2, kG2, (fi + 1) * 16 + s);
#pragma unroll
          for (int n = 0; n < 5; ++n) FO[((d * a.nf + f) * 5 + n) * 256 + t * 16 + s] = v[n];
        }
      }
    }
    __syncthreads();
  }
  flush_diag(a, fails, floors);
}

}  // namespace muscl
}  // namespace hy
