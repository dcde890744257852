// First stage of the VL scheme (arXiv:1103.3373, Sec. 2): Riemann fluxes on
// piecewise-constant data at every face, then the unsplit half step
//   W* = W(U^n - dt/(2dh) sum_d (F1_{d,+} - F1_{d,-}))   (with floors)
// on every cell that the second stage reconstructs from.  Two layouts:
//  * ghosted groups (input ghost width G = g of the scheme): the interior
//    plus G-1 ghost layers, [group][5][N'][N'][N'], N' = 16 + 2(G-1);
//  * periodic boxes (G = 1): the interior only, [group][5][16][16][16], so
//    every cell's W* is computed once and the second stage reads its ghost
//    cells from the neighbouring groups of this grouped box.
//
// One workgroup per group marching along z; a thread per (x, y) column of
// the padded input plane keeps U and W of planes z, z+1 and the z face flux
// below in registers; x and y face fluxes of the plane go through LDS, each
// computed once.  Two barriers per plane.
#pragma once

#include "fused_common.hpp"

namespace hy {
namespace vlpred {

using namespace fz;

// Threads per workgroup.  Ghosted groups: one per column of the padded input
// plane, rounded up to wavefronts.  Periodic boxes (G = 1): the faces of the
// interior read only the interior columns and the one-cell ring beside its
// four sides (not the four corner columns), so 320 threads: the interior
// first (tid 0..255), then the ring.
template <int G> constexpr int threads() { return G == 1 ? 320 : ((16 + 2 * G) * (16 + 2 * G) + 63) / 64 * 64; }

template <typename T, int G, int RS>
__global__ void __launch_bounds__(threads<G>(), 2) vl_predict_kernel(FusedArgs<T> a) {
  constexpr int kThreads = threads<G>();
  constexpr int N = 16 + 2 * G;   // G: input ghost width
  constexpr int Gs = G - 1;        // output ghost width
  constexpr int Ns = 16 + 2 * Gs;
  constexpr long NCs = (long)Ns * Ns * Ns;
  constexpr int nF = (N - 1) * Ns;  // x faces between x = i and i+1, i in -G .. 14+G; rows -Gs .. 15+Gs
  extern __shared__ unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  T* sP = sm;                       // [5][N*N]
  T* sFX = sP + 5 * N * N;          // [5][nF]   index (y + Gs) * (N - 1) + (i + G)
  T* sFY = sFX + 5 * nF;            // [5][nF]   index (j + G) * Ns + (x + Gs)

  const int tid = threadIdx.x;
  int x, y;
  bool active, out_col;
  if constexpr (G == 1) {
    if (tid < 256) {
      x = tid & 15;
      y = tid >> 4;
    } else {  // the ring: x = -1, x = 16, y = -1, y = 16, 16 columns each
      const int q = tid - 256, s = q & 15, side = q >> 4;
      x = side == 0 ? -1 : (side == 1 ? 16 : s);
      y = side == 2 ? -1 : (side == 3 ? 16 : s);
    }
    active = true;
    out_col = uni(tid & ~63) < 256;  // waves 0-3: wave-uniform
  } else {
    active = tid < N * N;
    x = tid % N - G;
    y = tid / N - G;
    out_col = active && x >= -Gs && x <= 15 + Gs && y >= -Gs && y <= 15 + Gs;
  }
  const int pc = (y + G) * N + (x + G);  // the column's cell in the plane
  // byte offset of the column's cell in a half-step plane (output columns)
  const unsigned wo = out_col ? (unsigned)(((y + Gs) * Ns + (x + Gs)) * (int)sizeof(T)) : 0u;
  int fails = 0, floors = 0;
  Phys<T> ph = make_phys(a);

  int seg = 0;
  const GroupOrder order = group_order(a.n_groups);
  for (long long grp = order.first; grp < order.end; grp += order.stride) {
    double dt;
    const USeg S = find_seg(a, grp, seg, dt);
    const long long lg = grp - S.first;
    // A box segment beyond the addressing limit: a NaN dt/dh makes every
    // half-step state NaN.
    const T poison = slab_fits<T>(S) ? T(0) : T(__builtin_nan(""));
    ph.dtdh = (T)(dt / S.dh) + poison;
    ph.hdtdh = (T)(0.5 * dt / S.dh) + poison;
    ColumnReader<T, G> rd;
    rd.init(S, lg, active ? x : 0, active ? y : 0);
    T* __restrict__ Wo = a.wstar + grp * 5 * NCs;  // the group's half-step array (uniform)

    V5<T> u0, w0, u1, w1, hm, unext;
    if (active) {
      u0 = rd.load(-Gs - 1);
      w0 = prim_of(u0, ph);
      u1 = rd.load(-Gs);
      w1 = prim_of(u1, ph);
      if (out_col) hm = from_frame<2>(riemann<RS>(to_frame<2>(w0), to_frame<2>(w1), ph, &fails));
      u0 = u1;
      w0 = w1;
      unext = rd.load(-Gs + 1);
    }
    for (int z = -Gs; z <= 15 + Gs; ++z) {
      // ---- A: plane z to LDS; z flux above the column's cell.  The column's
      //         plane z+1 was loaded one plane ahead; plane z+2 is requested
      //         now and arrives while phases B and C run --------------------
      V5<T> hp;
      if (active) {
        sts5(sP, N * N, pc, w0);
        u1 = unext;
        unext = rd.load(z + 2 <= 16 + Gs ? z + 2 : 16 + Gs);  // clamped on the last plane
        w1 = prim_of(u1, ph);
        if (out_col) hp = from_frame<2>(riemann<RS>(to_frame<2>(w0), to_frame<2>(w1), ph, &fails));
      }
      __syncthreads();
      // ---- B: x and y face fluxes of plane z --------------------------------
      for (int q = tid; q < 2 * nF; q += kThreads) {
        if (q < nF) {
          const int i = q % (N - 1) - G, r = q / (N - 1) - Gs;  // face between i and i+1, row r
          const int c = (r + G) * N + (i + G);
          V5<T> F = riemann<RS>(to_frame<0>(lds5(sP, N * N, c)), to_frame<0>(lds5(sP, N * N, c + 1)), ph, &fails);
          sts5(sFX, nF, q, from_frame<0>(F));
        } else {
          const int qq = q - nF;
          const int cx = qq % Ns - Gs, j = qq / Ns - G;  // face between j and j+1, column cx
          const int c = (j + G) * N + (cx + G);
          V5<T> F = riemann<RS>(to_frame<1>(lds5(sP, N * N, c)), to_frame<1>(lds5(sP, N * N, c + N)), ph, &fails);
          sts5(sFY, nF, qq, from_frame<1>(F));
        }
      }
      __syncthreads();
      // ---- C: half-step state of the column's cell --------------------------
      if (out_col) {
        const int fx = (y + Gs) * (N - 1) + (x + G);   // face x+1/2; x-1/2 is fx - 1
        const int fy = (y + G) * Ns + (x + Gs);        // face y+1/2; y-1/2 is fy - Ns
        V5<T> dx = sub5(lds5(sFX, nF, fx), lds5(sFX, nF, fx - 1));
        V5<T> dy = sub5(lds5(sFY, nF, fy), lds5(sFY, nF, fy - Ns));
        V5<T> u = u0;
#pragma unroll
        for (int n = 0; n < 5; ++n) u[n] -= ph.hdtdh * (dx[n] + dy[n] + (hp[n] - hm[n]));
        V5<T> w = prim_of(u, ph);
        floors += floor_state(w, ph);
        T* o = Wo + (long)(z + Gs) * Ns * Ns;
#pragma unroll
        for (int n = 0; n < 5; ++n) gstore(o + n * NCs, wo, w[n]);
        hm = hp;
      }
      if (active) {
        u0 = u1;
        w0 = w1;
      }
    }
    __syncthreads();
  }
  flush_diag(a, fails, floors);
}

template <int G> constexpr int lds_elems() {
  constexpr int N = 16 + 2 * G;
  constexpr int Ns = 16 + 2 * (G - 1);
  return 5 * N * N + 10 * (N - 1) * Ns;
}

}  // namespace vlpred
}  // namespace hy
