// Plain per-patch-group solver: the paper's own GPU design (Sec. 3.1) on
// gfx950, kept as the baseline path.
//
//  * one workgroup per patch group (a grid-stride loop over groups);
//  * every stage is a flattened 1D loop over the cells of its range with
//    integer div/mod index recovery, as the paper describes (Sec. 3.1);
//  * intermediates (primitive variables, face states, fluxes) live in
//    per-workgroup global temporaries that never leave the device (Sec. 3.1);
//  * stages are separated by workgroup barriers.
// Each stage is computed on the range its stencil allows inside the padded
// group, so the interior 16^3 cells are exact for the ghost width chosen.
#include "hydro_internal.h"
#include "hydro_math.hpp"
#include "riemann_exact.hpp"

namespace hy {

struct Box3 {
  int lo[3], hi[3];
};
HY_DEV Box3 box_full(int N) { return Box3{{0, 0, 0}, {N, N, N}}; }
HY_DEV Box3 box_shrink(Box3 b, int a, int rl, int rh) { b.lo[a] += rl; b.hi[a] -= rh; return b; }
HY_DEV Box3 box_and(Box3 a, const Box3& b) {
  for (int k = 0; k < 3; ++k) { a.lo[k] = max(a.lo[k], b.lo[k]); a.hi[k] = min(a.hi[k], b.hi[k]); }
  return a;
}

// Flattened loop over a box (Sec. 3.1: count/blocksize with div and mod).
template <typename F> HY_DEV void plain_for(const Box3& b, F&& body) {
  const int nx = b.hi[0] - b.lo[0], ny = b.hi[1] - b.lo[1], nz = b.hi[2] - b.lo[2];
  const int tot = (nx > 0 && ny > 0 && nz > 0) ? nx * ny * nz : 0;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    const int i = b.lo[0] + t % nx;
    const int j = b.lo[1] + (t / nx) % ny;
    const int k = b.lo[2] + t / (nx * ny);
    body(i, j, k);
  }
}

template <typename T>
struct PlainCtx {
  int N;
  long nc;        // N^3
  T* W;           // [5][nc] primitive (VL: overwritten by the half-step state)
  T* Wm[3];       // [5][nc] left-face state of each cell, lab frame
  T* Wp[3];       // [5][nc] right-face state
  T* F[3];        // [5][nc] flux at face i+1/2 stored at i, lab frame
  int roe_fb_exact;
  HY_DEV long at(int i, int j, int k) const { return ((long)k * N + j) * N + i; }
};

// Riemann solver of the plain path: RS = 3 is the exact solver; with
// roe_fb_exact a face where the Roe linearization fails (counted in *fails)
// takes the exact flux instead of the HLLE/HLLC fallback.
template <int RS, typename T>
HY_DEV V5<T> plain_solve(const V5<T>& L, const V5<T>& R, const Phys<T>& ph, int roe_fb_exact, int* fails) {
  if constexpr (RS == 3) {
    return exact_flux(L, R, ph, fails);
  } else if constexpr (RS == 0) {
    int f = 0;
    V5<T> F = riemann<0>(L, R, ph, &f);
    if (f) {
      *fails += f;
      if (roe_fb_exact) {
        int ignored = 0;
        F = exact_flux(L, R, ph, &ignored);
      }
    }
    return F;
  } else {
    return riemann<RS>(L, R, ph, fails);
  }
}

template <typename T> HY_DEV V5<T> ld(const T* a, long nc, long q) {
  V5<T> v;
#pragma unroll
  for (int n = 0; n < 5; ++n) v[n] = a[n * nc + q];
  return v;
}
template <typename T> HY_DEV void st(T* a, long nc, long q, const V5<T>& v) {
#pragma unroll
  for (int n = 0; n < 5; ++n) a[n * nc + q] = v[n];
}

template <int D> HY_DEV long dstride(int N) { return D == 0 ? 1 : (D == 1 ? N : (long)N * N); }

// Step (1): face states along D from the primitive field Wsrc valid on wr.
template <int D, bool PPM, bool TRACE, typename T>
HY_DEV Box3 plain_faces(const PlainCtx<T>& c, const T* Wsrc, Box3 wr, const Phys<T>& ph, int* floors) {
  Box3 fr = box_shrink(wr, D, PPM ? 2 : 1, PPM ? 2 : 1);
  const long s = dstride<D>(c.N);
  plain_for(fr, [&](int i, int j, int k) {
    const long q = c.at(i, j, k);
    V5<T> w0 = to_frame<D>(ld(Wsrc, c.nc, q));
    V5<T> wm = to_frame<D>(ld(Wsrc, c.nc, q - s));
    V5<T> wp = to_frame<D>(ld(Wsrc, c.nc, q + s));
    V5<T> fl, fr2;
    if (PPM) {
      V5<T> wmm = to_frame<D>(ld(Wsrc, c.nc, q - 2 * s));
      V5<T> wpp = to_frame<D>(ld(Wsrc, c.nc, q + 2 * s));
      V5<T> sm = slope<PPM>(wmm, wm, w0, ph), s0 = slope<PPM>(wm, w0, wp, ph), sp = slope<PPM>(w0, wp, wpp, ph);
      fl = ppm_edge(wm, w0, sm, s0);
      fr2 = ppm_edge(w0, wp, s0, sp);
      ppm_mono(w0, fl, fr2);
    } else {
      V5<T> s0 = slope<PPM>(wm, w0, wp, ph);
      plm_faces(wm, w0, wp, s0, ph, fl, fr2);
    }
    if (TRACE) ctu_trace<PPM>(w0, fl, fr2, ph);
    *floors += floor_state(fl, ph) + floor_state(fr2, ph);
    st(c.Wm[D], c.nc, q, from_frame<D>(fl));
    st(c.Wp[D], c.nc, q, from_frame<D>(fr2));
  });
  return fr;
}

// Step (2): Riemann solves along D between the right state of cell i (SL)
// and the left state of cell i+1 (SR) for cells in cr.
template <int D, int RS, typename T>
HY_DEV Box3 plain_riemann(const PlainCtx<T>& c, const T* SL, const T* SR, Box3 cr, const Phys<T>& ph, int* fails) {
  Box3 fb = box_shrink(cr, D, 0, 1);
  const long s = dstride<D>(c.N);
  plain_for(fb, [&](int i, int j, int k) {
    const long q = c.at(i, j, k);
    V5<T> L = to_frame<D>(ld(SL, c.nc, q));
    V5<T> R = to_frame<D>(ld(SR, c.nc, q + s));
    st(c.F[D], c.nc, q, from_frame<D>(plain_solve<RS>(L, R, ph, c.roe_fb_exact, fails)));
  });
  return fb;
}

template <int D, typename T> HY_DEV V5<T> dflux(const PlainCtx<T>& c, long q) {
  V5<T> a = ld(c.F[D], c.nc, q), b = ld(c.F[D], c.nc, q - dstride<D>(c.N));
  V5<T> r;
#pragma unroll
  for (int n = 0; n < 5; ++n) r[n] = a[n] - b[n];
  return r;
}
HY_DEV Box3 diff_box(Box3 fb, int d) { return box_shrink(fb, d, 1, 0); }

// CTU step (3): correct both face states of direction D of every cell in cr
// by -dt/(2dh) times the two transverse first-set flux differences at that
// cell, in conserved variables; then back to primitive with floors.
template <int E1, int E2, int D, typename T>
HY_DEV void ctu_correct(const PlainCtx<T>& c, const T* U, Box3 cr, const Phys<T>& ph, int* floors) {
  const long nc = c.nc;
  plain_for(cr, [&](int i, int j, int k) {
    const long q = c.at(i, j, k);
    V5<T> t1 = dflux<E1>(c, q), t2 = dflux<E2>(c, q);
    V5<T> um = cons_of(ld(c.Wm[D], nc, q), ph), up = cons_of(ld(c.Wp[D], nc, q), ph);
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      T t = ph.hdtdh * (t1[n] + t2[n]);
      um[n] -= t;
      up[n] -= t;
    }
    V5<T> wm = prim_of(um, ph), wp = prim_of(up, ph);
    *floors += floor_state(wm, ph) + floor_state(wp, ph);
    st(c.Wm[D], nc, q, wm);
    st(c.Wp[D], nc, q, wp);
  });
}

template <typename T, int SCHEME, bool PPM, int RS>
__global__ void __launch_bounds__(256) plain_kernel(PlainArgs<T> a) {
  const int N = a.N, g = a.g;
  const long nc = (long)N * N * N;
  PlainCtx<T> c;
  c.N = N;
  c.nc = nc;
  c.roe_fb_exact = a.roe_fb_exact;
  T* base = a.ws + (long)blockIdx.x * a.ws_stride;
  c.W = base;
  for (int d = 0; d < 3; ++d) {
    c.Wm[d] = base + (5 + 10 * d) * nc;
    c.Wp[d] = base + (10 + 10 * d) * nc;
    c.F[d] = base + (35 + 5 * d) * nc;
  }
  const Phys<T>& ph = a.ph;
  int fails = 0, floors = 0;

  for (long grp = blockIdx.x; grp < a.n_groups; grp += gridDim.x) {
    const T* U = a.in + grp * 5 * nc;
    Box3 all = box_full(N);
    plain_for(all, [&](int i, int j, int k) {
      const long q = c.at(i, j, k);
      st(c.W, nc, q, prim_of(ld(U, nc, q), ph));
    });
    __syncthreads();

    Box3 fb[3];
    if (SCHEME == 0) {  // MHM
      Box3 sr0 = plain_faces<0, PPM, false>(c, c.W, all, ph, &floors);
      Box3 sr1 = plain_faces<1, PPM, false>(c, c.W, all, ph, &floors);
      Box3 sr2 = plain_faces<2, PPM, false>(c, c.W, all, ph, &floors);
      __syncthreads();
      Box3 hr = box_and(box_and(sr0, sr1), sr2);
      // Hancock half step: one cell-centred dU from the six face fluxes.
      plain_for(hr, [&](int i, int j, int k) {
        const long q = c.at(i, j, k);
        V5<T> dU;
#pragma unroll
        for (int n = 0; n < 5; ++n) dU[n] = T(0);
        {
          V5<T> Fp = from_frame<0>(flux_of(to_frame<0>(ld(c.Wp[0], nc, q)), ph));
          V5<T> Fm = from_frame<0>(flux_of(to_frame<0>(ld(c.Wm[0], nc, q)), ph));
#pragma unroll
          for (int n = 0; n < 5; ++n) dU[n] += Fp[n] - Fm[n];
        }
        {
          V5<T> Fp = from_frame<1>(flux_of(to_frame<1>(ld(c.Wp[1], nc, q)), ph));
          V5<T> Fm = from_frame<1>(flux_of(to_frame<1>(ld(c.Wm[1], nc, q)), ph));
#pragma unroll
          for (int n = 0; n < 5; ++n) dU[n] += Fp[n] - Fm[n];
        }
        {
          V5<T> Fp = from_frame<2>(flux_of(to_frame<2>(ld(c.Wp[2], nc, q)), ph));
          V5<T> Fm = from_frame<2>(flux_of(to_frame<2>(ld(c.Wm[2], nc, q)), ph));
#pragma unroll
          for (int n = 0; n < 5; ++n) dU[n] += Fp[n] - Fm[n];
        }
        for (int d = 0; d < 3; ++d) {
          T* pm = c.Wm[d];
          T* pp = c.Wp[d];
          V5<T> um = cons_of(ld(pm, nc, q), ph), up = cons_of(ld(pp, nc, q), ph);
#pragma unroll
          for (int n = 0; n < 5; ++n) { um[n] -= ph.hdtdh * dU[n]; up[n] -= ph.hdtdh * dU[n]; }
          V5<T> wm = prim_of(um, ph), wp = prim_of(up, ph);
          floors += floor_state(wm, ph) + floor_state(wp, ph);
          st(pm, nc, q, wm);
          st(pp, nc, q, wp);
        }
      });
      __syncthreads();
      fb[0] = plain_riemann<0, RS>(c, c.Wp[0], c.Wm[0], hr, ph, &fails);
      fb[1] = plain_riemann<1, RS>(c, c.Wp[1], c.Wm[1], hr, ph, &fails);
      fb[2] = plain_riemann<2, RS>(c, c.Wp[2], c.Wm[2], hr, ph, &fails);
    } else if (SCHEME == 1) {  // VL
      Box3 f0 = plain_riemann<0, RS>(c, c.W, c.W, all, ph, &fails);
      Box3 f1 = plain_riemann<1, RS>(c, c.W, c.W, all, ph, &fails);
      Box3 f2 = plain_riemann<2, RS>(c, c.W, c.W, all, ph, &fails);
      __syncthreads();
      Box3 hr = box_and(box_and(diff_box(f0, 0), diff_box(f1, 1)), diff_box(f2, 2));
      plain_for(hr, [&](int i, int j, int k) {
        const long q = c.at(i, j, k);
        V5<T> dx = dflux<0>(c, q), dy = dflux<1>(c, q), dz = dflux<2>(c, q);
        V5<T> u = ld(U, nc, q);
#pragma unroll
        for (int n = 0; n < 5; ++n) u[n] -= ph.hdtdh * (dx[n] + dy[n] + dz[n]);
        V5<T> w = prim_of(u, ph);
        floors += floor_state(w, ph);
        st(c.W, nc, q, w);  // W now holds the half-step state on hr
      });
      __syncthreads();
      Box3 sr0 = plain_faces<0, PPM, false>(c, c.W, hr, ph, &floors);
      Box3 sr1 = plain_faces<1, PPM, false>(c, c.W, hr, ph, &floors);
      Box3 sr2 = plain_faces<2, PPM, false>(c, c.W, hr, ph, &floors);
      __syncthreads();
      fb[0] = plain_riemann<0, RS>(c, c.Wp[0], c.Wm[0], sr0, ph, &fails);
      fb[1] = plain_riemann<1, RS>(c, c.Wp[1], c.Wm[1], sr1, ph, &fails);
      fb[2] = plain_riemann<2, RS>(c, c.Wp[2], c.Wm[2], sr2, ph, &fails);
    } else {  // CTU
      Box3 sr[3];
      sr[0] = plain_faces<0, PPM, true>(c, c.W, all, ph, &floors);
      sr[1] = plain_faces<1, PPM, true>(c, c.W, all, ph, &floors);
      sr[2] = plain_faces<2, PPM, true>(c, c.W, all, ph, &floors);
      __syncthreads();
      Box3 f1[3];
      f1[0] = plain_riemann<0, RS>(c, c.Wp[0], c.Wm[0], sr[0], ph, &fails);
      f1[1] = plain_riemann<1, RS>(c, c.Wp[1], c.Wm[1], sr[1], ph, &fails);
      f1[2] = plain_riemann<2, RS>(c, c.Wp[2], c.Wm[2], sr[2], ph, &fails);
      __syncthreads();
      // Transverse flux-gradient correction in conserved variables.
      Box3 cr[3];
      for (int d = 0; d < 3; ++d) {
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        cr[d] = box_and(box_and(sr[d], diff_box(f1[e1], e1)), diff_box(f1[e2], e2));
      }
      ctu_correct<1, 2, 0>(c, U, cr[0], ph, &floors);
      ctu_correct<2, 0, 1>(c, U, cr[1], ph, &floors);
      ctu_correct<0, 1, 2>(c, U, cr[2], ph, &floors);
      __syncthreads();
      fb[0] = plain_riemann<0, RS>(c, c.Wp[0], c.Wm[0], cr[0], ph, &fails);
      fb[1] = plain_riemann<1, RS>(c, c.Wp[1], c.Wm[1], cr[1], ph, &fails);
      fb[2] = plain_riemann<2, RS>(c, c.Wp[2], c.Wm[2], cr[2], ph, &fails);
    }
    __syncthreads();

    // Step (4): conservative update of the interior; step (5): fluxes on the
    // group's faces (and optionally the internal patch mid planes).
    T* O = a.out + grp * 5 * 4096;
    Box3 in = Box3{{g, g, g}, {g + 16, g + 16, g + 16}};
    plain_for(in, [&](int i, int j, int k) {
      const long q = c.at(i, j, k);
      V5<T> dx = dflux<0>(c, q), dy = dflux<1>(c, q), dz = dflux<2>(c, q);
      V5<T> u = ld(U, nc, q);
      const int o = ((k - g) * 16 + (j - g)) * 16 + (i - g);
#pragma unroll
      for (int n = 0; n < 5; ++n) O[n * 4096 + o] = u[n] - ph.dtdh * (dx[n] + dy[n] + dz[n]);
    });
    if (a.flux) {
      T* FO = a.flux + grp * 3 * a.nf * 5 * 256;
      const int total = 3 * a.nf * 256;
      for (int t = threadIdx.x; t < total; t += blockDim.x) {
        const int b = t % 16, s = (t / 16) % 16, f = (t / 256) % a.nf, d = t / (256 * a.nf);
        const int off = (f == 0) ? 0 : (f == 1 ? 16 : 8);
        const int fi = g + off - 1;
        long q;
        if (d == 0) q = c.at(fi, b + g, s + g);
        else if (d == 1) q = c.at(b + g, fi, s + g);
        else q = c.at(b + g, s + g, fi);
#pragma unroll
        for (int n = 0; n < 5; ++n) FO[((d * a.nf + f) * 5 + n) * 256 + s * 16 + b] = c.F[d][n * nc + q];
      }
    }
    __syncthreads();
  }
  if (a.diag) {
    if (fails) atomicAdd(&a.diag[0], (unsigned long long)fails);
    if (floors) atomicAdd(&a.diag[1], (unsigned long long)floors);
  }
}

template <typename T>
hipError_t launch_plain_t(const PlainArgs<T>& a, int scheme, int recon, int riemann, int grid, hipStream_t st) {
  dim3 blk(256), grd(grid);
#define PL(S, P, R) \
  if (scheme == S && recon == P && riemann == R) { plain_kernel<T, S, P == 1, R><<<grd, blk, 0, st>>>(a); return hipGetLastError(); }
#define PLR(S, P) PL(S, P, 0) PL(S, P, 1) PL(S, P, 2) PL(S, P, 3)
  PLR(0, 0) PLR(0, 1) PLR(1, 0) PLR(1, 1) PLR(2, 0) PLR(2, 1)
#undef PLR
#undef PL
  return hipErrorInvalidValue;
}

hipError_t launch_plain(const PlainArgs<float>& a, int s, int p, int r, int grid, hipStream_t st) {
  return launch_plain_t(a, s, p, r, grid, st);
}
hipError_t launch_plain(const PlainArgs<double>& a, int s, int p, int r, int grid, hipStream_t st) {
  return launch_plain_t(a, s, p, r, grid, st);
}

}  // namespace hy
