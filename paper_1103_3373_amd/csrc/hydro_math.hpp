// Device-side building blocks of the unsplit schemes (arXiv:1103.3373, Sec. 2):
// ideal-gas relations, physical fluxes, slope limiters, primitive and
// characteristic limiting, PLM / PPM face values, CTU characteristic tracing,
// and the Roe (with positivity fallback), HLLC and HLLE Riemann solvers.
//
// All functions are templated on the arithmetic type T (float or double) and
// work on 5-component states held in registers (the paper's Sec. 3.1 advice:
// small structs, force-inlined).  A state in "frame d" has its velocity
// components cyclically rotated so that component 1 is normal to direction d:
// x -> (u, v, w), y -> (v, w, u), z -> (w, u, v).  Direction d is always a
// template parameter so that no register array is indexed at run time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HY_DEV __device__ __forceinline__

namespace hy {

template <typename T>
struct V5 {
  T q[5];
  HY_DEV T& operator[](int i) { return q[i]; }
  HY_DEV const T& operator[](int i) const { return q[i]; }
};

// Per-launch constants.  dt/dh and dt/(2dh) are formed in double on the host
// and rounded once to T.
template <typename T>
struct Phys {
  T gamma, gm1, inv_gm1, dtdh, hdtdh, theta, floor;
  int limiter;
  int charlim;
  int roe_fb_hllc;
};

// ---- scalar helpers ---------------------------------------------------------
// min / max map to single v_min / v_max instructions (operands are never NaN).
HY_DEV float vmin(float a, float b) { return __builtin_fminf(a, b); }
HY_DEV double vmin(double a, double b) { return __builtin_fmin(a, b); }
HY_DEV float vmax(float a, float b) { return __builtin_fmaxf(a, b); }
HY_DEV double vmax(double a, double b) { return __builtin_fmax(a, b); }
HY_DEV float vsign_of(float m, float s) { return __builtin_copysignf(m, s); }
HY_DEV double vsign_of(double m, double s) { return __builtin_copysign(m, s); }
HY_DEV float vabs(float a) { return __builtin_fabsf(a); }
HY_DEV double vabs(double a) { return __builtin_fabs(a); }
// Median of three: one v_med3_f32 in FP32; FP64 (no such instruction)
// composes it from min and max.
HY_DEV float vmed3(float a, float b, float c) { return __builtin_amdgcn_fmed3f(a, b, c); }
HY_DEV double vmed3(double a, double b, double c) { return vmax(vmin(a, b), vmin(vmax(a, b), c)); }
// FP32 uses the hardware reciprocal and square root (about 1 ulp) instead
// of the multi-instruction correctly rounded sequences; FP64 stays IEEE.
HY_DEV float vsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
HY_DEV double vsqrt(double a) { return __builtin_sqrt(a); }
HY_DEV float vrcp(float a) { return __builtin_amdgcn_rcpf(a); }
HY_DEV double vrcp(double a) { return 1.0 / a; }
HY_DEV float vdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
HY_DEV double vdiv(double a, double b) { return a / b; }
// 1/sqrt(a): one transcendental in FP32 instead of a square root and a
// reciprocal.  The FP32 kernels use it to share 1/sqrt(rho) and 1/c between
// the quantities that need them; FP64 keeps the square roots and quotients
// in the order of their definitions.
HY_DEV float vrsq(float a) { return __builtin_amdgcn_rsqf(a); }
HY_DEV double vrsq(double a) { return 1.0 / __builtin_sqrt(a); }
template <typename T> struct FastMath { static constexpr bool on = false; };
template <> struct FastMath<float> { static constexpr bool on = true; };

// ---- frames -----------------------------------------------------------------
template <int D> struct Frame {
  static constexpr int n = 1 + D;
  static constexpr int t1 = 1 + (D + 1) % 3;
  static constexpr int t2 = 1 + (D + 2) % 3;
};
template <int D, typename T> HY_DEV V5<T> to_frame(const V5<T>& a) {
  V5<T> r;
  r[0] = a[0]; r[1] = a[Frame<D>::n]; r[2] = a[Frame<D>::t1]; r[3] = a[Frame<D>::t2]; r[4] = a[4];
  return r;
}
template <int D, typename T> HY_DEV V5<T> from_frame(const V5<T>& a) {
  V5<T> r;
  r[0] = a[0]; r[Frame<D>::n] = a[1]; r[Frame<D>::t1] = a[2]; r[Frame<D>::t2] = a[3]; r[4] = a[4];
  return r;
}

// ---- ideal gas --------------------------------------------------------------
template <typename T> HY_DEV V5<T> prim_of(const V5<T>& U, const Phys<T>& ph) {
  V5<T> W;
  T ir = vrcp(U[0]);
  W[0] = U[0];
  W[1] = U[1] * ir;
  W[2] = U[2] * ir;
  W[3] = U[3] * ir;
  W[4] = ph.gm1 * (U[4] - T(0.5) * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3]));
  return W;
}
template <typename T> HY_DEV V5<T> cons_of(const V5<T>& W, const Phys<T>& ph) {
  V5<T> U;
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  U[4] = W[4] * ph.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  return U;
}
// Physical flux normal to the frame (component 1 normal).
template <typename T> HY_DEV V5<T> flux_of(const V5<T>& W, const Phys<T>& ph) {
  V5<T> F;
  T E = W[4] * ph.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  F[0] = W[0] * W[1];
  F[1] = F[0] * W[1] + W[4];
  F[2] = F[0] * W[2];
  F[3] = F[0] * W[3];
  F[4] = W[1] * (E + W[4]);
  return F;
}
template <typename T> HY_DEV T sound(const V5<T>& W, const Phys<T>& ph) {
  return vsqrt(ph.gamma * W[4] * vrcp(W[0]));
}
// Sound speed c and 1/c of a state whose 1/rho is known.
template <typename T> HY_DEV void sound_pair(const V5<T>& W, T ir, const Phys<T>& ph, T& c, T& ic) {
  const T c2 = ph.gamma * W[4] * ir;
  if constexpr (FastMath<T>::on) {
    ic = vrsq(c2);
    c = c2 * ic;
  } else {
    c = vsqrt(c2);
    ic = vrcp(c);
  }
}
// Floor on density and pressure of face / half-step states; returns hits.
template <typename T> HY_DEV int floor_state(V5<T>& W, const Phys<T>& ph) {
  int h = 0;
  if (W[0] < ph.floor) { W[0] = ph.floor; ++h; }
  if (W[4] < ph.floor) { W[4] = ph.floor; ++h; }
  return h;
}

// The same floors with the hits counted for the whole wavefront: the compare
// masks of the active lanes are popcounted by scalar instructions, so the
// per-lane cost is the clamp's two compares and two selects.  Returns the
// wavefront's number of hits (uniform across its lanes).
template <typename T> HY_DEV unsigned floor_wave(V5<T>& W, const Phys<T>& ph) {
  const bool l0 = W[0] < ph.floor, l4 = W[4] < ph.floor;
  W[0] = l0 ? ph.floor : W[0];
  W[4] = l4 ? ph.floor : W[4];
  return (unsigned)(__builtin_popcountll(__builtin_amdgcn_ballot_w64(l0)) +
                    __builtin_popcountll(__builtin_amdgcn_ballot_w64(l4)));
}

// ---- limiters -----------------------------------------------------------------
// 0 generalized minmod (theta), 1 van Leer, 2 van Albada, 3 hybrid (van Leer
// bounded by generalized minmod).  Zero at extrema.  The result is scaled by
// ks (1 unless the caller carries its slopes scaled).
template <typename T> HY_DEV T limit(T dl, T dr, const Phys<T>& ph, T ks = T(1)) {
  T prod = dl * dr;
  if (!(prod > T(0))) return T(0);
  T dc = T(0.5) * (dl + dr);
  T r;
  switch (ph.limiter) {
    case 0: {
      T m = vmin(vmin(ph.theta * vabs(dl), ph.theta * vabs(dr)), vabs(dc));
      r = vsign_of(m, dc) * ks;  // dc != 0 because dl and dr share a sign
      break;
    }
    case 1: r = vdiv((T(2) * ks) * prod, dl + dr); break;
    case 2: r = vdiv(prod * (dl + dr), dl * dl + dr * dr) * ks; break;
    default: {
      T vl = vabs(vdiv(T(2) * prod, dl + dr));
      T m = vmin(vmin(vmin(ph.theta * vabs(dl), ph.theta * vabs(dr)), vabs(dc)), vl);
      r = vsign_of(m, dc) * ks;
      break;
    }
  }
  return r;
}

// Characteristic projection a = L dw and expansion dw = R a at a frame
// state W with sound speed c (waves u-c, u, u, u, u+c).
template <typename T> HY_DEV V5<T> char_L(const V5<T>& W, T c, T ic, T ic2, const V5<T>& dw) {
  V5<T> a;
  T rc = T(0.5) * W[0] * ic;
  if constexpr (FastMath<T>::on) {
    // FP32: the density wave from the acoustic term (dw0 - dp/c^2 = dw0 - 2 pc)
    T pc = dw[4] * (T(0.5) * ic2);
    a[0] = pc - rc * dw[1];
    a[1] = dw[0] - T(2) * pc;
    a[4] = pc + rc * dw[1];
  } else {
    T pc = T(0.5) * dw[4] * ic2;
    a[0] = pc - rc * dw[1];
    a[1] = dw[0] - dw[4] * ic2;
    a[4] = pc + rc * dw[1];
  }
  a[2] = dw[2];
  a[3] = dw[3];
  return a;
}
template <typename T> HY_DEV V5<T> char_R(const V5<T>& W, T c, T ir, const V5<T>& a) {
  V5<T> dw;
  dw[0] = a[0] + a[1] + a[4];
  dw[1] = c * ir * (a[4] - a[0]);
  dw[2] = a[2];
  dw[3] = a[3];
  dw[4] = c * c * (a[0] + a[4]);
  return dw;
}

// Limited slope of the middle cell (frame states).  PPM uses a slope only in
// the edge formula, divided by 6; in FP32 the slopes of PPM are carried
// already divided by 6 (SlopeScale::div6), which folds the division into the
// limiter's own multiplication (van Leer's factor 2 becomes 1/3) and saves
// an operation per component and edge.  FP64 and PLM carry the slope.
template <bool PPM, typename T> struct SlopeScale {
  static constexpr bool div6 = PPM && FastMath<T>::on;
};
template <bool PPM, typename T>
HY_DEV V5<T> slope(const V5<T>& wm, const V5<T>& w0, const V5<T>& wp, const Phys<T>& ph) {
  const T ks = SlopeScale<PPM, T>::div6 ? T(1) / T(6) : T(1);
  V5<T> dl, dr, s;
#pragma unroll
  for (int n = 0; n < 5; ++n) { dl[n] = w0[n] - wm[n]; dr[n] = wp[n] - w0[n]; }
  if (!ph.charlim) {
#pragma unroll
    for (int n = 0; n < 5; ++n) s[n] = limit(dl[n], dr[n], ph, ks);
    return s;
  }
  T ir = vrcp(w0[0]);
  T c, ic;
  sound_pair(w0, ir, ph, c, ic);
  T ic2 = ic * ic;
  V5<T> al = char_L(w0, c, ic, ic2, dl);
  V5<T> ar = char_L(w0, c, ic, ic2, dr);
  V5<T> am;
#pragma unroll
  for (int n = 0; n < 5; ++n) am[n] = limit(al[n], ar[n], ph, ks);
  return char_R(w0, c, ir, am);
}

// PPM edge between cells a and b (states, limited slopes from slope<true>),
// clipped into the range of the two cell values: the median of the edge and
// the two values.
template <typename T>
HY_DEV V5<T> ppm_edge(const V5<T>& wa, const V5<T>& wb, const V5<T>& sa, const V5<T>& sb) {
  V5<T> e;
  const T sixth = T(1) / T(6);
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    T v;
    if constexpr (SlopeScale<true, T>::div6) v = T(0.5) * (wa[n] + wb[n]) + (sa[n] - sb[n]);  // slopes / 6
    else v = T(0.5) * (wa[n] + wb[n]) - (sb[n] - sa[n]) * sixth;
    e[n] = vmed3(v, wa[n], wb[n]);
  }
  return e;
}

// Parabola monotonization per component, in median form.  For a cell value
// a with edges l and r the three cases of the monotonization are:
//   local extremum ((r - a)(a - l) <= 0): both edges become a;
//   the left edge overshoots (the parabola has an extremum inside the cell
//     next to l): l becomes 3a - 2r; likewise r becomes 3a - 2l;
//   otherwise the edges stay.
// With dl = a - l and dr = r - a of one sign, the overshoot test
// 6 (r - l)(a - (l + r)/2) > (r - l)^2 reduces to |dl| > 2|dr|, and all
// three cases are l = med3(l, a, 3a - 2r), r = med3(r, a, 3a - 2l): a lies
// between the other two exactly at an extremum, and otherwise the median
// picks the edge or its replacement, whichever is nearer to a.  The forms
// coincide at every switching point.
template <typename T> HY_DEV void ppm_mono(const V5<T>& w, V5<T>& wl, V5<T>& wr) {
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    const T a = w[n], a3 = T(3) * a, l = wl[n], r = wr[n];
    wl[n] = vmed3(l, a, a3 - T(2) * r);
    wr[n] = vmed3(r, a, a3 - T(2) * l);
  }
}

// PLM face values from the limited slope; characteristic mode clips them
// between the cell value and its neighbour across each face.
template <typename T>
HY_DEV void plm_faces(const V5<T>& wm, const V5<T>& w, const V5<T>& wp, const V5<T>& s, const Phys<T>& ph,
                      V5<T>& fl, V5<T>& fr) {
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    fl[n] = w[n] - T(0.5) * s[n];
    fr[n] = w[n] + T(0.5) * s[n];
  }
  if (ph.charlim) {
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      fl[n] = vmed3(fl[n], w[n], wm[n]);
      fr[n] = vmed3(fr[n], w[n], wp[n]);
    }
  }
}

// CTU characteristic tracing to t+dt/2 with Colella's reference states.
// In: cell state w, face values fl (left face) and fr (right face); PPM adds
// the parabola term.  Out: fl = right state of the left face at the half
// step, fr = left state of the right face at the half step.
template <bool PPM, typename T>
HY_DEV void ctu_trace(const V5<T>& w, V5<T>& fl, V5<T>& fr, const Phys<T>& ph) {
  T ir = vrcp(w[0]);
  T c, ic;
  sound_pair(w, ir, ph, c, ic);
  T ic2 = ic * ic;
  const T two3 = T(2) / T(3);
  if constexpr (FastMath<T>::on) {
    // FP32: the reference-state extrapolation and the correction of the
    // waves that reach a face add up, wave by wave, to one coefficient.  With
    // sigma the wave's own speed when it reaches the face and the reference
    // speed (sM right, sm left) otherwise, the right face gets
    //   fr - R [sigma/2 (da - (1 - 2/3 sigma) a6)]
    // and the left face fl - R [sigma/2 (da + (1 + 2/3 sigma) a6)]: the same
    // states as the form below (R L = I), with one expansion per face.  The
    // speeds are formed as halves, h = sigma/2 = lambda dt/(2 dh); the
    // parabola amplitudes are projected as a sixth of themselves,
    // L (w - (fl + fr)/2), and their factors (6 - 8h, 6 + 8h) carry the 6.
    // The slowest wave reaches the left face only with its own speed or sm,
    // which is min(its speed, 0) = sm; likewise the fastest on the right.
    // (u -+ c) first: its sign decides the switch at lambda = 0 exactly.
    const T uh = w[1] * ph.hdtdh, h0 = (w[1] - c) * ph.hdtdh, h4 = (w[1] + c) * ph.hdtdh;
    const T hM = vmax(h4, T(0)), hm0 = vmin(h0, T(0));
    V5<T> dw, wc;
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      dw[n] = fr[n] - fl[n];
      wc[n] = PPM ? w[n] - T(0.5) * (fl[n] + fr[n]) : T(0);
    }
    const V5<T> da = char_L(w, c, ic, ic2, dw);
    V5<T> a6;
    if (PPM) a6 = char_L(w, c, ic, ic2, wc);
    T hp[3], gp[3], hm[3], gm[3];
    hp[0] = h0 > T(0) ? h0 : hM;
    hp[1] = uh > T(0) ? uh : hM;
    hp[2] = hM;
    hm[0] = hm0;
    hm[1] = uh < T(0) ? uh : hm0;
    hm[2] = h4 < T(0) ? h4 : hm0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gp[k] = T(6) - T(8) * hp[k];
      gm[k] = T(6) + T(8) * hm[k];
    }
    V5<T> cp, cm;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int k = a == 0 ? 0 : (a == 4 ? 2 : 1);
      cp[a] = hp[k] * (PPM ? da[a] - gp[k] * a6[a] : da[a]);
      cm[a] = hm[k] * (PPM ? da[a] + gm[k] * a6[a] : da[a]);
    }
    const V5<T> eR = char_R(w, c, ir, cp), eL = char_R(w, c, ir, cm);
#pragma unroll
    for (int n = 0; n < 5; ++n) {
      fr[n] -= eR[n];
      fl[n] -= eL[n];
    }
    return;
  }
  T s[5];
  s[0] = (w[1] - c) * ph.dtdh;
  s[1] = w[1] * ph.dtdh;
  s[4] = (w[1] + c) * ph.dtdh;
  T sM = vmax(s[4], T(0));
  T sm = vmin(s[0], T(0));
  V5<T> dw, w6;
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    dw[n] = fr[n] - fl[n];
    w6[n] = PPM ? T(6) * (w[n] - T(0.5) * (fl[n] + fr[n])) : T(0);
  }
  V5<T> da = char_L(w, c, ic, ic2, dw);
  V5<T> a6;
  if (PPM) a6 = char_L(w, c, ic, ic2, w6);
  V5<T> L, R;
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    T t6p = PPM ? (T(1) - two3 * sM) * w6[n] : T(0);
    T t6m = PPM ? (T(1) + two3 * sm) * w6[n] : T(0);
    L[n] = fr[n] - T(0.5) * sM * (dw[n] - t6p);
    R[n] = fl[n] - T(0.5) * sm * (dw[n] + t6m);
  }
  // Amplitudes of the waves that reach each face, relative to the reference.
  // A wave moving right (s > 0) reaches the right face only, with the
  // reference speed sM; one moving left reaches the left face, with sm.  So
  // each wave has one amplitude, formed with its own reference and routed
  // to its face; the three middle waves share the speed u and its factors.
  const T third = T(1) / T(3);
  V5<T> aL, aR;
  T sa[5] = {s[0], s[1], s[1], s[1], s[4]};
  T hk[3], qk[3], gk[3];  // per distinct speed: (sr - s)/2, (sr^2 - s^2)/3, -1 or +1
  {
    const T sk[3] = {s[0], s[1], s[4]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const bool pos = sk[k] > T(0);
      const T sr = pos ? sM : sm;
      hk[k] = T(0.5) * (sr - sk[k]);
      qk[k] = PPM ? (sr * sr - sk[k] * sk[k]) * third : T(0);
      gk[k] = pos ? T(-1) : T(1);
    }
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int k = a == 0 ? 0 : (a == 4 ? 2 : 1);
    T x6 = PPM ? a6[a] : T(0);
    T v = hk[k] * (PPM ? da[a] + gk[k] * x6 : da[a]);
    if (PPM) v += qk[k] * x6;
    aL[a] = sa[a] > T(0) ? v : T(0);
    aR[a] = sa[a] < T(0) ? v : T(0);
  }
  V5<T> cL = char_R(w, c, ir, aL);
  V5<T> cR = char_R(w, c, ir, aR);
#pragma unroll
  for (int n = 0; n < 5; ++n) {
    fr[n] = L[n] + cL[n];
    fl[n] = R[n] + cR[n];
  }
}

// ---- Riemann solvers (frame states in, frame flux out) ----------------------
template <typename T> struct Roe {
  T u, v, w, H, c2;
  T rL, rR;  // FP32: 1/sqrt(rho) of the left and right states (unused in FP64)
};
template <typename T> HY_DEV Roe<T> roe_avg(const V5<T>& L, const V5<T>& R, T EL, T ER, const Phys<T>& ph) {
  Roe<T> a;
  T sL, sR, hL, hR;  // sqrt(rho) and (E + p) / sqrt(rho) of each side
  if constexpr (FastMath<T>::on) {
    a.rL = vrsq(L[0]);
    a.rR = vrsq(R[0]);
    sL = L[0] * a.rL;
    sR = R[0] * a.rR;
    hL = (EL + L[4]) * a.rL;
    hR = (ER + R[4]) * a.rR;
  } else {
    a.rL = a.rR = T(0);
    sL = vsqrt(L[0]);
    sR = vsqrt(R[0]);
    hL = vdiv(EL + L[4], sL);
    hR = vdiv(ER + R[4], sR);
  }
  T inv = vrcp(sL + sR);
  T wl = sL * inv, wr = sR * inv;
  a.u = wl * L[1] + wr * R[1];
  a.v = wl * L[2] + wr * R[2];
  a.w = wl * L[3] + wr * R[3];
  // H = (E + p) / rho; sqrt(rho) * H = (E + p) / sqrt(rho)
  a.H = (hL + hR) * inv;
  a.c2 = ph.gm1 * (a.H - T(0.5) * (a.u * a.u + a.v * a.v + a.w * a.w));
  return a;
}
// Sound speed of a state; FP32 forms sqrt(gamma p) / sqrt(rho) with the
// known 1/sqrt(rho).
template <typename T> HY_DEV T sound_rs(const V5<T>& W, T rs, const Phys<T>& ph) {
  if constexpr (FastMath<T>::on) return vsqrt(ph.gamma * W[4]) * rs;
  else return sound(W, ph);
}
template <typename T> HY_DEV T total_energy(const V5<T>& W, const Phys<T>& ph) {
  return W[4] * ph.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
}

// Physical flux of a frame state whose total energy E is known.
template <typename T> HY_DEV V5<T> flux_with_energy(const V5<T>& W, T E) {
  V5<T> F;
  F[0] = W[0] * W[1];
  F[1] = F[0] * W[1] + W[4];
  F[2] = F[0] * W[2];
  F[3] = F[0] * W[3];
  F[4] = W[1] * (E + W[4]);
  return F;
}

template <typename T>
HY_DEV V5<T> hlle(const V5<T>& L, const V5<T>& R, const Phys<T>& ph) {
  T EL = total_energy(L, ph), ER = total_energy(R, ph);
  Roe<T> a = roe_avg(L, R, EL, ER, ph);
  T ct = vsqrt(vmax(a.c2, T(0)));
  T cL = sound_rs(L, a.rL, ph), cR = sound_rs(R, a.rR, ph);
  T SL = vmin(L[1] - cL, a.u - ct);
  T SR = vmax(R[1] + cR, a.u + ct);
  T bm = vmin(SL, T(0)), bp = vmax(SR, T(0));
  T idb = vrcp(bp - bm);
  V5<T> FL = flux_with_energy(L, EL), FR = flux_with_energy(R, ER);
  V5<T> UL, UR;
  UL[0] = L[0]; UL[1] = L[0] * L[1]; UL[2] = L[0] * L[2]; UL[3] = L[0] * L[3]; UL[4] = EL;
  UR[0] = R[0]; UR[1] = R[0] * R[1]; UR[2] = R[0] * R[2]; UR[3] = R[0] * R[3]; UR[4] = ER;
  V5<T> F;
  T bb = bp * bm;
#pragma unroll
  for (int n = 0; n < 5; ++n) F[n] = (bp * FL[n] - bm * FR[n] + bb * (UR[n] - UL[n])) * idb;
  return F;
}

template <typename T>
HY_DEV V5<T> hllc(const V5<T>& L, const V5<T>& R, const Phys<T>& ph) {
  T EL = total_energy(L, ph), ER = total_energy(R, ph);
  Roe<T> a = roe_avg(L, R, EL, ER, ph);
  T ct = vsqrt(vmax(a.c2, T(0)));
  T cL = sound_rs(L, a.rL, ph), cR = sound_rs(R, a.rR, ph);
  T SL = vmin(L[1] - cL, a.u - ct);
  T SR = vmax(R[1] + cR, a.u + ct);
  T mL = L[0] * (SL - L[1]);
  T mR = R[0] * (SR - R[1]);
  T Ss = vdiv(R[4] - L[4] + mL * L[1] - mR * R[1], mL - mR);
  // Select the side, then form its star flux; supersonic cases reduce to
  // the upwind physical flux.
  bool supL = SL >= T(0), supR = SR <= T(0);
  bool left = supL || (!supR && Ss >= T(0));
  V5<T> W = left ? L : R;
  T E = left ? EL : ER;
  T S = left ? SL : SR;
  T m = left ? mL : mR;
  T rs = left ? a.rL : a.rR;
  V5<T> F = flux_with_energy(W, E);
  if (supL || supR) return F;
  if constexpr (FastMath<T>::on) {
    // FP32: F* = F + S (U* - U) with one reciprocal r = 1/(S - S*):
    // U* = m r (1, S*, v, w, E/rho + (S* - u)(S* + p/m)), so with
    // d = m r - rho the momentum and energy parts are
    //   rho* - rho = d, (rho u)* - rho u = m r S* - rho u, transverse d v, d w,
    //   E* - E = d E / rho + (S* - u)(m r S* + p r).
    const T r = vrcp(S - Ss);
    const T fac = m * r;
    const T d = fac - W[0];
    const T facS = fac * Ss;
    const T Er = E * (rs * rs);  // E / rho
    const T dE = d * Er + (Ss - W[1]) * (facS + W[4] * r);
    V5<T> Fs;
    Fs[0] = F[0] + S * d;
    Fs[1] = F[1] + S * (facS - W[0] * W[1]);
    Fs[2] = F[2] + S * (d * W[2]);
    Fs[3] = F[3] + S * (d * W[3]);
    Fs[4] = F[4] + S * dE;
    return Fs;
  } else {
    T fac = vdiv(m, S - Ss);
    V5<T> U;
    U[0] = W[0]; U[1] = W[0] * W[1]; U[2] = W[0] * W[2]; U[3] = W[0] * W[3]; U[4] = E;
    V5<T> Us;
    Us[0] = fac;
    Us[1] = fac * Ss;
    Us[2] = fac * W[2];
    Us[3] = fac * W[3];
    Us[4] = fac * (vdiv(E, W[0]) + (Ss - W[1]) * (Ss + vdiv(W[4], m)));
    V5<T> Fs;
#pragma unroll
    for (int n = 0; n < 5; ++n) Fs[n] = F[n] + S * (Us[n] - U[n]);
    return Fs;
  }
}

// Roe flux; on failure of the linearization (non-positive averaged c^2, or
// negative density / pressure in either intermediate state) the HLLE flux
// (or HLLC with the fallback flag) is used and *fails is set.
template <typename T>
HY_DEV V5<T> roe(const V5<T>& L, const V5<T>& R, const Phys<T>& ph, int* fails) {
  T EL = total_energy(L, ph), ER = total_energy(R, ph);
  Roe<T> a = roe_avg(L, R, EL, ER, ph);
  bool ok = a.c2 > T(0);
  T ct = vsqrt(vmax(a.c2, T(0)));
  T ict = vrcp(ct);
  V5<T> dU;
  dU[0] = R[0] - L[0];
  dU[1] = R[0] * R[1] - L[0] * L[1];
  dU[2] = R[0] * R[2] - L[0] * L[2];
  dU[3] = R[0] * R[3] - L[0] * L[3];
  dU[4] = ER - EL;
  T q2 = a.u * a.u + a.v * a.v + a.w * a.w;
  T a3 = dU[2] - a.v * dU[0];
  T a4 = dU[3] - a.w * dU[0];
  T dEp = dU[4] - a3 * a.v - a4 * a.w;
  T a2 = ph.gm1 * ict * ict * (dU[0] * (a.H - a.u * a.u) + a.u * dU[1] - dEp);
  T a1 = (dU[0] * (a.u + ct) - dU[1] - ct * a2) * T(0.5) * ict;
  T a5 = dU[0] - a1 - a2;
  // Intermediate states U_L + a1 K1 and U_R - a5 K5.
  {
    T r1 = L[0] + a1;
    T m1n = L[0] * L[1] + a1 * (a.u - ct);
    T m1a = L[0] * L[2] + a1 * a.v;
    T m1b = L[0] * L[3] + a1 * a.w;
    T e1 = EL + a1 * (a.H - a.u * ct);
    T p1 = ph.gm1 * (e1 - vdiv(T(0.5) * (m1n * m1n + m1a * m1a + m1b * m1b), r1));
    T r2 = R[0] - a5;
    T m2n = R[0] * R[1] - a5 * (a.u + ct);
    T m2a = R[0] * R[2] - a5 * a.v;
    T m2b = R[0] * R[3] - a5 * a.w;
    T e2 = ER - a5 * (a.H + a.u * ct);
    T p2 = ph.gm1 * (e2 - vdiv(T(0.5) * (m2n * m2n + m2a * m2a + m2b * m2b), r2));
    ok = ok && r1 > T(0) && p1 > T(0) && r2 > T(0) && p2 > T(0);
  }
  if (!ok) {
    ++*fails;
    return ph.roe_fb_hllc ? hllc(L, R, ph) : hlle(L, R, ph);
  }
  V5<T> FL = flux_with_energy(L, EL), FR = flux_with_energy(R, ER);
  T l1 = vabs(a.u - ct) * a1, l2 = vabs(a.u), l5 = vabs(a.u + ct) * a5;
  T l2a2 = l2 * a2, l2a3 = l2 * a3, l2a4 = l2 * a4;
  V5<T> F;
  F[0] = T(0.5) * (FL[0] + FR[0] - (l1 + l2a2 + l5));
  F[1] = T(0.5) * (FL[1] + FR[1] - (l1 * (a.u - ct) + l2a2 * a.u + l5 * (a.u + ct)));
  F[2] = T(0.5) * (FL[2] + FR[2] - ((l1 + l2a2 + l5) * a.v + l2a3));
  F[3] = T(0.5) * (FL[3] + FR[3] - ((l1 + l2a2 + l5) * a.w + l2a4));
  F[4] = T(0.5) * (FL[4] + FR[4] -
                   (l1 * (a.H - a.u * ct) + l2a2 * T(0.5) * q2 + l2a3 * a.v + l2a4 * a.w + l5 * (a.H + a.u * ct)));
  return F;
}

// Riemann dispatch: RS = 0 Roe, 1 HLLC, 2 HLLE.
template <int RS, typename T>
HY_DEV V5<T> riemann(const V5<T>& L, const V5<T>& R, const Phys<T>& ph, int* fails) {
  if (RS == 1) return hllc(L, R, ph);
  if (RS == 2) return hlle(L, R, ph);
  return roe(L, R, ph, fails);
}

}  // namespace hy
