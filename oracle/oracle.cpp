// FP64 CPU oracle for the directionally unsplit hydrodynamic schemes of
// Schive, Zhang & Chiueh, "Directionally Unsplit Hydrodynamic Schemes with
// Hybrid MPI/OpenMP/GPU Parallelization in AMR" (arXiv:1103.3373).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
// GPU path is checked against.  Only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it.  It shares no code, header or
// table with the HIP library and includes nothing from it.
//
// What it computes (paper Sec. 2, steps (1)-(5)):
//   * MHM  : reconstruction, Hancock half step by flux differences of the
//            face states in all three directions (no Riemann solver), one set
//            of Riemann solves, conservative update.
//   * VL   : first-order Riemann fluxes on piecewise-constant data, half-step
//            unsplit update, reconstruction from the half-step state, Riemann
//            solves, conservative update.
//   * CTU  : reconstruction with characteristic tracing to t+dt/2 (step 1),
//            Riemann solves (step 2), transverse flux-gradient correction and
//            second Riemann solves (step 3), conservative update (step 4),
//            patch-boundary flux store (step 5).
//   * PLM / PPM reconstruction; generalized minmod, van Leer, van Albada and
//     hybrid limiters; primitive or characteristic limiting (Sec. 2).
//   * Exact, Roe (with positivity failure test and HLLE/HLLC fallback), HLLC
//     and HLLE Riemann solvers (Sec. 2).
//   * CFL time step and conserved-variable sums.
// The paper defers every formula to published methods; the concrete reading
// used here (eigenvectors, limiter forms, tracing formulas, wave-speed
// estimates, floors) is listed with the design notes of the repository.
//
// Data layout: conserved variables (rho, mx, my, mz, E), array [var][z][y][x]
// with x fastest (Sec. 3.1 layout).  Two grid modes share one driver:
//   periodic : a whole box with periodic wrap; every quantity on every cell.
//   padded   : one patch group with g ghost cells per side; each stage is
//              computed on the range its stencil allows and the interior
//              16^3 (or whatever lies g cells inside) is returned.
//
// Build with -O2 -ffp-contract=off and without fast-math.  Compiling with
// -DORACLE_COUNT_OPS replaces the scalar type by an operation-counting type;
// that build only counts the floating-point work of a step.

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

// ---------------------------------------------------------------------------
// Scalar type: double, or a double that counts the operations applied to it.
// Counted: + - * / sqrt, comparisons (and therefore min/max).  Not counted:
// negation and absolute value (sign-bit manipulation).
// ---------------------------------------------------------------------------
#ifdef ORACLE_COUNT_OPS
static unsigned long long g_ops = 0;
struct real {
  double x;
  real() : x(0.0) {}
  real(double v) : x(v) {}
};
static inline real operator+(real a, real b) { ++g_ops; return real(a.x + b.x); }
static inline real operator-(real a, real b) { ++g_ops; return real(a.x - b.x); }
static inline real operator*(real a, real b) { ++g_ops; return real(a.x * b.x); }
static inline real operator/(real a, real b) { ++g_ops; return real(a.x / b.x); }
static inline real operator-(real a) { return real(-a.x); }
static inline real& operator+=(real& a, real b) { a = a + b; return a; }
static inline real& operator-=(real& a, real b) { a = a - b; return a; }
static inline real& operator*=(real& a, real b) { a = a * b; return a; }
static inline bool operator<(real a, real b) { ++g_ops; return a.x < b.x; }
static inline bool operator<=(real a, real b) { ++g_ops; return a.x <= b.x; }
static inline bool operator>(real a, real b) { ++g_ops; return a.x > b.x; }
static inline bool operator>=(real a, real b) { ++g_ops; return a.x >= b.x; }
static inline double to_d(real a) { return a.x; }
static inline real r_sqrt(real a) { ++g_ops; return real(std::sqrt(a.x)); }
static inline real r_abs(real a) { return real(std::fabs(a.x)); }
static inline real r_pow(real a, double e) { ++g_ops; return real(std::pow(a.x, e)); }
#else
typedef double real;
static inline double to_d(double a) { return a; }
static inline double r_sqrt(double a) { return std::sqrt(a); }
static inline double r_abs(double a) { return std::fabs(a); }
static inline double r_pow(double a, double e) { return std::pow(a, e); }
#endif

static inline real r_min(real a, real b) { return (a < b) ? a : b; }
static inline real r_max(real a, real b) { return (a > b) ? a : b; }

// ---------------------------------------------------------------------------
// Options (values match the public C enums of the library so that tests can
// pass the same integers to both; the oracle defines its own copy).
// ---------------------------------------------------------------------------
enum { S_MHM = 0, S_VL = 1, S_CTU = 2 };
enum { R_PLM = 0, R_PPM = 1 };
enum { RS_ROE = 0, RS_HLLC = 1, RS_HLLE = 2, RS_EXACT = 3 };
enum { L_GMINMOD = 0, L_VANLEER = 1, L_VANALBADA = 2, L_HYBRID = 3 };
enum { F_CHAR = 0x02, F_FLUX_MID = 0x04, F_ROE_FB_HLLC = 0x10, F_ROE_FB_EXACT = 0x80 };
// Oracle-only switches that turn the nonlinear parts of the reconstruction
// off, so that the smooth-data convergence of the underlying linear scheme
// can be pinned on its own: L_CENTRAL takes the unlimited centred slope,
// F_NO_MONO skips the PPM edge clipping and the parabola monotonization.
// The HIP library has neither.
enum { L_CENTRAL = 4 };
enum { F_NO_MONO = 0x100 };

struct V5 {
  real v[5];
  real& operator[](int i) { return v[i]; }
  const real& operator[](int i) const { return v[i]; }
};

struct Cfg {
  real gamma, gm1;   // ratio of specific heats and gamma-1
  real dtdh;         // dt/dh
  real hdtdh;        // dt/(2 dh)
  real theta;        // generalized-minmod parameter
  real floor;        // density and pressure floor for face / half-step states
  int scheme, recon, riemann, limiter;
  bool charlim, fb_hllc, fb_exact, no_mono;
};

struct Stats {
  long long solves;      // Riemann solves
  long long roe_fail;    // interfaces where the Roe linearization failed
  long long floor_hits;  // floor activations
  long long exact_fail;  // exact solver: vacuum generated / no convergence
};
static Stats g_stats;

// Velocity component (1..3) that plays the role of normal (k=0), first
// transverse (k=1) and second transverse (k=2) in direction d: cyclic, so
// x -> (u,v,w), y -> (v,w,u), z -> (w,u,v).
static inline int vcomp(int d, int k) { return 1 + (d + k) % 3; }

static V5 to_frame(const V5& a, int d) {
  V5 r;
  r[0] = a[0];
  r[1] = a[vcomp(d, 0)];
  r[2] = a[vcomp(d, 1)];
  r[3] = a[vcomp(d, 2)];
  r[4] = a[4];
  return r;
}
static V5 from_frame(const V5& a, int d) {
  V5 r;
  r[0] = a[0];
  r[vcomp(d, 0)] = a[1];
  r[vcomp(d, 1)] = a[2];
  r[vcomp(d, 2)] = a[3];
  r[4] = a[4];
  return r;
}

// ---------------------------------------------------------------------------
// Ideal-gas relations.  W = (rho, u, v, w, p), U = (rho, mx, my, mz, E).
// These are frame independent (velocity components only permute).
// ---------------------------------------------------------------------------
static V5 prim_of(const V5& U, const Cfg& c) {
  V5 W;
  real r = U[0];
  W[0] = r;
  W[1] = U[1] / r;
  W[2] = U[2] / r;
  W[3] = U[3] / r;
  real ke = 0.5 * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3]);
  W[4] = c.gm1 * (U[4] - ke);
  return W;
}
static V5 cons_of(const V5& W, const Cfg& c) {
  V5 U;
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  U[4] = W[4] / c.gm1 + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  return U;
}
// Physical flux along the first velocity component of a frame-ordered state.
static V5 phys_flux(const V5& W, const Cfg& c) {
  V5 F;
  real E = W[4] / c.gm1 + 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  F[0] = W[0] * W[1];
  F[1] = F[0] * W[1] + W[4];
  F[2] = F[0] * W[2];
  F[3] = F[0] * W[3];
  F[4] = W[1] * (E + W[4]);
  return F;
}
static real sound_speed(const V5& W, const Cfg& c) { return r_sqrt(c.gamma * W[4] / W[0]); }

static void apply_floor(V5& W, const Cfg& c) {
  if (W[0] < c.floor) { W[0] = c.floor; ++g_stats.floor_hits; }
  if (W[4] < c.floor) { W[4] = c.floor; ++g_stats.floor_hits; }
}

// ---------------------------------------------------------------------------
// Slope limiters (Sec. 2: generalized minmod, van Leer-type, van Albada-type,
// and the hybrid of generalized minmod and van Leer).  All return 0 at an
// extremum (dl*dr <= 0).
// ---------------------------------------------------------------------------
static real limit_slope(real dl, real dr, const Cfg& c) {
  if (c.limiter == L_CENTRAL) return 0.5 * (dl + dr);
  if (dl * dr <= 0.0) return 0.0;
  real dc = 0.5 * (dl + dr);
  switch (c.limiter) {
    case L_GMINMOD: {
      real m = r_min(r_min(c.theta * r_abs(dl), c.theta * r_abs(dr)), r_abs(dc));
      return (dc > 0.0) ? m : -m;
    }
    case L_VANLEER:
      return 2.0 * dl * dr / (dl + dr);
    case L_VANALBADA:
      return dl * dr * (dl + dr) / (dl * dl + dr * dr);
    default: {  // L_HYBRID: van Leer slope bounded by the generalized minmod slope
      real vl = r_abs(2.0 * dl * dr / (dl + dr));
      real m = r_min(r_min(r_min(c.theta * r_abs(dl), c.theta * r_abs(dr)), r_abs(dc)), vl);
      return (dc > 0.0) ? m : -m;
    }
  }
}

// Characteristic decomposition of the primitive Euler system in a frame
// (normal velocity first) at state W with sound speed cs.  Eigenvalues in
// order (u-c, u, u, u, u+c).
static V5 char_project(const V5& W, real cs, const V5& dw) {  // a = L dw
  V5 a;
  real c2 = cs * cs;
  a[0] = -0.5 * W[0] / cs * dw[1] + 0.5 * dw[4] / c2;
  a[1] = dw[0] - dw[4] / c2;
  a[2] = dw[2];
  a[3] = dw[3];
  a[4] = 0.5 * W[0] / cs * dw[1] + 0.5 * dw[4] / c2;
  return a;
}
static V5 char_expand(const V5& W, real cs, const V5& a) {  // dw = R a
  V5 dw;
  dw[0] = a[0] + a[1] + a[4];
  dw[1] = cs / W[0] * (a[4] - a[0]);
  dw[2] = a[2];
  dw[3] = a[3];
  dw[4] = cs * cs * (a[0] + a[4]);
  return dw;
}

// Limited slope of the middle cell from three frame-ordered states.
static V5 limited_slope(const V5& wm, const V5& w0, const V5& wp, const Cfg& c) {
  V5 dl, dr, s;
  for (int n = 0; n < 5; ++n) { dl[n] = w0[n] - wm[n]; dr[n] = wp[n] - w0[n]; }
  if (!c.charlim) {
    for (int n = 0; n < 5; ++n) s[n] = limit_slope(dl[n], dr[n], c);
    return s;
  }
  real cs = sound_speed(w0, c);
  V5 al = char_project(w0, cs, dl);
  V5 ar = char_project(w0, cs, dr);
  V5 am;
  for (int n = 0; n < 5; ++n) am[n] = limit_slope(al[n], ar[n], c);
  return char_expand(w0, cs, am);
}

// PPM edge value between cells a and b from their states and limited slopes,
// clipped into the range of the two cell values (unless `clip` is false).
static V5 ppm_edge(const V5& wa, const V5& wb, const V5& sa, const V5& sb, bool clip = true) {
  V5 e;
  for (int n = 0; n < 5; ++n) {
    real v = 0.5 * (wa[n] + wb[n]) - (sb[n] - sa[n]) / 6.0;
    real lo = r_min(wa[n], wb[n]), hi = r_max(wa[n], wb[n]);
    e[n] = clip ? r_min(r_max(v, lo), hi) : v;
  }
  return e;
}

// Parabola monotonization (per primitive component).
static void ppm_monotonize(const V5& w, V5& wl, V5& wr) {
  for (int n = 0; n < 5; ++n) {
    real a = w[n], l = wl[n], r = wr[n];
    if ((r - a) * (a - l) <= 0.0) {
      l = a;
      r = a;
    } else {
      real d = r - l;
      real t = d * (a - 0.5 * (l + r));
      real d2 = d * d / 6.0;
      if (t > d2) l = 3.0 * a - 2.0 * r;
      else if (t < -d2) r = 3.0 * a - 2.0 * l;
    }
    wl[n] = l;
    wr[n] = r;
  }
}

// Curvature coefficient of the parabola through the face values wl, wr with
// cell mean w: W6 = 6 (W - (WL + WR) / 2).
static V5 ppm_w6(const V5& w, const V5& wl, const V5& wr) {
  V5 w6;
  for (int n = 0; n < 5; ++n) w6[n] = 6.0 * (w[n] - 0.5 * (wl[n] + wr[n]));
  return w6;
}

// Characteristic tracing to t+dt/2 (CTU step (1)): Colella's reference-state
// form.  Input: cell state w, its face values wl (left face) and wr (right
// face) and the parabola coefficient w6 (zero for PLM).  Output overwrites
// wl / wr with the states at the left / right faces at the half step.
static void ctu_trace(const V5& w, V5& wl, V5& wr, const V5& w6, bool ppm, const Cfg& c) {
  real cs = sound_speed(w, c);
  real lam[5] = {w[1] - cs, w[1], w[1], w[1], w[1] + cs};
  real s[5];
  for (int a = 0; a < 5; ++a) s[a] = lam[a] * c.dtdh;
  real sM = r_max(s[4], 0.0);
  real sm = r_min(s[0], 0.0);
  V5 dw;
  for (int n = 0; n < 5; ++n) dw[n] = wr[n] - wl[n];
  V5 da = char_project(w, cs, dw);
  V5 a6 = ppm ? char_project(w, cs, w6) : w6;

  V5 L, R;  // state at the right face (left state of face i+1/2), left face
  for (int n = 0; n < 5; ++n) {
    real t6p = ppm ? (1.0 - 2.0 / 3.0 * sM) * w6[n] : real(0.0);
    real t6m = ppm ? (1.0 + 2.0 / 3.0 * sm) * w6[n] : real(0.0);
    L[n] = wr[n] - 0.5 * sM * (dw[n] - t6p);
    R[n] = wl[n] - 0.5 * sm * (dw[n] + t6m);
  }
  for (int a = 0; a < 5; ++a) {
    V5 unit;
    for (int n = 0; n < 5; ++n) unit[n] = 0.0;
    if (lam[a] > 0.0) {
      real amp = 0.5 * (sM - s[a]) * (da[a] - a6[a]);
      if (ppm) amp += (sM * sM - s[a] * s[a]) / 3.0 * a6[a];
      unit[a] = amp;
      V5 contrib = char_expand(w, cs, unit);
      for (int n = 0; n < 5; ++n) L[n] += contrib[n];
    }
    if (lam[a] < 0.0) {
      real amp = 0.5 * (sm - s[a]) * (da[a] + a6[a]);
      if (ppm) amp += (sm * sm - s[a] * s[a]) / 3.0 * a6[a];
      unit[a] = amp;
      V5 contrib = char_expand(w, cs, unit);
      for (int n = 0; n < 5; ++n) R[n] += contrib[n];
    }
  }
  wr = L;
  wl = R;
}

// ---------------------------------------------------------------------------
// Riemann solvers.  Inputs and outputs are frame ordered (normal first).
// ---------------------------------------------------------------------------
struct RoeAvg {
  real u, v, w, H, c2;
};
static RoeAvg roe_average(const V5& L, const V5& R, const Cfg& c) {
  real EL = L[4] / c.gm1 + 0.5 * L[0] * (L[1] * L[1] + L[2] * L[2] + L[3] * L[3]);
  real ER = R[4] / c.gm1 + 0.5 * R[0] * (R[1] * R[1] + R[2] * R[2] + R[3] * R[3]);
  real HL = (EL + L[4]) / L[0];
  real HR = (ER + R[4]) / R[0];
  real sL = r_sqrt(L[0]), sR = r_sqrt(R[0]);
  real inv = 1.0 / (sL + sR);
  RoeAvg a;
  a.u = (sL * L[1] + sR * R[1]) * inv;
  a.v = (sL * L[2] + sR * R[2]) * inv;
  a.w = (sL * L[3] + sR * R[3]) * inv;
  a.H = (sL * HL + sR * HR) * inv;
  a.c2 = c.gm1 * (a.H - 0.5 * (a.u * a.u + a.v * a.v + a.w * a.w));
  return a;
}

// Einfeldt wave-speed estimates (used by HLLE and HLLC).
static void einfeldt_speeds(const V5& L, const V5& R, const Cfg& c, real& SL, real& SR) {
  RoeAvg a = roe_average(L, R, c);
  real ct = r_sqrt(r_max(a.c2, 0.0));
  real cL = sound_speed(L, c), cR = sound_speed(R, c);
  SL = r_min(L[1] - cL, a.u - ct);
  SR = r_max(R[1] + cR, a.u + ct);
}

static V5 flux_hlle(const V5& L, const V5& R, const Cfg& c) {
  real SL, SR;
  einfeldt_speeds(L, R, c, SL, SR);
  real bm = r_min(SL, 0.0), bp = r_max(SR, 0.0);
  V5 FL = phys_flux(L, c), FR = phys_flux(R, c);
  V5 UL = cons_of(L, c), UR = cons_of(R, c);
  V5 F;
  for (int n = 0; n < 5; ++n)
    F[n] = (bp * FL[n] - bm * FR[n] + bp * bm * (UR[n] - UL[n])) / (bp - bm);
  return F;
}

static V5 flux_hllc(const V5& L, const V5& R, const Cfg& c) {
  real SL, SR;
  einfeldt_speeds(L, R, c, SL, SR);
  V5 FL = phys_flux(L, c), FR = phys_flux(R, c);
  if (SL >= 0.0) return FL;
  if (SR <= 0.0) return FR;
  real mL = L[0] * (SL - L[1]);  // rho_L (S_L - u_L)
  real mR = R[0] * (SR - R[1]);
  real Ss = (R[4] - L[4] + mL * L[1] - mR * R[1]) / (mL - mR);
  const V5& W = (Ss >= 0.0) ? L : R;
  real S = (Ss >= 0.0) ? SL : SR;
  real m = (Ss >= 0.0) ? mL : mR;
  V5 U = cons_of(W, c);
  V5 F = (Ss >= 0.0) ? FL : FR;
  real fac = m / (S - Ss);
  V5 Us;
  Us[0] = fac;
  Us[1] = fac * Ss;
  Us[2] = fac * W[2];
  Us[3] = fac * W[3];
  Us[4] = fac * (U[4] / W[0] + (Ss - W[1]) * (Ss + W[4] / m));
  V5 Fs;
  for (int n = 0; n < 5; ++n) Fs[n] = F[n] + S * (Us[n] - U[n]);
  return Fs;
}

// Returns false when the Roe linearization fails (negative density or
// pressure in an intermediate state, or a non-positive averaged c^2).
static bool flux_roe(const V5& L, const V5& R, const Cfg& c, V5& F) {
  RoeAvg a = roe_average(L, R, c);
  if (a.c2 <= 0.0) return false;
  real ct = r_sqrt(a.c2);
  V5 UL = cons_of(L, c), UR = cons_of(R, c);
  V5 dU;
  for (int n = 0; n < 5; ++n) dU[n] = UR[n] - UL[n];
  real q2 = a.u * a.u + a.v * a.v + a.w * a.w;
  real a3 = dU[2] - a.v * dU[0];
  real a4 = dU[3] - a.w * dU[0];
  real dEp = dU[4] - a3 * a.v - a4 * a.w;
  real a2 = c.gm1 / a.c2 * (dU[0] * (a.H - a.u * a.u) + a.u * dU[1] - dEp);
  real a1 = (dU[0] * (a.u + ct) - dU[1] - ct * a2) / (2.0 * ct);
  real a5 = dU[0] - a1 - a2;
  V5 K1, K2, K3, K4, K5;
  K1[0] = 1.0; K1[1] = a.u - ct; K1[2] = a.v; K1[3] = a.w; K1[4] = a.H - a.u * ct;
  K2[0] = 1.0; K2[1] = a.u; K2[2] = a.v; K2[3] = a.w; K2[4] = 0.5 * q2;
  K3[0] = 0.0; K3[1] = 0.0; K3[2] = 1.0; K3[3] = 0.0; K3[4] = a.v;
  K4[0] = 0.0; K4[1] = 0.0; K4[2] = 0.0; K4[3] = 1.0; K4[4] = a.w;
  K5[0] = 1.0; K5[1] = a.u + ct; K5[2] = a.v; K5[3] = a.w; K5[4] = a.H + a.u * ct;
  // Positivity of the two intermediate states.
  V5 Us1, Us2;
  for (int n = 0; n < 5; ++n) { Us1[n] = UL[n] + a1 * K1[n]; Us2[n] = UR[n] - a5 * K5[n]; }
  V5 Ws1 = prim_of(Us1, c), Ws2 = prim_of(Us2, c);
  if (Us1[0] <= 0.0 || Ws1[4] <= 0.0 || Us2[0] <= 0.0 || Ws2[4] <= 0.0) return false;
  V5 FL = phys_flux(L, c), FR = phys_flux(R, c);
  real l1 = r_abs(a.u - ct), l2 = r_abs(a.u), l5 = r_abs(a.u + ct);
  for (int n = 0; n < 5; ++n)
    F[n] = 0.5 * (FL[n] + FR[n]) -
           0.5 * (l1 * a1 * K1[n] + l2 * a2 * K2[n] + l2 * a3 * K3[n] + l2 * a4 * K4[n] + l5 * a5 * K5[n]);
  return true;
}

// Exact Riemann solver: pressure function with Newton iteration for p*, then
// sampling of the self-similar solution at xi = x/t.
struct ExactStar {
  real p, u, rhoL, rhoR;
  int ok;
};
static void pfunc(real p, real rk, real pk, real ck, const Cfg& c, real& f, real& df) {
  if (p > pk) {
    real A = 2.0 / ((c.gamma + 1.0) * rk);
    real B = c.gm1 / (c.gamma + 1.0) * pk;
    real q = r_sqrt(A / (p + B));
    f = (p - pk) * q;
    df = q * (1.0 - 0.5 * (p - pk) / (B + p));
  } else {
    real pr = p / pk;
    f = 2.0 * ck / c.gm1 * (r_pow(pr, to_d(c.gm1 / (2.0 * c.gamma))) - 1.0);
    df = 1.0 / (rk * ck) * r_pow(pr, to_d(-(c.gamma + 1.0) / (2.0 * c.gamma)));
  }
}
static ExactStar exact_star(const V5& L, const V5& R, const Cfg& c) {
  ExactStar s;
  real cL = sound_speed(L, c), cR = sound_speed(R, c);
  real du = R[1] - L[1];
  s.ok = 1;
  if (2.0 / c.gm1 * (cL + cR) <= du) {  // vacuum generated
    s.ok = 0; s.p = 0.0; s.u = 0.5 * (L[1] + R[1]); s.rhoL = 0.0; s.rhoR = 0.0;
    return s;
  }
  real ppv = 0.5 * (L[4] + R[4]) - 0.125 * du * (L[0] + R[0]) * (cL + cR);
  real p = r_max(ppv, 1e-8 * r_min(L[4], R[4]));
  int it = 0;
  for (; it < 200; ++it) {
    real fL, dL, fR, dR;
    pfunc(p, L[0], L[4], cL, c, fL, dL);
    pfunc(p, R[0], R[4], cR, c, fR, dR);
    real pn = p - (fL + fR + du) / (dL + dR);
    if (pn < 0.0) pn = 1e-12 * p;
    real ch = 2.0 * r_abs(pn - p) / (pn + p);
    p = pn;
    if (ch < 1e-15) break;
  }
  if (it >= 200) s.ok = 0;
  real fL, dL, fR, dR;
  pfunc(p, L[0], L[4], cL, c, fL, dL);
  pfunc(p, R[0], R[4], cR, c, fR, dR);
  s.p = p;
  s.u = 0.5 * (L[1] + R[1]) + 0.5 * (fR - fL);
  real g6 = c.gm1 / (c.gamma + 1.0);
  if (p > L[4]) s.rhoL = L[0] * (p / L[4] + g6) / (g6 * p / L[4] + 1.0);
  else s.rhoL = L[0] * r_pow(p / L[4], to_d(1.0 / c.gamma));
  if (p > R[4]) s.rhoR = R[0] * (p / R[4] + g6) / (g6 * p / R[4] + 1.0);
  else s.rhoR = R[0] * r_pow(p / R[4], to_d(1.0 / c.gamma));
  return s;
}
// Sample the exact solution at xi; returns the frame-ordered primitive state.
static V5 exact_sample(const V5& L, const V5& R, const ExactStar& s, real xi, const Cfg& c) {
  V5 W;
  real gp1 = c.gamma + 1.0;
  if (xi <= s.u) {  // left of the contact
    real cL = sound_speed(L, c);
    W[2] = L[2]; W[3] = L[3];
    if (s.p > L[4]) {  // left shock
      real SL = L[1] - cL * r_sqrt(gp1 / (2.0 * c.gamma) * s.p / L[4] + c.gm1 / (2.0 * c.gamma));
      if (xi <= SL) { W = L; }
      else { W[0] = s.rhoL; W[1] = s.u; W[4] = s.p; }
    } else {  // left rarefaction
      real csL = cL * r_pow(s.p / L[4], to_d(c.gm1 / (2.0 * c.gamma)));
      real head = L[1] - cL, tail = s.u - csL;
      if (xi <= head) { W = L; }
      else if (xi > tail) { W[0] = s.rhoL; W[1] = s.u; W[4] = s.p; }
      else {
        real b = 2.0 / gp1 + c.gm1 / (gp1 * cL) * (L[1] - xi);
        W[0] = L[0] * r_pow(b, to_d(2.0 / c.gm1));
        W[1] = 2.0 / gp1 * (cL + 0.5 * c.gm1 * L[1] + xi);
        W[4] = L[4] * r_pow(b, to_d(2.0 * c.gamma / c.gm1));
      }
    }
  } else {  // right of the contact
    real cR = sound_speed(R, c);
    W[2] = R[2]; W[3] = R[3];
    if (s.p > R[4]) {  // right shock
      real SR = R[1] + cR * r_sqrt(gp1 / (2.0 * c.gamma) * s.p / R[4] + c.gm1 / (2.0 * c.gamma));
      if (xi >= SR) { W = R; }
      else { W[0] = s.rhoR; W[1] = s.u; W[4] = s.p; }
    } else {  // right rarefaction
      real csR = cR * r_pow(s.p / R[4], to_d(c.gm1 / (2.0 * c.gamma)));
      real head = R[1] + cR, tail = s.u + csR;
      if (xi >= head) { W = R; }
      else if (xi < tail) { W[0] = s.rhoR; W[1] = s.u; W[4] = s.p; }
      else {
        real b = 2.0 / gp1 - c.gm1 / (gp1 * cR) * (R[1] - xi);
        W[0] = R[0] * r_pow(b, to_d(2.0 / c.gm1));
        W[1] = 2.0 / gp1 * (-cR + 0.5 * c.gm1 * R[1] + xi);
        W[4] = R[4] * r_pow(b, to_d(2.0 * c.gamma / c.gm1));
      }
    }
  }
  return W;
}
static V5 flux_exact(const V5& L, const V5& R, const Cfg& c) {
  ExactStar s = exact_star(L, R, c);
  if (!s.ok) ++g_stats.exact_fail;
  return phys_flux(exact_sample(L, R, s, 0.0, c), c);
}

// Riemann dispatcher (frame-ordered states in, frame-ordered flux out).
static V5 riemann_solve(const V5& L, const V5& R, const Cfg& c) {
  ++g_stats.solves;
  switch (c.riemann) {
    case RS_HLLC: return flux_hllc(L, R, c);
    case RS_HLLE: return flux_hlle(L, R, c);
    case RS_EXACT: return flux_exact(L, R, c);
    default: {
      V5 F;
      if (flux_roe(L, R, c, F)) return F;
      ++g_stats.roe_fail;
      if (c.fb_exact) return flux_exact(L, R, c);  // Roe -> exact fallback (Sec. 2)
      return c.fb_hllc ? flux_hllc(L, R, c) : flux_hlle(L, R, c);
    }
  }
}

// ---------------------------------------------------------------------------
// Grid bookkeeping.  A Range is a half-open box of cell indices.  A face
// array stores at index i the face between cells i and i+1 along its axis.
// ---------------------------------------------------------------------------
struct Grid {
  int n[3];
  bool periodic;
  long ncell() const { return (long)n[0] * n[1] * n[2]; }
  long at(int i, int j, int k) const {
    if (periodic) {
      i = ((i % n[0]) + n[0]) % n[0];
      j = ((j % n[1]) + n[1]) % n[1];
      k = ((k % n[2]) + n[2]) % n[2];
    } else if (i < 0 || i >= n[0] || j < 0 || j >= n[1] || k < 0 || k >= n[2]) {
      std::fprintf(stderr, "oracle: index (%d,%d,%d) outside padded grid\n", i, j, k);
      std::abort();
    }
    return ((long)k * n[1] + j) * n[0] + i;
  }
};
struct Range {
  int lo[3], hi[3];
};
static Range full_range(const Grid& g) {
  Range r;
  for (int a = 0; a < 3; ++a) { r.lo[a] = 0; r.hi[a] = g.n[a]; }
  return r;
}
// Shrink along axis a: lo by rl, hi by rh.  No-op on a periodic grid.
static Range shrink(const Grid& g, Range r, int a, int rl, int rh) {
  if (!g.periodic) { r.lo[a] += rl; r.hi[a] -= rh; }
  return r;
}
static Range intersect(Range a, const Range& b) {
  for (int k = 0; k < 3; ++k) {
    if (b.lo[k] > a.lo[k]) a.lo[k] = b.lo[k];
    if (b.hi[k] < a.hi[k]) a.hi[k] = b.hi[k];
  }
  return a;
}
static void step_of(int d, int o[3]) { o[0] = o[1] = o[2] = 0; o[d] = 1; }

#define FOR_RANGE(r, i, j, k)                      \
  for (int k = (r).lo[2]; k < (r).hi[2]; ++k)      \
    for (int j = (r).lo[1]; j < (r).hi[1]; ++j)    \
      for (int i = (r).lo[0]; i < (r).hi[0]; ++i)

typedef std::vector<V5> Field;

// Step (1): face states of direction d for every cell where the stencil of
// the reconstruction fits inside `wr` (the range where W is valid).  States
// are stored in the lab frame.  With `trace`, CTU characteristic tracing is
// applied.  Floors are applied to the resulting states.
static Range face_states(const Grid& g, const Field& W, Range wr, int d, const Cfg& c, bool trace,
                         Field& Wm, Field& Wp) {
  int o[3];
  step_of(d, o);
  // Limited slopes (frame of direction d).
  Range sr = shrink(g, wr, d, 1, 1);
  Field S(g.ncell());
  FOR_RANGE(sr, i, j, k) {
    V5 a = to_frame(W[g.at(i - o[0], j - o[1], k - o[2])], d);
    V5 b = to_frame(W[g.at(i, j, k)], d);
    V5 e = to_frame(W[g.at(i + o[0], j + o[1], k + o[2])], d);
    S[g.at(i, j, k)] = limited_slope(a, b, e, c);
  }
  bool ppm = (c.recon == R_PPM);
  Range fr = ppm ? shrink(g, wr, d, 2, 2) : sr;
  FOR_RANGE(fr, i, j, k) {
    long ic = g.at(i, j, k);
    long im = g.at(i - o[0], j - o[1], k - o[2]);
    long ip = g.at(i + o[0], j + o[1], k + o[2]);
    V5 w = to_frame(W[ic], d);
    V5 wl, wr2, w6;
    if (ppm) {
      V5 wm = to_frame(W[im], d), wp = to_frame(W[ip], d);
      wl = ppm_edge(wm, w, S[im], S[ic], !c.no_mono);
      wr2 = ppm_edge(w, wp, S[ic], S[ip], !c.no_mono);
      if (!c.no_mono) ppm_monotonize(w, wl, wr2);
      w6 = ppm_w6(w, wl, wr2);
    } else {
      for (int n = 0; n < 5; ++n) {
        wl[n] = w[n] - 0.5 * S[ic][n];
        wr2[n] = w[n] + 0.5 * S[ic][n];
        w6[n] = 0.0;
      }
      if (c.charlim) {  // keep the face values between the neighbouring cell values
        V5 wm = to_frame(W[im], d), wp = to_frame(W[ip], d);
        for (int n = 0; n < 5; ++n) {
          wl[n] = r_min(r_max(wl[n], r_min(w[n], wm[n])), r_max(w[n], wm[n]));
          wr2[n] = r_min(r_max(wr2[n], r_min(w[n], wp[n])), r_max(w[n], wp[n]));
        }
      }
    }
    if (trace) ctu_trace(w, wl, wr2, w6, ppm, c);
    apply_floor(wl, c);
    apply_floor(wr2, c);
    Wm[ic] = from_frame(wl, d);
    Wp[ic] = from_frame(wr2, d);
  }
  return fr;
}

// Step (2): Riemann solves along d between the right state of cell i (WpL)
// and the left state of cell i+1 (WmR), for every face whose two cells lie in
// `cr`.  Fluxes are stored in the lab frame.  Returns the face range.
static Range riemann_faces(const Grid& g, const Field& WpL, const Field& WmR, Range cr, int d, const Cfg& c,
                           Field& F) {
  int o[3];
  step_of(d, o);
  Range fr = shrink(g, cr, d, 0, 1);
  FOR_RANGE(fr, i, j, k) {
    V5 L = to_frame(WpL[g.at(i, j, k)], d);
    V5 R = to_frame(WmR[g.at(i + o[0], j + o[1], k + o[2])], d);
    F[g.at(i, j, k)] = from_frame(riemann_solve(L, R, c), d);
  }
  return fr;
}
// Cells where a flux difference along d is available from face range fr.
static Range diff_range(const Grid& g, Range fr, int d) { return shrink(g, fr, d, 1, 0); }
static V5 flux_diff(const Grid& g, const Field& F, int d, int i, int j, int k) {
  int o[3];
  step_of(d, o);
  const V5& a = F[g.at(i, j, k)];
  const V5& b = F[g.at(i - o[0], j - o[1], k - o[2])];
  V5 r;
  for (int n = 0; n < 5; ++n) r[n] = a[n] - b[n];
  return r;
}

// Step (4): U^{n+1} = U^n - dt/dh (dF_x + dF_y + dF_z) over `ur`.
static void conservative_update(const Grid& g, const Field& U, const Field* F, Range ur, const Cfg& c,
                                Field& Unew) {
  FOR_RANGE(ur, i, j, k) {
    V5 dx = flux_diff(g, F[0], 0, i, j, k);
    V5 dy = flux_diff(g, F[1], 1, i, j, k);
    V5 dz = flux_diff(g, F[2], 2, i, j, k);
    const V5& u = U[g.at(i, j, k)];
    V5 r;
    for (int n = 0; n < 5; ++n) r[n] = u[n] - c.dtdh * (dx[n] + dy[n] + dz[n]);
    Unew[g.at(i, j, k)] = r;
  }
}

// One step of the selected scheme on grid g.  Writes the new state on the
// returned range of Unew and the final fluxes into F[3].
static Range scheme_step(const Grid& g, const Field& U, const Cfg& c, Field& Unew, Field* F) {
  long nc = g.ncell();
  Range all = full_range(g);
  Field W(nc);
  FOR_RANGE(all, i, j, k) W[g.at(i, j, k)] = prim_of(U[g.at(i, j, k)], c);

  Field Wm[3], Wp[3];
  for (int d = 0; d < 3; ++d) { Wm[d].resize(nc); Wp[d].resize(nc); F[d].resize(nc); }
  Range fr[3];

  if (c.scheme == S_MHM) {
    Range sr[3];
    for (int d = 0; d < 3; ++d) sr[d] = face_states(g, W, all, d, c, false, Wm[d], Wp[d]);
    Range hr = intersect(intersect(sr[0], sr[1]), sr[2]);
    // Hancock half step: one cell-centred dU from the physical fluxes of the
    // six face states, added to every face state of the cell.
    FOR_RANGE(hr, i, j, k) {
      long ic = g.at(i, j, k);
      V5 dU;
      for (int n = 0; n < 5; ++n) dU[n] = 0.0;
      for (int d = 0; d < 3; ++d) {
        V5 Fp = from_frame(phys_flux(to_frame(Wp[d][ic], d), c), d);
        V5 Fm = from_frame(phys_flux(to_frame(Wm[d][ic], d), c), d);
        for (int n = 0; n < 5; ++n) dU[n] += Fp[n] - Fm[n];
      }
      for (int d = 0; d < 3; ++d) {
        V5 um = cons_of(Wm[d][ic], c), up = cons_of(Wp[d][ic], c);
        for (int n = 0; n < 5; ++n) { um[n] -= c.hdtdh * dU[n]; up[n] -= c.hdtdh * dU[n]; }
        V5 wm = prim_of(um, c), wp = prim_of(up, c);
        apply_floor(wm, c);
        apply_floor(wp, c);
        Wm[d][ic] = wm;
        Wp[d][ic] = wp;
      }
    }
    for (int d = 0; d < 3; ++d) fr[d] = riemann_faces(g, Wp[d], Wm[d], hr, d, c, F[d]);
  } else if (c.scheme == S_VL) {
    // First-order predictor with the same Riemann solver on piecewise-constant data.
    Field F1[3];
    Range f1r[3];
    for (int d = 0; d < 3; ++d) {
      F1[d].resize(nc);
      f1r[d] = riemann_faces(g, W, W, all, d, c, F1[d]);
    }
    Range hr = intersect(intersect(diff_range(g, f1r[0], 0), diff_range(g, f1r[1], 1)), diff_range(g, f1r[2], 2));
    Field Wh(nc);
    FOR_RANGE(hr, i, j, k) {
      V5 dx = flux_diff(g, F1[0], 0, i, j, k);
      V5 dy = flux_diff(g, F1[1], 1, i, j, k);
      V5 dz = flux_diff(g, F1[2], 2, i, j, k);
      V5 u = U[g.at(i, j, k)];
      for (int n = 0; n < 5; ++n) u[n] -= c.hdtdh * (dx[n] + dy[n] + dz[n]);
      V5 w = prim_of(u, c);
      apply_floor(w, c);
      Wh[g.at(i, j, k)] = w;
    }
    Range sr[3];
    for (int d = 0; d < 3; ++d) sr[d] = face_states(g, Wh, hr, d, c, false, Wm[d], Wp[d]);
    for (int d = 0; d < 3; ++d) fr[d] = riemann_faces(g, Wp[d], Wm[d], sr[d], d, c, F[d]);
  } else {  // CTU
    Range sr[3];
    Field F1[3];
    Range f1r[3];
    for (int d = 0; d < 3; ++d) sr[d] = face_states(g, W, all, d, c, true, Wm[d], Wp[d]);
    for (int d = 0; d < 3; ++d) {
      F1[d].resize(nc);
      f1r[d] = riemann_faces(g, Wp[d], Wm[d], sr[d], d, c, F1[d]);
    }
    // Transverse flux-gradient correction of the half-step face states.
    Range cr[3];
    for (int d = 0; d < 3; ++d) {
      int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
      cr[d] = intersect(intersect(sr[d], diff_range(g, f1r[e1], e1)), diff_range(g, f1r[e2], e2));
    }
    Field Cm[3], Cp[3];
    for (int d = 0; d < 3; ++d) {
      Cm[d].resize(nc);
      Cp[d].resize(nc);
      int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
      FOR_RANGE(cr[d], i, j, k) {
        long ic = g.at(i, j, k);
        V5 t1 = flux_diff(g, F1[e1], e1, i, j, k);
        V5 t2 = flux_diff(g, F1[e2], e2, i, j, k);
        V5 um = cons_of(Wm[d][ic], c), up = cons_of(Wp[d][ic], c);
        for (int n = 0; n < 5; ++n) {
          real t = c.hdtdh * (t1[n] + t2[n]);
          um[n] -= t;
          up[n] -= t;
        }
        V5 wm = prim_of(um, c), wp = prim_of(up, c);
        apply_floor(wm, c);
        apply_floor(wp, c);
        Cm[d][ic] = wm;
        Cp[d][ic] = wp;
      }
    }
    for (int d = 0; d < 3; ++d) fr[d] = riemann_faces(g, Cp[d], Cm[d], cr[d], d, c, F[d]);
  }
  Range ur = intersect(intersect(diff_range(g, fr[0], 0), diff_range(g, fr[1], 1)), diff_range(g, fr[2], 2));
  conservative_update(g, U, F, ur, c, Unew);
  return ur;
}

static int make_cfg(Cfg& c, double dt, double dh, double gamma, int scheme, int recon, int riemann, int limiter,
                    int flags) {
  if (!(dt > 0.0) || !(dh > 0.0) || !(gamma > 1.0)) return -1;
  if (scheme < 0 || scheme > 2 || recon < 0 || recon > 1 || riemann < 0 || riemann > 3 || limiter < 0 ||
      limiter > L_CENTRAL)
    return -1;
  c.gamma = gamma;
  c.gm1 = gamma - 1.0;
  c.dtdh = dt / dh;
  c.hdtdh = 0.5 * dt / dh;
  c.theta = 1.5;
  c.floor = 1e-10;
  c.scheme = scheme;
  c.recon = recon;
  c.riemann = riemann;
  c.limiter = limiter;
  c.charlim = (flags & F_CHAR) != 0;
  c.fb_hllc = (flags & F_ROE_FB_HLLC) != 0;
  c.fb_exact = (flags & F_ROE_FB_EXACT) != 0;
  c.no_mono = (flags & F_NO_MONO) != 0;
  return 0;
}

static void load(const double* src, long nc, Field& U) {
  U.resize(nc);
  for (long q = 0; q < nc; ++q)
    for (int n = 0; n < 5; ++n) U[q][n] = src[n * nc + q];
}

extern "C" {

// Minimum ghost width for a scheme / reconstruction (stencil count).
int oracle_ghost_width(int scheme, int recon) {
  int r = (recon == R_PPM) ? 2 : 1;
  return (scheme == S_VL) ? r + 2 : r + 1;
}

// One step on a periodic box [5][nz][ny][nx] -> same shape.
int oracle_step_box(const double* U_in, double* U_out, int nx, int ny, int nz, double dt, double dh,
                    double gamma, int scheme, int recon, int riemann, int limiter, int flags) {
  Cfg c;
  if (make_cfg(c, dt, dh, gamma, scheme, recon, riemann, limiter, flags)) return -1;
  Grid g = {{nx, ny, nz}, true};
  long nc = g.ncell();
  Field U, Unew(nc), F[3];
  load(U_in, nc, U);
  scheme_step(g, U, c, Unew, F);
  for (long q = 0; q < nc; ++q)
    for (int n = 0; n < 5; ++n) U_out[n * nc + q] = to_d(Unew[q][n]);
  return 0;
}

// One step on a batch of padded patch groups.
//   in   [n_groups][5][N][N][N], N = 16 + 2 g
//   out  [n_groups][5][16][16][16]
//   flux [n_groups][3][nf][5][16][16] or NULL; nf = 2 (faces -,+) or 3 with
//        the internal mid plane (flag 0x04) stored after the two faces.
//        Transverse index order (slow, fast): x faces (z,y), y faces (z,x),
//        z faces (y,x).  The physical flux F is stored (not F*dt).
int oracle_solve_groups(const double* in, double* out, double* flux, int n_groups, int g, double dt, double dh,
                        double gamma, int scheme, int recon, int riemann, int limiter, int flags) {
  Cfg c;
  if (make_cfg(c, dt, dh, gamma, scheme, recon, riemann, limiter, flags)) return -1;
  if (g < oracle_ghost_width(scheme, recon)) return -2;
  const int N = 16 + 2 * g;
  Grid gr = {{N, N, N}, false};
  long nc = gr.ncell();
  const int nf = (flags & F_FLUX_MID) ? 3 : 2;
  for (int q = 0; q < n_groups; ++q) {
    Field U, Unew(nc), F[3];
    load(in + (long)q * 5 * nc, nc, U);
    Range ur = scheme_step(gr, U, c, Unew, F);
    for (int a = 0; a < 3; ++a)
      if (ur.lo[a] > g || ur.hi[a] < g + 16) {
        std::fprintf(stderr, "oracle: ghost width %d too small\n", g);
        std::abort();
      }
    double* o = out + (long)q * 5 * 4096;
    for (int k = 0; k < 16; ++k)
      for (int j = 0; j < 16; ++j)
        for (int i = 0; i < 16; ++i)
          for (int n = 0; n < 5; ++n)
            o[n * 4096 + (k * 16 + j) * 16 + i] = to_d(Unew[gr.at(i + g, j + g, k + g)][n]);
    if (flux) {
      double* fo = flux + (long)q * 3 * nf * 5 * 256;
      // Face positions as offsets from the first interior cell: the face
      // between interior cells s-1 and s is stored at face index g+s-1.
      const int off[3] = {0, 16, 8};
      for (int d = 0; d < 3; ++d)
        for (int f = 0; f < nf; ++f)
          for (int a = 0; a < 16; ++a)      // slow transverse index
            for (int b = 0; b < 16; ++b) {  // fast transverse index
              int idx[3];
              int fi = g + off[f] - 1;
              if (d == 0) { idx[0] = fi; idx[1] = b + g; idx[2] = a + g; }
              else if (d == 1) { idx[0] = b + g; idx[1] = fi; idx[2] = a + g; }
              else { idx[0] = b + g; idx[1] = a + g; idx[2] = fi; }
              const V5& v = F[d][gr.at(idx[0], idx[1], idx[2])];
              for (int n = 0; n < 5; ++n)
                fo[(((long)d * nf + f) * 5 + n) * 256 + a * 16 + b] = to_d(v[n]);
            }
    }
  }
  return 0;
}

// Periodic ghost fill: box [5][nz][ny][nx] (multiples of 16) -> groups
// [G][5][N][N][N], group G = (gz*ngy + gy)*ngx + gx.
int oracle_fill_ghosts_periodic(const double* box, int nx, int ny, int nz, int g, double* groups) {
  if (nx % 16 || ny % 16 || nz % 16 || g < 0) return -1;
  int ngx = nx / 16, ngy = ny / 16, ngz = nz / 16, N = 16 + 2 * g;
  Grid b = {{nx, ny, nz}, true};
  long nc = b.ncell(), gc = (long)N * N * N;
  for (int gz = 0; gz < ngz; ++gz)
    for (int gy = 0; gy < ngy; ++gy)
      for (int gx = 0; gx < ngx; ++gx) {
        double* o = groups + (long)((gz * ngy + gy) * ngx + gx) * 5 * gc;
        for (int k = 0; k < N; ++k)
          for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
              long s = b.at(gx * 16 + i - g, gy * 16 + j - g, gz * 16 + k - g);
              for (int n = 0; n < 5; ++n) o[n * gc + ((long)k * N + j) * N + i] = box[n * nc + s];
            }
      }
  return 0;
}

// AMR-shaped groups: each padded-group cell is the trilinear interpolation,
// at its centre, of a periodic coarse field [5][cn][cn][cn] on the unit box
// (spatial interpolation at coarse-fine boundaries, Sec. 4.2).  layout[G] =
// (level, ox, oy, oz), the first interior cell on the level grid with
// spacing base_dh / 2^level.
int oracle_fill_groups_interp(const double* coarse, int cn, const int* layout, int n_groups, int g, double base_dh,
                              double* groups) {
  int N = 16 + 2 * g;
  long gc = (long)N * N * N, cc = (long)cn * cn * cn;
  for (int G = 0; G < n_groups; ++G) {
    const int* L = layout + 4 * G;
    double dh = base_dh / (double)(1 << L[0]);
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
          // position of the cell centre in units of coarse cells, relative to coarse centres
          double pos[3] = {((double)(L[1] + i - g) + 0.5) * dh * cn - 0.5,
                           ((double)(L[2] + j - g) + 0.5) * dh * cn - 0.5,
                           ((double)(L[3] + k - g) + 0.5) * dh * cn - 0.5};
          int lo[3], hi[3];
          double w[3];
          for (int a = 0; a < 3; ++a) {
            double f = std::floor(pos[a]);
            w[a] = pos[a] - f;
            int l = (int)f;
            lo[a] = ((l % cn) + cn) % cn;
            hi[a] = (lo[a] + 1) % cn;
          }
          for (int n = 0; n < 5; ++n) {
            const double* c = coarse + n * cc;
            double v = 0.0;
            for (int dz = 0; dz < 2; ++dz)
              for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                  double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
                  long q = ((long)(dz ? hi[2] : lo[2]) * cn + (dy ? hi[1] : lo[1])) * cn + (dx ? hi[0] : lo[0]);
                  v += wt * c[q];
                }
            groups[(long)G * 5 * gc + n * gc + ((long)k * N + j) * N + i] = v;
          }
        }
  }
  return 0;
}

// AMR preparation step for groups next to coarse-fine boundaries (Sec. 4.2:
// ghost data by spatial and temporal interpolation).  Group G of level l =
// layout[G][0] covers interior cells layout[G][1..3] + [0, 16) of the level
// grid, which spans the periodic unit box with nl = 16 * (ng0 << l) cells per
// side.  Each cell of its padded region [5][N][N][N] (N = 16 + 2g) is
//  * an interior cell: the group's own value from fine[G];
//  * a ghost cell covered by another group of the same level: that group's
//    value (where several groups cover it, the highest index);
//  * any other ghost cell: the coarse state at the fine sub-step time,
//    (1 - alpha_l) * coarse0 + alpha_l * coarse1 at the coarse cell centres,
//    interpolated trilinearly to the fine cell centre (as
//    oracle_fill_groups_interp, with base_dh = 1 / (16 ng0)).
// fine: [n][5][16][16][16]; coarse0/1: [5][cn][cn][cn]; alpha: [n_levels].
int oracle_fill_groups_amr(const double* fine, const int* layout, int n_groups, int ng0, int n_levels,
                           const double* coarse0, const double* coarse1, int cn, const double* alpha, int g,
                           double* groups) {
  if (ng0 <= 0 || n_levels <= 0 || cn <= 0 || g < 0) return -1;
  const int N = 16 + 2 * g;
  const long gc = (long)N * N * N, cc = (long)cn * cn * cn;
  for (int G = 0; G < n_groups; ++G) {
    const int* L = layout + 4 * G;
    const int lev = L[0];
    if (lev < 0 || lev >= n_levels) return -1;
    const int nl = 16 * (ng0 << lev);
    for (int a = 1; a <= 3; ++a)
      if (L[a] < 0 || L[a] >= nl || L[a] % 16) return -1;  // group origins on the level's 16-cell grid
    const double dh = 1.0 / (double)nl;
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
          double* o = groups + (long)G * 5 * gc + ((long)k * N + j) * N + i;
          const int ci = i - g, cj = j - g, ck = k - g;
          if (ci >= 0 && ci < 16 && cj >= 0 && cj < 16 && ck >= 0 && ck < 16) {
            for (int n = 0; n < 5; ++n) o[n * gc] = fine[((long)G * 5 + n) * 4096 + (ck * 16 + cj) * 16 + ci];
            continue;
          }
          // Level-grid cell (periodic) and the same-level group covering it.
          const int p[3] = {((L[1] + ci) % nl + nl) % nl, ((L[2] + cj) % nl + nl) % nl, ((L[3] + ck) % nl + nl) % nl};
          int owner = -1;
          for (int H = 0; H < n_groups; ++H) {
            const int* M = layout + 4 * H;
            if (M[0] != lev) continue;
            bool in = true;
            for (int a = 0; a < 3; ++a) in = in && p[a] >= M[1 + a] && p[a] < M[1 + a] + 16;
            if (in) owner = H;  // highest index wins
          }
          if (owner >= 0) {
            const int* M = layout + 4 * owner;
            const long c = ((long)(p[2] - M[3]) * 16 + (p[1] - M[2])) * 16 + (p[0] - M[1]);
            for (int n = 0; n < 5; ++n) o[n * gc] = fine[((long)owner * 5 + n) * 4096 + c];
            continue;
          }
          const double pos[3] = {((double)(L[1] + ci) + 0.5) * dh * cn - 0.5, ((double)(L[2] + cj) + 0.5) * dh * cn - 0.5,
                                 ((double)(L[3] + ck) + 0.5) * dh * cn - 0.5};
          int lo[3], hi[3];
          double w[3];
          for (int a = 0; a < 3; ++a) {
            const double f = std::floor(pos[a]);
            w[a] = pos[a] - f;
            const int l = (int)f;
            lo[a] = ((l % cn) + cn) % cn;
            hi[a] = (lo[a] + 1) % cn;
          }
          const double al = alpha[lev];
          for (int n = 0; n < 5; ++n) {
            double v = 0.0;
            for (int dz = 0; dz < 2; ++dz)
              for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                  const double wt = (dx ? w[0] : 1.0 - w[0]) * (dy ? w[1] : 1.0 - w[1]) * (dz ? w[2] : 1.0 - w[2]);
                  const long q = n * cc + ((long)(dz ? hi[2] : lo[2]) * cn + (dy ? hi[1] : lo[1])) * cn +
                                 (dx ? hi[0] : lo[0]);
                  v += wt * ((1.0 - al) * coarse0[q] + al * coarse1[q]);
                }
            o[n * gc] = v;
          }
        }
  }
  return 0;
}

// Coarse-grid correction (Sec. 2 step 5, Sec. 4.3): after one step of a
// periodic coarse box and the sub-steps of refined groups of ratio 2, every
// fine group covering exactly one coarse patch (8^3 coarse cells: fine
// origin (ox, oy, oz) on the fine grid, multiples of 16):
//  * refluxing: an uncovered coarse cell a whose neighbour b across a face
//    is covered by fine group F had its update formed with the coarse flux
//    Fc of that face; it is corrected to the mean Ff of the four fine fluxes
//    on the same face (F's face towards a, averaged over the sub-steps by
//    the caller): U_a -= dt/dh (Ff - Fc) if b lies on a's + side,
//    U_a += dt/dh (Ff - Fc) if on its - side (directions x, y, z, sides -, +
//    in that order);
//  * restriction: a covered coarse cell becomes the mean of its 8 children.
// coarse: [Gc][5][16][16][16] in patch-group order of an nx x ny x nz box;
// cflux: [Gc][3][3][5][16][16] (faces -, +, mid at offset 8; transverse
// indices (z, y), (z, x), (y, x)); fine: [nf][5][16][16][16]; flayout:
// [nf][4] (unused, ox, oy, oz); fflux: [nf][3][2][5][16][16].
int oracle_amr_correct(double* coarse, int nx, int ny, int nz, const double* cflux, const double* fine,
                       const int* flayout, int nf, const double* fflux, double dt, double dh) {
  if (nx % 16 || ny % 16 || nz % 16) return -1;
  const int n3[3] = {nx, ny, nz};
  const int ngx = nx / 16, ngy = ny / 16;
  for (int F = 0; F < nf; ++F)
    for (int a = 1; a <= 3; ++a)
      if (flayout[4 * F + a] % 16 || flayout[4 * F + a] < 0 || flayout[4 * F + a] >= 2 * n3[a - 1]) return -1;
  auto cell = [&](int x, int y, int z, int n) -> double& {
    const long G = ((long)(z / 16) * ngy + y / 16) * ngx + x / 16;
    return coarse[(G * 5 + n) * 4096 + ((z % 16) * 16 + (y % 16)) * 16 + x % 16];
  };
  auto owner = [&](const int c[3]) -> int {  // fine group covering coarse cell c, or -1
    int o = -1;
    for (int F = 0; F < nf; ++F) {
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        const int lo = flayout[4 * F + 1 + a] / 2;
        in = in && c[a] >= lo && c[a] < lo + 8;
      }
      if (in) o = F;
    }
    return o;
  };
  // Refluxing (uncovered cells only; increments do not depend on U).
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int c[3] = {x, y, z};
        if (owner(c) >= 0) continue;
        const long G = ((long)(z / 16) * ngy + y / 16) * ngx + x / 16;
        for (int d = 0; d < 3; ++d)
          for (int side = -1; side <= 1; side += 2) {
            int b[3] = {x, y, z};
            b[d] = (b[d] + side + n3[d]) % n3[d];
            const int F = owner(b);
            if (F < 0) continue;
            // transverse coordinates (slow, fast) of the face: x (z, y), y (z, x), z (y, x)
            const int ts = d == 2 ? 1 : 2, tf = d == 0 ? 1 : 0;
            const int loc = c[d] % 16;
            int slot;
            if (side > 0) slot = loc == 15 ? 1 : (loc == 7 ? 2 : -1);
            else slot = loc == 0 ? 0 : (loc == 8 ? 2 : -1);
            if (slot < 0) return -2;  // fine coverage off the coarse patch grid
            const int fo[3] = {flayout[4 * F + 1], flayout[4 * F + 2], flayout[4 * F + 3]};
            const int fs0 = 2 * (c[ts] - fo[ts] / 2), ff0 = 2 * (c[tf] - fo[tf] / 2);
            const int fslot = side > 0 ? 0 : 1;  // F's face towards a
            for (int n = 0; n < 5; ++n) {
              const double Fc = cflux[((((G * 3 + d) * 3 + slot) * 5 + n) * 16 + c[ts] % 16) * 16 + c[tf] % 16];
              double Ff = 0.0;
              for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                  Ff += fflux[((((long)(F * 3 + d) * 2 + fslot) * 5 + n) * 16 + fs0 + i) * 16 + ff0 + j];
              Ff *= 0.25;
              cell(x, y, z, n) += (side > 0 ? -1.0 : 1.0) * (dt / dh) * (Ff - Fc);
            }
          }
      }
  // Restriction.
  for (int F = 0; F < nf; ++F) {
    const int* o = flayout + 4 * F;
    for (int k = 0; k < 8; ++k)
      for (int j = 0; j < 8; ++j)
        for (int i = 0; i < 8; ++i)
          for (int n = 0; n < 5; ++n) {
            double s = 0.0;
            for (int dz = 0; dz < 2; ++dz)
              for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx)
                  s += fine[((long)F * 5 + n) * 4096 + ((2 * k + dz) * 16 + 2 * j + dy) * 16 + 2 * i + dx];
            cell(o[1] / 2 + i, o[2] / 2 + j, o[3] / 2 + k, n) = 0.125 * s;
          }
  }
  return 0;
}

// CFL time step from conserved cells (any layout; n_cells cells per
// variable-plane, n_blocks blocks of [5][n_cells]):
//   dt = cfl * dh / max over cells of max_d(|v_d| + c).
double oracle_cfl_dt(const double* U, long n_blocks, long n_cells, double dh, double gamma, double cfl) {
  double smax = 0.0;
  for (long b = 0; b < n_blocks; ++b) {
    const double* u = U + b * 5 * n_cells;
    for (long q = 0; q < n_cells; ++q) {
      double rho = u[q];
      double vx = u[n_cells + q] / rho;
      double vy = u[2 * n_cells + q] / rho;
      double vz = u[3 * n_cells + q] / rho;
      double ke = 0.5 * (u[n_cells + q] * vx + u[2 * n_cells + q] * vy + u[3 * n_cells + q] * vz);
      double p = (gamma - 1.0) * (u[4 * n_cells + q] - ke);
      double cs = std::sqrt(gamma * p / rho);
      double av = std::fabs(vx);
      if (std::fabs(vy) > av) av = std::fabs(vy);
      if (std::fabs(vz) > av) av = std::fabs(vz);
      double s = av + cs;
      if (s > smax) smax = s;
    }
  }
  return cfl * dh / smax;
}

// Conserved sums: sums[v] = dh^3 * sum over cells of U_v (plain summation).
void oracle_conserved_sums(const double* U, long n_blocks, long n_cells, double dh, double* sums) {
  double vol = dh * dh * dh;
  for (int n = 0; n < 5; ++n) {
    double s = 0.0;
    for (long b = 0; b < n_blocks; ++b) {
      const double* u = U + (b * 5 + n) * n_cells;
      for (long q = 0; q < n_cells; ++q) s += u[q];
    }
    sums[n] = s * vol;
  }
}

// ---- single-function entry points used by the pins ----------------------

// Riemann flux in direction d (0,1,2) between lab-frame primitive states.
int oracle_riemann_flux(const double* WL, const double* WR, int d, double gamma, int riemann, int flags,
                        double* F) {
  Cfg c;
  if (make_cfg(c, 1.0, 1.0, gamma, 0, 0, riemann, 0, flags)) return -1;
  V5 L, R;
  for (int n = 0; n < 5; ++n) { L[n] = WL[n]; R[n] = WR[n]; }
  V5 f = from_frame(riemann_solve(to_frame(L, d), to_frame(R, d), c), d);
  for (int n = 0; n < 5; ++n) F[n] = to_d(f[n]);
  return 0;
}
// Roe solve only: returns 1 if the linearization is accepted, 0 if it fails.
int oracle_roe_ok(const double* WL, const double* WR, double gamma) {
  Cfg c;
  make_cfg(c, 1.0, 1.0, gamma, 0, 0, 0, 0, 0);
  V5 L, R, F;
  for (int n = 0; n < 5; ++n) { L[n] = WL[n]; R[n] = WR[n]; }
  return flux_roe(L, R, c, F) ? 1 : 0;
}
// Exact solution of the 1D Riemann problem along x: star values
// (p*, u*, rho*_L, rho*_R, ok) and samples at n_xi points xi[] -> W[n_xi][5].
int oracle_exact_riemann(const double* WL, const double* WR, double gamma, double* star, const double* xi,
                         int n_xi, double* W) {
  Cfg c;
  make_cfg(c, 1.0, 1.0, gamma, 0, 0, 3, 0, 0);
  V5 L, R;
  for (int n = 0; n < 5; ++n) { L[n] = WL[n]; R[n] = WR[n]; }
  ExactStar s = exact_star(L, R, c);
  star[0] = to_d(s.p); star[1] = to_d(s.u); star[2] = to_d(s.rhoL); star[3] = to_d(s.rhoR); star[4] = s.ok;
  for (int q = 0; q < n_xi; ++q) {
    V5 w = exact_sample(L, R, s, xi[q], c);
    for (int n = 0; n < 5; ++n) W[q * 5 + n] = to_d(w[n]);
  }
  return s.ok ? 0 : -1;
}
double oracle_limiter(double dl, double dr, int limiter) {
  Cfg c;
  make_cfg(c, 1.0, 1.0, 1.4, 0, 0, 0, limiter, 0);
  return to_d(limit_slope(dl, dr, c));
}
// Limited slope of the middle of three lab-frame states along d.
void oracle_slope(const double* wm, const double* w0, const double* wp, int d, double gamma, int limiter,
                  int flags, double* s) {
  Cfg c;
  make_cfg(c, 1.0, 1.0, gamma, 0, 0, 0, limiter, flags);
  V5 a, b, e;
  for (int n = 0; n < 5; ++n) { a[n] = wm[n]; b[n] = w0[n]; e[n] = wp[n]; }
  V5 r = from_frame(limited_slope(to_frame(a, d), to_frame(b, d), to_frame(e, d), c), d);
  for (int n = 0; n < 5; ++n) s[n] = to_d(r[n]);
}
// PPM edge between a and b from given slopes (no limiting applied here).
void oracle_ppm_edge(const double* wa, const double* wb, const double* sa, const double* sb, double* e) {
  V5 a, b, x, y;
  for (int n = 0; n < 5; ++n) { a[n] = wa[n]; b[n] = wb[n]; x[n] = sa[n]; y[n] = sb[n]; }
  V5 r = ppm_edge(a, b, x, y);
  for (int n = 0; n < 5; ++n) e[n] = to_d(r[n]);
}
// Characteristic projection and expansion at a frame-ordered state.
void oracle_char(const double* w, const double* dw, double gamma, double* a, double* back) {
  Cfg c;
  make_cfg(c, 1.0, 1.0, gamma, 0, 0, 0, 0, 0);
  V5 W, D;
  for (int n = 0; n < 5; ++n) { W[n] = w[n]; D[n] = dw[n]; }
  real cs = sound_speed(W, c);
  V5 A = char_project(W, cs, D);
  V5 B = char_expand(W, cs, A);
  for (int n = 0; n < 5; ++n) { a[n] = to_d(A[n]); back[n] = to_d(B[n]); }
}

// Characteristic tracing of one cell (CTU step (1)) in the frame of its
// direction (normal velocity first): cell state w, face values wl (left face)
// and wr (right face) from the reconstruction, Courant factor dtdh = dt/dh.
// ppm = 1 uses the parabola through wl, wr with mean w (W6 from ppm_w6);
// ppm = 0 the linear profile from wl to wr.  Writes the half-step states at
// the left face (out_l) and the right face (out_r); no floors are applied.
void oracle_ctu_trace(const double* w, const double* wl, const double* wr, int ppm, double dtdh, double gamma,
                      double* out_l, double* out_r) {
  Cfg c;
  make_cfg(c, dtdh, 1.0, gamma, S_CTU, ppm ? R_PPM : R_PLM, 0, 0, 0);
  V5 W, L, R, w6;
  for (int n = 0; n < 5; ++n) { W[n] = w[n]; L[n] = wl[n]; R[n] = wr[n]; w6[n] = 0.0; }
  if (ppm) w6 = ppm_w6(W, L, R);
  ctu_trace(W, L, R, w6, ppm != 0, c);
  for (int n = 0; n < 5; ++n) { out_l[n] = to_d(L[n]); out_r[n] = to_d(R[n]); }
}
// PPM parabola monotonization of one cell (per component, in place).
void oracle_ppm_monotonize(const double* w, double* wl, double* wr) {
  V5 W, L, R;
  for (int n = 0; n < 5; ++n) { W[n] = w[n]; L[n] = wl[n]; R[n] = wr[n]; }
  ppm_monotonize(W, L, R);
  for (int n = 0; n < 5; ++n) { wl[n] = to_d(L[n]); wr[n] = to_d(R[n]); }
}

void oracle_reset_stats(void) { std::memset(&g_stats, 0, sizeof(g_stats)); }
void oracle_get_stats(long long* out) {
  out[0] = g_stats.solves;
  out[1] = g_stats.roe_fail;
  out[2] = g_stats.floor_hits;
  out[3] = g_stats.exact_fail;
}
unsigned long long oracle_get_ops(void) {
#ifdef ORACLE_COUNT_OPS
  return g_ops;
#else
  return 0ULL;
#endif
}
void oracle_reset_ops(void) {
#ifdef ORACLE_COUNT_OPS
  g_ops = 0;
#endif
}

}  // extern "C"
