// Exact Riemann solver for the ideal-gas Euler equations (arXiv:1103.3373,
// Sec. 2 lists it among the solvers: reference solutions and a fallback),
// following the standard construction in Toro, "Riemann Solvers and
// Numerical Methods for Fluid Dynamics", ch. 4:
//  * the star pressure p* is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0,
//    where f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the
//    rarefaction (isentropic) branch otherwise;
//  * Newton iteration from the primitive-variable (PVRS) estimate, bounded
//    below by 1e-8 min(p_L, p_R), until the relative change
//    2 |p_new - p| / (p_new + p) falls below 1e-15 (FP64) or 1e-6 (FP32),
//    at most 200 iterations;
//  * the flux is the physical flux of the self-similar solution sampled on
//    the face (x/t = 0).
// States are in the rotated frame (rho, u_n, u_t1, u_t2, p).  A pair that
// generates vacuum ((2/(gamma-1))(c_L + c_R) <= u_R - u_L) or does not
// converge is counted in *fails and sampled with p* = 0 (vacuum) or the
// last iterate.
#pragma once

#include "hydro_math.hpp"

namespace hy {

template <typename T> HY_DEV T xpow(T a, T b);
template <> HY_DEV double xpow<double>(double a, double b) { return pow(a, b); }
template <> HY_DEV float xpow<float>(float a, float b) { return powf(a, b); }

template <typename T>
HY_DEV void exact_pfun(T p, T rk, T pk, T ck, const Phys<T>& ph, T& f, T& df) {
  const T gp1 = ph.gamma + T(1);
  if (p > pk) {  // shock
    const T A = T(2) / (gp1 * rk);
    const T B = ph.gm1 / gp1 * pk;
    const T q = sqrt(A / (p + B));
    f = (p - pk) * q;
    df = q * (T(1) - T(0.5) * (p - pk) / (B + p));
  } else {  // rarefaction
    const T pr = p / pk;
    f = T(2) * ck / ph.gm1 * (xpow<T>(pr, ph.gm1 / (T(2) * ph.gamma)) - T(1));
    df = T(1) / (rk * ck) * xpow<T>(pr, -gp1 / (T(2) * ph.gamma));
  }
}

template <typename T>
HY_DEV V5<T> exact_flux(const V5<T>& L, const V5<T>& R, const Phys<T>& ph, int* fails) {
  const T gp1 = ph.gamma + T(1);
  const T cL = sqrt(ph.gamma * L[4] / L[0]), cR = sqrt(ph.gamma * R[4] / R[0]);
  const T du = R[1] - L[1];
  T p, u, rhoL, rhoR;
  if (T(2) / ph.gm1 * (cL + cR) <= du) {  // vacuum is generated
    ++*fails;
    p = T(0);
    u = T(0.5) * (L[1] + R[1]);
    rhoL = rhoR = T(0);
  } else {
    const T ppv = T(0.5) * (L[4] + R[4]) - T(0.125) * du * (L[0] + R[0]) * (cL + cR);
    p = fmax(ppv, T(1e-8) * fmin(L[4], R[4]));
    const T tol = sizeof(T) == 8 ? T(1e-15) : T(1e-6);
    int it = 0;
    for (; it < 200; ++it) {
      T fL, dL, fR, dR;
      exact_pfun(p, L[0], L[4], cL, ph, fL, dL);
      exact_pfun(p, R[0], R[4], cR, ph, fR, dR);
      T pn = p - (fL + fR + du) / (dL + dR);
      if (pn < T(0)) pn = T(1e-12) * p;
      const T ch = T(2) * fabs(pn - p) / (pn + p);
      p = pn;
      if (ch < tol) break;
    }
    if (it >= 200) ++*fails;
    T fL, dL, fR, dR;
    exact_pfun(p, L[0], L[4], cL, ph, fL, dL);
    exact_pfun(p, R[0], R[4], cR, ph, fR, dR);
    u = T(0.5) * (L[1] + R[1]) + T(0.5) * (fR - fL);
    const T g6 = ph.gm1 / gp1;
    rhoL = p > L[4] ? L[0] * (p / L[4] + g6) / (g6 * p / L[4] + T(1)) : L[0] * xpow<T>(p / L[4], T(1) / ph.gamma);
    rhoR = p > R[4] ? R[0] * (p / R[4] + g6) / (g6 * p / R[4] + T(1)) : R[0] * xpow<T>(p / R[4], T(1) / ph.gamma);
  }
  // Sample the solution on the face, x/t = 0.
  V5<T> W;
  if (T(0) <= u) {  // left of the contact
    W = L;
    if (p > L[4]) {  // left shock
      const T SL = L[1] - cL * sqrt(gp1 / (T(2) * ph.gamma) * p / L[4] + ph.gm1 / (T(2) * ph.gamma));
      if (!(T(0) <= SL)) { W[0] = rhoL; W[1] = u; W[4] = p; }
    } else {  // left rarefaction
      const T csL = cL * xpow<T>(p / L[4], ph.gm1 / (T(2) * ph.gamma));
      const T head = L[1] - cL, tail = u - csL;
      if (T(0) <= head) {
      } else if (T(0) > tail) {
        W[0] = rhoL; W[1] = u; W[4] = p;
      } else {  // inside the fan
        const T b = T(2) / gp1 + ph.gm1 / (gp1 * cL) * L[1];
        W[0] = L[0] * xpow<T>(b, T(2) / ph.gm1);
        W[1] = T(2) / gp1 * (cL + T(0.5) * ph.gm1 * L[1]);
        W[4] = L[4] * xpow<T>(b, T(2) * ph.gamma / ph.gm1);
      }
    }
  } else {  // right of the contact
    W = R;
    if (p > R[4]) {  // right shock
      const T SR = R[1] + cR * sqrt(gp1 / (T(2) * ph.gamma) * p / R[4] + ph.gm1 / (T(2) * ph.gamma));
      if (!(T(0) >= SR)) { W[0] = rhoR; W[1] = u; W[4] = p; }
    } else {  // right rarefaction
      const T csR = cR * xpow<T>(p / R[4], ph.gm1 / (T(2) * ph.gamma));
      const T head = R[1] + cR, tail = u + csR;
      if (T(0) >= head) {
      } else if (T(0) < tail) {
        W[0] = rhoR; W[1] = u; W[4] = p;
      } else {
        const T b = T(2) / gp1 - ph.gm1 / (gp1 * cR) * R[1];
        W[0] = R[0] * xpow<T>(b, T(2) / ph.gm1);
        W[1] = T(2) / gp1 * (-cR + T(0.5) * ph.gm1 * R[1]);
        W[4] = R[4] * xpow<T>(b, T(2) * ph.gamma / ph.gm1);
      }
    }
  }
  return flux_of(W, ph);
}

}  // namespace hy
