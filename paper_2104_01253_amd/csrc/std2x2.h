// Standard form of a real 2x2 Schur block, shared by the host Schur code (schur.cpp)
// and the batched restart's device Schur code (batched.hip).
#pragma once

#include <cmath>

#if defined(__HIP__)
#define DCGS2_HOST_DEVICE __host__ __device__
#else
#define DCGS2_HOST_DEVICE
#endif

namespace dcgs2 {

// Standard form of a real 2x2 block M = [a b; c d]: an orthogonal G = [cs -sn; sn cs]
// with M = G M' G^T, where M' = [a' b'; c' d'] has c' = 0 when the eigenvalues are real
// and a' = d', b' c' < 0 when they are a complex pair.
//
// Derivation used here: write M = m I + [t s; s -t] + r [0 1; -1 0] with m = (a+d)/2,
// t = (a-d)/2, s = (b+c)/2, r = (b-c)/2.  Conjugation by a rotation through theta
// leaves m and the skew part r unchanged and turns the symmetric traceless part's
// vector (t, s) = rho (cos phi, sin phi) into rho (cos(phi - 2 theta), sin(phi - 2 theta)),
// of the same length rho.  Then c' = s' - r and b' = s' + r, and the eigenvalues are
// m +- sqrt(delta), delta = t^2 + b c = rho^2 - r^2.
//   delta >= 0: choose s' = r (so c' = 0) and t' = +-sqrt(delta) (the sign of t, the
//               nearer target);
//   delta <  0: choose t' = 0 (so a' = d' = m) and s' = +-rho (the sign of s); then
//               b' c' = rho^2 - r^2 = delta < 0.
// theta is half the angle from (t', s') to (t, s); cs and sn follow from that angle's
// cosine and sine by the half-angle formulas, choosing the branch that does not
// divide by a small number.  M' is then formed explicitly and the entry that must
// vanish (c') or the two that must agree (a', d') are set exactly; when rounding
// turns a nearly double complex pair real, a second rotation triangularises it.
DCGS2_HOST_DEVICE inline void std2x2(double& a, double& b, double& c, double& d, double& cs, double& sn) {
  cs = 1.0;
  sn = 0.0;
  for (int pass = 0; pass < 2 && c != 0.0; ++pass) {
    const double m = 0.5 * (a + d), t = 0.5 * (a - d);
    const double s = 0.5 * (b + c), r = 0.5 * (b - c);
    const double rho = std::hypot(t, s);
    const double delta = t * t + b * c;
    double tp, sp;
    if (delta >= 0.0) {
      tp = std::copysign(std::sqrt(delta), t);
      sp = r;
    } else {
      tp = 0.0;
      sp = std::copysign(rho, s);
    }
    double gc = 1.0, gs = 0.0;               // rotation of this pass
    if (rho > 0.0) {
      // angle Delta = phi - phi' between (t, s) and (t', s') (both of length rho)
      const double cd = (t * tp + s * sp) / (rho * rho);
      const double sd = (s * tp - t * sp) / (rho * rho);
      if (cd >= 0.0) {
        gc = std::sqrt(0.5 * (1.0 + cd));
        gs = sd / (2.0 * gc);
      } else {
        gs = std::copysign(std::sqrt(0.5 * (1.0 - cd)), sd);
        gc = sd / (2.0 * gs);
      }
    }
    // M' = G^T M G
    const double ua = gc * a + gs * c, ub = gc * b + gs * d;
    const double la = -gs * a + gc * c, lb = -gs * b + gc * d;
    a = ua * gc + ub * gs;
    b = -ua * gs + ub * gc;
    c = la * gc + lb * gs;
    d = -la * gs + lb * gc;
    if (delta >= 0.0) {
      c = 0.0;
    } else {
      a = m;
      d = m;
    }
    const double ncs = cs * gc - sn * gs;    // accumulated G = G_1 G_2
    sn = sn * gc + cs * gs;
    cs = ncs;
    // a complex pair stays one when b' and c' have strictly opposite signs; otherwise
    // (rounding at a nearly double eigenvalue) the next pass finds delta >= 0
    if (delta < 0.0 && b != 0.0 && std::signbit(b) != std::signbit(c)) break;
  }
}

}  // namespace dcgs2
