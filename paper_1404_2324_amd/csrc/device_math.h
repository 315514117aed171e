// Device-side FP64 building blocks of the hybrid symplectic step
// (Grimm & Stadel, "The GENGA Code", arXiv:1404.2324), written for gfx950.
// Included by every kernel translation unit of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace genga {

constexpr double kTiny = 2.2250738585072014e-308;  // smallest normal double

// ---- wave helpers (wave64) -------------------------------------------------
__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 p = *reinterpret_cast<int2*>(&v);
  int lo = __builtin_amdgcn_readlane(p.x, lane);
  int hi = __builtin_amdgcn_readlane(p.y, lane);
  int2 q = make_int2(lo, hi);
  return *reinterpret_cast<double*>(&q);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

// ---- reciprocal square root ------------------------------------------------
// 1/sqrt(x) for positive normal x: the hardware estimate y (24.2 bits
// measured) refined by one step of third order on the residual
// e = 1 - x y^2 (evaluated with FMA): y (1 + e/2 + 3 e^2/8), the Taylor
// series of y / sqrt(1 - e), leaves an error of order e^3 (~2^-72).
// Measured on gfx950 over 4M arguments spanning 16 decades: max error
// 0.991 ulp, mean signed error -2e-4 ulp, 13.5 % of results beyond 0.5 ulp
// (two Newton steps: 0.996 ulp, 1e-4, 13.5 %), i.e. as accurate as before
// with six FP64 instructions instead of eight and a shorter dependency
// chain.  x = 0 gives NaN (callers mask that case).
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// m / r^3 from r2 = r^2 (positive normal): with the hardware estimate y of
// 1/sqrt(r2) and its residual e = 1 - r2 y^2, r^-3 = y^3 (1 - e)^(-3/2),
// summed to second order, m y^3 (1 + 3e/2 + 15e^2/8): the next term,
// 35e^3/16, is ~2^-71 for the 24-bit estimate.  Eight FP64 instructions
// against nine for the refined 1/sqrt cubed and scaled, and a shorter
// dependency chain.  r2 = 0 gives NaN or infinity (callers mask that case).
// c1875 = 1.875 and c15 = 1.5 may be passed in registers that a caller's
// loop holds (this target's three-operand FMA takes no literal operand).
__device__ __forceinline__ double m_rinv3(double m, double r2, double c1875 = 1.875,
                                          double c15 = 1.5) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double my3 = (m * y) * y2;
  return fma(my3, e * fma(e, c1875, c15), my3);
}

// 1/x for x in a bounded, well-scaled range (no zero, infinity or denormal):
// the hardware estimate y (24.4 bits measured) refined by one step of third
// order on e = 1 - x y: y (1 + e + e^2), the series of y / (1 - e), leaves an
// error of order e^3.  Measured on gfx950 over 4M arguments in [1/2, 1] and
// 4M in [1e-6, 1e6]: every result within 0.5 ulp (correctly rounded), as
// with two Newton steps, with one dependent operation fewer.
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y, 1.0);
  return fma(y * e, 1.0 + e, y);
}

// ---- changeover function, Eq. (4)-(5) ---------------------------------------
// K(y) = 0 (y <= 0), y^2/(2y^2-2y+1) (0<y<1), 1 (y >= 1),
// y = (r - 0.1 rc) / (0.9 rc); returns K and dK/dr.  rc <= 0: no changeover.
__device__ __forceinline__ void changeover(double r, double rc, double& K,
                                           double& dKdr) {
  if (!(rc > 0.0)) {
    K = 1.0;
    dKdr = 0.0;
    return;
  }
  // the reciprocals by rcp_nr (correctly rounded for these well-scaled
  // arguments, as the division; 0.9 rc is a length of order 1e-4..1, D is in
  // [1/2, 1])
  const double inv = rcp_nr(0.9 * rc);
  const double y = (r - 0.1 * rc) * inv;
  if (y <= 0.0) {
    K = 0.0;
    dKdr = 0.0;
  } else if (y >= 1.0) {
    K = 1.0;
    dKdr = 0.0;
  } else {
    const double D = 2.0 * y * y - 2.0 * y + 1.0;
    const double iD = rcp_nr(D);
    K = y * y * iD;
    dKdr = 2.0 * y * (1.0 - y) * iD * iD * inv;
  }
}

// Branch-free form for a known pair radius (i09 = 1/(0.9 rc)): clamping y to
// [0, 1] reproduces both constant branches exactly (K(0) = 0, K(1) = 1 and
// K' = 0 at both ends), and D = 2y^2 - 2y + 1 lies in [1/2, 1].
__device__ __forceinline__ void changeover_clamped(double r, double rc,
                                                   double i09, double& K,
                                                   double& dKdr) {
  const double y = fmin(fmax((r - 0.1 * rc) * i09, 0.0), 1.0);
  const double iD = rcp_nr(2.0 * y * y - 2.0 * y + 1.0);
  K = y * y * iD;
  dKdr = 2.0 * y * (1.0 - y) * iD * iD * i09;
}

// ---- critical radius, Eq. (6) ----------------------------------------------
// rc = max(n1 R_H, n2 |dt| |v|); R_H = a (m / 3 m0)^(1/3) with the osculating
// semi-major axis about mu = G m0 (heliocentric distance when unbound).
__device__ __forceinline__ double rcrit(double x, double y, double z, double vx,
                                        double vy, double vz, double m,
                                        double mu, double m0, double n1,
                                        double n2, double absdt) {
  const double r = sqrt(x * x + y * y + z * z);
  const double vv = vx * vx + vy * vy + vz * vz;
  const double inva = 2.0 / r - vv / mu;
  const double a = inva > 0.0 ? 1.0 / inva : r;
  const double rh = a * cbrt(m / (3.0 * m0));
  return fmax(n1 * rh, n2 * absdt * sqrt(vv));
}

// ---- Stumpff functions ------------------------------------------------------
// c_k(z) = sum_n (-z)^n/(k+2n)!.  Horner series of c2, c3 for |z| < 0.1
// (eight terms leave < 1e-20); larger |z| is quartered first and rebuilt with
// c0(4z)=2c0^2-1, c1(4z)=c0 c1, c2(4z)=c1^2/2, c3(4z)=(c2+c0 c3)/4.
__device__ __forceinline__ void stumpff(double z, double& c0, double& c1,
                                        double& c2, double& c3) {
  int nq = 0;
  while (fabs(z) >= 0.1 && nq < 64) {  // bounded: an infinite z must not spin
    z *= 0.25;
    ++nq;
  }
  c2 = 1.0 / 2.0 +
       z * (-1.0 / 24.0 +
            z * (1.0 / 720.0 +
                 z * (-1.0 / 40320.0 +
                      z * (1.0 / 3628800.0 +
                           z * (-1.0 / 479001600.0 +
                                z * (1.0 / 87178291200.0 +
                                     z * (-1.0 / 20922789888000.0)))))));
  c3 = 1.0 / 6.0 +
       z * (-1.0 / 120.0 +
            z * (1.0 / 5040.0 +
                 z * (-1.0 / 362880.0 +
                      z * (1.0 / 39916800.0 +
                           z * (-1.0 / 6227020800.0 +
                                z * (1.0 / 1307674368000.0 +
                                     z * (-1.0 / 355687428096000.0)))))));
  c0 = 1.0 - z * c2;
  c1 = 1.0 - z * c3;
  for (int q = 0; q < nq; ++q) {
    const double a0 = 2.0 * c0 * c0 - 1.0;
    const double a1 = c0 * c1;
    const double a2 = 0.5 * c1 * c1;
    const double a3 = 0.25 * (c2 + c0 * c3);
    c0 = a0;
    c1 = a1;
    c2 = a2;
    c3 = a3;
  }
}

// ---- Kepler drift in universal variables, Eq. (9) ---------------------------
// x = f x0 + g v0, v = fdot x0 + gdot v0 about mu = G m0.  The universal Kepler
// equation F(s) = r0 G1 + eta0 G2 + mu G3 - dt = 0 (G_k = s^k c_k(beta s^2),
// beta = 2 mu/r0 - v0^2) is solved by the Laguerre-Conway iteration of order
// 5 until |ds| <= 2^-50 |s| or |F| <= 2^-48 times the sum of the magnitudes
// of its terms (rounding floor).  The first guess inverts the cubic Taylor
// form dt = r0 s + eta0 s^2/2 + zeta0 s^3/6 (zeta0 = mu - beta r0) for s,
// s = t - eta0 t^2/(2 r0) + (eta0^2/2 - r0 zeta0/6) t^3/r0^2 with t = dt/r0,
// when its corrections are small against t (short steps); otherwise s = t.
// The Stumpff values of the last residual evaluation are reused for f and g
// when the iteration stopped there; 1/r0 and 1/r are formed once and
// multiplied in.  Returns the iteration count, or a
// negative count when max_iter was reached without convergence.
// s_out (optional) receives the converged universal anomaly s.
__device__ __forceinline__ int kepler_drift(double mu, double dt, double& x,
                                            double& y, double& z, double& vx,
                                            double& vy, double& vz,
                                            int max_iter, double* s_out = nullptr) {
  const double r0 = sqrt(x * x + y * y + z * z);
  const double ir0 = 1.0 / r0;
  const double eta0 = x * vx + y * vy + z * vz;
  const double beta = 2.0 * mu * ir0 - (vx * vx + vy * vy + vz * vz);
  const double zeta0 = mu - beta * r0;
  const double t = dt * ir0;
  const double k2 = -0.5 * eta0 * ir0 * t;
  const double k3 = (0.5 * eta0 * eta0 - r0 * zeta0 * (1.0 / 6.0)) * ir0 * ir0 * t * t;
  double s = (fabs(k2) + fabs(k3) <= 0.125) ? t * (1.0 + k2 + k3) : t;
  int it = 1;
  bool ok = false, fresh = false;  // fresh: c0..c3 belong to the current s
  double c0, c1, c2, c3;
  for (; it <= max_iter; ++it) {
    stumpff(beta * s * s, c0, c1, c2, c3);
    const double G1 = s * c1, G2 = s * s * c2, G3 = s * s * s * c3;
    const double F = r0 * G1 + eta0 * G2 + mu * G3 - dt;
    // residual already at the rounding level of its terms: s cannot improve
    const double Fs = fabs(r0 * G1) + fabs(eta0 * G2) + fabs(mu * G3) + fabs(dt);
    if (fabs(F) <= 0x1p-48 * Fs) {
      ok = true;
      fresh = true;
      break;
    }
    const double Fp = r0 + eta0 * G1 + zeta0 * G2;
    const double Fpp = eta0 * c0 + zeta0 * G1;
    const double disc = 16.0 * Fp * Fp - 20.0 * F * Fpp;
    const double sq = sqrt(fabs(disc));
    const double ds = -5.0 * F / (Fp + copysign(sq, Fp));
    s += ds;
    if (fabs(ds) <= 0x1p-50 * fabs(s)) {
      ok = true;
      break;
    }
  }
  if (s_out) *s_out = s;
  if (!fresh) stumpff(beta * s * s, c0, c1, c2, c3);
  const double G1 = s * c1, G2 = s * s * c2, G3 = s * s * s * c3;
  const double r = r0 + eta0 * G1 + zeta0 * G2;
  const double ir = 1.0 / r;
  const double f = 1.0 - mu * G2 * ir0;
  const double g = dt - mu * G3;
  const double fd = -mu * G1 * ir0 * ir;
  const double gd = 1.0 - mu * G2 * ir;
  const double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
  const double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy,
               nvz = fd * z + gd * vz;
  x = nx;
  y = ny;
  z = nz;
  vx = nvx;
  vy = nvy;
  vz = nvz;
  return ok ? it : -max_iter;
}

// ---- close-encounter test, Eqs. (10)-(12) -----------------------------------
// Minimum over t in [0,1] of the cubic Hermite interpolant of the squared
// separation; the stationary points solve a t^2 + b t + c = 0 with
// a = 6(P0-P1) + 3 dt (Pd0+Pd1) (derivative of Eq. 10; the printed sign of
// the Pd1 term is a typo), b = 6(P1-P0) - 2 dt (2 Pd0 + Pd1), c = dt Pd0.
__device__ __forceinline__ double hermite_P(double t, double dt, double P0,
                                            double P1, double Pd0, double Pd1) {
  const double u = 1.0 - t;
  return P0 * (1.0 + 2.0 * t) * u * u + P1 * t * t * (3.0 - 2.0 * t) +
         Pd0 * dt * t * u * u - Pd1 * dt * t * t * u;
}

__device__ __forceinline__ double hermite_dmin2(double dt, double dx0,
                                                double dy0, double dz0,
                                                double dvx0, double dvy0,
                                                double dvz0, double dx1,
                                                double dy1, double dz1,
                                                double dvx1, double dvy1,
                                                double dvz1) {
  const double P0 = dx0 * dx0 + dy0 * dy0 + dz0 * dz0;
  const double P1 = dx1 * dx1 + dy1 * dy1 + dz1 * dz1;
  const double Pd0 = 2.0 * (dx0 * dvx0 + dy0 * dvy0 + dz0 * dvz0);
  const double Pd1 = 2.0 * (dx1 * dvx1 + dy1 * dvy1 + dz1 * dvz1);
  const double a = 6.0 * (P0 - P1) + 3.0 * dt * (Pd0 + Pd1);
  const double b = 6.0 * (P1 - P0) - 2.0 * dt * (2.0 * Pd0 + Pd1);
  const double c = dt * Pd0;
  double best = fmin(P0, P1);
  double t1 = -1.0, t2 = -1.0;
  if (a != 0.0) {
    const double disc = b * b - 4.0 * a * c;
    if (disc >= 0.0) {
      const double q = -0.5 * (b + copysign(sqrt(disc), b));
      t1 = q / a;
      if (q != 0.0) t2 = c / q;
    }
  } else if (b != 0.0) {
    t1 = -c / b;
  }
  if (t1 > 0.0 && t1 < 1.0) best = fmin(best, hermite_P(t1, dt, P0, P1, Pd0, Pd1));
  if (t2 > 0.0 && t2 < 1.0) best = fmin(best, hermite_P(t2, dt, P0, P1, Pd0, Pd1));
  return best;
}

}  // namespace genga
