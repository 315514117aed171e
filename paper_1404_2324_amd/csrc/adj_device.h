// Device pieces shared by the two adjoints (adj.hip, hadj.hip): the
// vector-Jacobian product of the Kepler drift in universal variables.
#pragma once

#include "device_math.h"

namespace genga {

// Stumpff c4, c5 next to c2, c3 (c_k = 1/k! - z c_{k+2}); series for |z| < 1.
__device__ __forceinline__ void stumpff45(double z, double c2, double c3, double& c4,
                                          double& c5) {
  if (fabs(z) < 1.0) {
    c4 = 1.0 / 24.0 +
         z * (-1.0 / 720.0 +
              z * (1.0 / 40320.0 +
                   z * (-1.0 / 3628800.0 +
                        z * (1.0 / 479001600.0 +
                             z * (-1.0 / 87178291200.0 +
                                  z * (1.0 / 20922789888000.0 +
                                       z * (-1.0 / 6402373705728000.0 +
                                            z * (1.0 / 2432902008176640000.0))))))));
    c5 = 1.0 / 120.0 +
         z * (-1.0 / 5040.0 +
              z * (1.0 / 362880.0 +
                   z * (-1.0 / 39916800.0 +
                        z * (1.0 / 6227020800.0 +
                             z * (-1.0 / 1307674368000.0 +
                                  z * (1.0 / 355687428096000.0 +
                                       z * (-1.0 / 121645100408832000.0 +
                                            z * (1.0 / 51090942171709440000.0))))))));
  } else {
    c4 = (0.5 - c2) / z;
    c5 = (1.0 / 6.0 - c3) / z;
  }
}

// Reverse of the Kepler drift: (x0, v0) -> (x1, v1).  In: pre-drift state,
// the converged s and the output adjoints; out: the input adjoints.
__device__ __forceinline__ void kepler_vjp(double mu, double dt, const double x0[3],
                                           const double v0[3], double s, const double lx1[3],
                                           const double lv1[3], double lx0[3], double lv0[3]) {
  // 1/r0 and 1/r are formed once and multiplied in
  const double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
  const double ir0 = 1.0 / r0;
  const double eta = x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2];
  const double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
  const double beta = 2.0 * mu * ir0 - vv;
  double c0, c1, c2, c3, c4, c5;
  const double zz = beta * s * s;
  stumpff(zz, c0, c1, c2, c3);
  stumpff45(zz, c2, c3, c4, c5);
  const double s2 = s * s;
  const double G0 = c0, G1 = s * c1, G2 = s2 * c2, G3 = s2 * s * c3, G4 = s2 * s2 * c4,
               G5 = s2 * s2 * s * c5;
  const double r = r0 * G0 + eta * G1 + mu * G2;
  const double ir = 1.0 / r;
  const double f = 1.0 - mu * G2 * ir0, g = dt - mu * G3;
  const double fd = -mu * G1 * ir * ir0, gd = 1.0 - mu * G2 * ir;
  // scalar adjoints of f, g, fdot, gdot
  const double wf = x0[0] * lx1[0] + x0[1] * lx1[1] + x0[2] * lx1[2];
  const double wg = v0[0] * lx1[0] + v0[1] * lx1[1] + v0[2] * lx1[2];
  const double wfd = x0[0] * lv1[0] + x0[1] * lv1[1] + x0[2] * lv1[2];
  const double wgd = v0[0] * lv1[0] + v0[1] * lv1[1] + v0[2] * lv1[2];
  double bG0 = 0.0, bG1 = 0.0, bG2 = 0.0, bG3 = 0.0, br = 0.0, br0 = 0.0, beta_ = 0.0, bb = 0.0;
  // gdot = 1 - mu G2/r
  bG2 += -mu * ir * wgd;
  br += mu * G2 * (ir * ir) * wgd;
  // fdot = -mu G1/(r r0)
  bG1 += -mu * (ir * ir0) * wfd;
  br += mu * G1 * (ir * ir * ir0) * wfd;
  br0 += mu * G1 * (ir * ir0 * ir0) * wfd;
  // g = dt - mu G3
  bG3 += -mu * wg;
  // f = 1 - mu G2/r0
  bG2 += -mu * ir0 * wf;
  br0 += mu * G2 * (ir0 * ir0) * wf;
  // r = r0 G0 + eta G1 + mu G2
  bG0 += r0 * br;
  bG1 += eta * br;
  bG2 += mu * br;
  br0 += G0 * br;
  beta_ += G1 * br;
  // G_k(s, beta): dG0/ds = -beta G1, dG_k/ds = G_{k-1}; dG_k/dbeta = (k G_{k+2} - s G_{k+1})/2
  const double bs = bG0 * (-beta * G1) + bG1 * G0 + bG2 * G1 + bG3 * G2;
  const double dG1b = 0.5 * (G3 - s * G2), dG2b = 0.5 * (2.0 * G4 - s * G3),
               dG3b = 0.5 * (3.0 * G5 - s * G4), dG0b = -0.5 * s * G1;
  bb += bG0 * dG0b + bG1 * dG1b + bG2 * dG2b + bG3 * dG3b;
  // s(r0, eta, beta) from r0 G1 + eta G2 + mu G3 = dt; dF/ds = r
  const double Fb = r0 * dG1b + eta * dG2b + mu * dG3b;
  br0 += bs * (-G1 * ir);
  beta_ += bs * (-G2 * ir);
  bb += bs * (-Fb * ir);
  // inputs: r0 = |x0|, eta = x0.v0, beta = 2 mu/r0 - v0.v0
  const double cx = br0 * ir0 - bb * 2.0 * mu * (ir0 * ir0 * ir0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lx0[k] = f * lx1[k] + fd * lv1[k] + cx * x0[k] + beta_ * v0[k];
    lv0[k] = g * lx1[k] + gd * lv1[k] + beta_ * x0[k] - 2.0 * bb * v0[k];
  }
}

}  // namespace genga
