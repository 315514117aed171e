// Reverse-mode gradient of the second-order hybrid step (Eq. 7) with its
// close-encounter machinery (the paper has no adjoint): the changeover K and
// K' of Eqs. (4)-(5) in both kicks, the critical radii of Eq. (6) as
// functions of the state and the masses, the Sun kicks, the Kepler drift,
// and the Bulirsch-Stoer integration of H_A for each close-encounter group
// (Sec. 2.2, 3.2.6).  It differentiates the map the step computes with every
// decision held where it falls: the candidate and encounter sets (Eqs.
// 10-12), the groups (App. A), the accepted BS substeps and the column each
// stops at, and the branches of K and of Eq. (6).  K = 1 outside the
// critical radius, so where a decision changes the map moves by no more
// than the BS tolerance: this is the derivative almost everywhere.
//
// The step follows the recipe of Sec. 2.2 as the main mode does: radii,
// kick tau/2 (H_B with K), Sun kick tau/2, Kepler drift tau, encounter test
// of the candidate pairs, groups, BS of each group over tau from the
// pre-drift state, Sun kick tau/2, kick tau/2, precheck (the next step's
// candidates).  The first step's candidates are the precheck of the initial
// state with its own radii.
//
// One wave per system, one lane per body; partner data by lane reads in
// wave-uniform loops.  BS of a group of up to 8 members runs its columns
// side by side (lane 8 c + q: column c of member slot q), larger groups one
// column after another.  Forward: the state and the candidate set every k
// steps.  Backward, per segment from the last: the segment replayed keeping
// each step's start (the tape), then per step in reverse the step
// recomputed and its pieces reversed:
//   kick   v' = v + h a_B(x; m, rc):  x^ += A^T (h v'^), with the mass and
//          radius adjoints; for a pair term G m_j f(r, rc) d, d = x_j - x_i,
//          f = K/r^3 - K'/r^2, the lane's share is
//          G [f u + (f_r / r)(d.u) d], u = m_i w_j - m_j w_i
//   Sun    x' = x + h P(v)/m0
//   drift  the Kepler VJP (implicit function for the universal anomaly)
//   BS     the group's BS rerun keeping the start of each accepted substep;
//          an accepted substep's value is a fixed linear combination
//          sum_q W_q G_q of the Gragg results of its columns (the
//          Aitken-Neville tableau is linear in them), so its adjoint is
//          sum_q G_q^T (W_q y^); each Gragg sequence is recomputed keeping
//          its positions and reversed substep by substep, with H_A's pair
//          terms weighted by 1 - K (g = 1/r^3 - f) and the star's term
//   radii  rc = max(n1 R_H, n2 |tau| |v|): x^, v^, m^ of the branch taken.
#include "adj_device.h"
#include "device_math.h"
#include "genga_impl.h"

namespace genga {
namespace {

constexpr int kHK = 8;              // BS columns, n_k = 2k substeps
constexpr int kHLeaf = 64;          // accepted BS substeps of one group in one step
constexpr int kHPos = 2 * kHK + 1;  // positions of the longest Gragg sequence

// Aitken-Neville weights: an attempt that stops at column kk (0-based)
// returns sum_q W[kk][q] G_q, G_q the Gragg result with 2 (q + 1) substeps
// (the tableau recursion applied to unit vectors).
struct NevilleW {
  double w[kHK][kHK];
};
constexpr NevilleW neville_weights() {
  NevilleW out{};
  double T[kHK][kHK][kHK] = {};  // T[k][j][q]
  for (int k = 0; k < kHK; ++k) {
    for (int q = 0; q < kHK; ++q) T[k][0][q] = q == k ? 1.0 : 0.0;
    for (int j = 1; j <= k; ++j) {
      const double ratio = (double)(2 * (k + 1)) / (double)(2 * (k - j + 1));
      const double den = ratio * ratio - 1.0;
      for (int q = 0; q < kHK; ++q)
        T[k][j][q] = T[k][j - 1][q] + (T[k][j - 1][q] - T[k - 1][j - 1][q]) / den;
    }
    for (int q = 0; q < kHK; ++q) out.w[k][q] = T[k][k][q];
  }
  return out;
}
__constant__ NevilleW kNW = neville_weights();

struct HArgs {
  double4* __restrict__ xm;  // batched state (x, m), advanced by the forward pass
  double4* __restrict__ vv;
  const int* __restrict__ off;
  const double* __restrict__ m0;
  double* __restrict__ ckpt;  // [C][7][nb]: x, y, z, vx, vy, vz, candidate bits
  double* __restrict__ tape;  // [K][7][nl]
  double* __restrict__ leaf;  // [kHLeaf][6][nl]: starts of accepted BS substeps
  double* __restrict__ zpos;  // [kHPos][3][nl]: positions of one Gragg sequence
  const double* __restrict__ gxT;
  const double* __restrict__ gvT;
  double* __restrict__ gx0;
  double* __restrict__ gv0;
  double* __restrict__ gm;
  unsigned* __restrict__ flags;
  int nsys, T, K, C, nl, max_iter, bs_depth;
  int64_t nb;
  double G, dt, h, n1, n2, pf, absdt, bs_tol;
};

// the lane's body
struct Sys {
  int lane, n, row;
  bool act;
  size_t gl;                  // lane index in the per-lane scratch
  double m, m0, Gm0;
  unsigned long long all;     // the system's bodies as a lane mask
};

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int j) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, j);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), j);
  return ((unsigned long long)hi << 32) | lo;
}

// Changeover of Eqs. (4)-(5) for a pair at r with pair radius rc:
// y = (r - 0.1 rc)/(0.9 rc), K = y^2/D, D = 2y^2 - 2y + 1, and dK/dr.  The
// forward map rounds like the plain definitions (divisions and square roots
// correctly rounded, no fused multiply-adds: this file is built with
// -ffp-contract=off), so that its close encounters follow the reference
// trajectory as closely as rounding allows.
__device__ __forceinline__ void chg(double r, double rc, double& K, double& Kr) {
  if (!(rc > 0.0)) {
    K = 1.0;
    Kr = 0.0;
    return;
  }
  const double y = (r - 0.1 * rc) / (0.9 * rc);
  if (y <= 0.0) {
    K = 0.0;
    Kr = 0.0;
  } else if (y >= 1.0) {
    K = 1.0;
    Kr = 0.0;
  } else {
    const double D = 2.0 * y * y - 2.0 * y + 1.0;
    K = y * y / D;
    Kr = 2.0 * y * (1.0 - y) / (D * D) / (0.9 * rc);
  }
}

// The same with the second derivatives for the reverse pass (reciprocals
// refined from the hardware estimates): K, dK/dr, d2K/dr2, dK/drc,
// d2K/(dr drc); kappa' = 2y(1-y)/D^2, kappa'' = (2 - 4y)(1 + 2y - 2y^2)/D^3,
// dy/drc = -r/(0.9 rc^2) = -0.9 r s^2 with s = 1/(0.9 rc).
__device__ __forceinline__ void chg2(double r, double rc, double& K, double& Kr, double& Krr,
                                     double& Kc, double& Krc) {
  Krr = Kc = Krc = 0.0;
  if (!(rc > 0.0)) {
    K = 1.0;
    Kr = 0.0;
    return;
  }
  const double s = rcp_nr(0.9 * rc);
  const double y = (r - 0.1 * rc) * s;
  if (y <= 0.0) {
    K = 0.0;
    Kr = 0.0;
  } else if (y >= 1.0) {
    K = 1.0;
    Kr = 0.0;
  } else {
    const double iD = rcp_nr(2.0 * y * y - 2.0 * y + 1.0);  // D in [1/2, 1]
    K = y * y * iD;
    const double k1 = 2.0 * y * (1.0 - y) * iD * iD;
    const double k2 = (2.0 - 4.0 * y) * (1.0 + 2.0 * y - 2.0 * y * y) * iD * iD * iD;
    const double yc = -0.9 * r * s * s;
    Kr = k1 * s;
    Krr = k2 * s * s;
    Kc = k1 * yc;
    Krc = k2 * yc * s - 0.9 * k1 * s * s;
  }
}

// ---- forward pieces ----------------------------------------------------------
// H_B acceleration (the gradient of Eq. 2): sum over the system's other bodies.
__device__ __forceinline__ void accel_B(const HArgs& a, const Sys& S, const double x[3], double rc, double acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.0;
  for (int j = 0; j < S.n; ++j) {
    const double xj = readlane_d(x[0], j), yj = readlane_d(x[1], j), zj = readlane_d(x[2], j);
    const double mj = readlane_d(S.m, j), rcj = readlane_d(rc, j);
    if (S.act && j != S.lane) {
      const double d0 = xj - x[0], d1 = yj - x[1], d2 = zj - x[2];
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double r = sqrt(r2);
      const double rcij = rc > rcj ? rc : rcj;
      double K, dK;
      chg(r, rcij, K, dK);
      const double f = K / (r2 * r) - dK / r2;
      const double s = a.G * mj * f;
      acc[0] += s * d0;
      acc[1] += s * d1;
      acc[2] += s * d2;
    }
  }
}

// P = sum_j m_j v_j in body order
__device__ __forceinline__ void momentum(const Sys& S, const double v[3], double P[3]) {
  P[0] = P[1] = P[2] = 0.0;
  for (int j = 0; j < S.n; ++j) {
    const double mj = readlane_d(S.m, j);
    P[0] += mj * readlane_d(v[0], j);
    P[1] += mj * readlane_d(v[1], j);
    P[2] += mj * readlane_d(v[2], j);
  }
}

__device__ __forceinline__ void lane_sum3(const Sys& S, const double w[3], double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int j = 0; j < S.n; ++j) {
    out[0] += readlane_d(w[0], j);
    out[1] += readlane_d(w[1], j);
    out[2] += readlane_d(w[2], j);
  }
}

// H_A derivative of a group member (star fixed at the origin, pair terms of
// the members weighted by 1 - K): y = (x, v) -> (v, a).
__device__ __forceinline__ void ha_deriv(const HArgs& a, const Sys& S, unsigned long long M, bool mem, double rc,
                         const double y[6], double dy[6]) {
  const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  const double r = sqrt(r2);
  const double fs = -S.Gm0 / (r2 * r);
  double a0 = fs * y[0], a1 = fs * y[1], a2 = fs * y[2];
  for (unsigned long long q = M; q; q &= q - 1) {
    const int j = __builtin_ctzll(q);
    const double xj = readlane_d(y[0], j), yj = readlane_d(y[1], j), zj = readlane_d(y[2], j);
    const double mj = readlane_d(S.m, j), rcj = readlane_d(rc, j);
    if (mem && j != S.lane) {
      const double d0 = xj - y[0], d1 = yj - y[1], d2 = zj - y[2];
      const double q2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double qq = sqrt(q2);
      const double rcij = rc > rcj ? rc : rcj;
      double K, dK;
      chg(qq, rcij, K, dK);
      const double f = (1.0 - K) / (q2 * qq) + dK / q2;
      const double sj = a.G * mj * f;
      a0 += sj * d0;
      a1 += sj * d1;
      a2 += sj * d2;
    }
  }
  dy[0] = y[3];
  dy[1] = y[4];
  dy[2] = y[5];
  dy[3] = a0;
  dy[4] = a1;
  dy[5] = a2;
}

// Gragg's modified midpoint rule over H with nsub substeps; with keep, the
// positions z_0 .. z_nsub go to the lane's zpos slots.  One derivative per
// pass of the loop: at z_0, at z_1 .. z_{nsub-1} (the midpoint steps), and at
// z_nsub (the smoothing step).
__device__ __forceinline__ void gragg(const HArgs& a, const Sys& S, unsigned long long M, bool mem,
                                      double rc, const double y0[6], double H, int nsub,
                                      double out[6], bool keep) {
  const double hs = H / nsub;
  double d[6], ym[6], yn[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) yn[c] = y0[c];
  if (keep) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.zpos[(size_t)c * a.nl + S.gl] = y0[c];
  }
  for (int m = 0; m <= nsub; ++m) {
    ha_deriv(a, S, M, mem, rc, yn, d);
    if (m == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        ym[c] = y0[c];
        yn[c] = y0[c] + hs * d[c];
      }
    } else if (m < nsub) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double t = ym[c] + 2.0 * hs * d[c];
        ym[c] = yn[c];
        yn[c] = t;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c) out[c] = 0.5 * (ym[c] + yn[c] + hs * d[c]);
    }
    if (keep && m < nsub) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.zpos[((size_t)(m + 1) * 3 + c) * a.nl + S.gl] = yn[c];
    }
  }
}

__device__ __forceinline__ double vrel3(const double* A, const double* B) {
  const double d0 = A[0] - B[0], d1 = A[1] - B[1], d2 = A[2] - B[2];
  const double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double den = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
  return den > 0.0 ? num / den : num;
}

// One BS attempt over H from y0: the accepted column (>= 1) with its value
// in yout (members), or -1 when no column meets the tolerance.  The lane's
// tableau row lives in LDS (its own column of tab), so that the columns can
// be a loop.
__device__ __forceinline__ int bs_attempt(const HArgs& a, const Sys& S, unsigned long long M,
                                          bool mem, double rc, const double y0[6], double H,
                                          double yout[6]) {
  __shared__ double tab[kHK][6][64];  // T(k - 1, j) on entry to column k, T(k, j) after
  const int L = S.lane;
  for (int k = 0; k < kHK; ++k) {
    double cur[6], up[6];
    gragg(a, S, M, mem, rc, y0, H, 2 * (k + 1), cur, false);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      up[c] = tab[0][c][L];
      tab[0][c][L] = cur[c];
    }
    for (int j = 1; j <= k; ++j) {
      const double ratio = (double)(2 * (k + 1)) / (double)(2 * (k - j + 1));
      const double den = ratio * ratio - 1.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double nw = cur[c] + (cur[c] - up[c]) / den;
        if (j < k) up[c] = tab[j][c][L];
        tab[j][c][L] = nw;
        cur[c] = nw;
      }
    }
    if (k >= 1) {
      double prev[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) prev[c] = tab[k - 1][c][L];
      double err = 0.0;
      if (mem) err = fmax(vrel3(&cur[0], &prev[0]), vrel3(&cur[3], &prev[3]));
      err = wave_max(err);
      if (err <= a.bs_tol) {
#pragma unroll
        for (int c = 0; c < 6; ++c) yout[c] = cur[c];
        return k;
      }
    }
  }
  return -1;
}

// ---- column-parallel BS for groups of up to 8 members ----------------------
// Lane L = 8 c + l holds column c (2 (c + 1) substeps); inside the column's
// eight lanes, l = w s + q: member slot q (the q-th member in body order) of
// depth slot s, w the smallest of 2, 4, 8 not below the group size.  Depth
// slot s attempts the substep of length H / 2^s from the same start (the
// attempts the sequential refinement makes after s failures), so a group of
// two tries four halvings at once and one of three or four two; the first
// slot in sequential order with an accepted column is taken.  The columns
// of an attempt run side by side: it takes as many derivative rounds as its
// longest column (17) instead of the sum over its columns (up to 80).  The
// Aitken-Neville tableau moves down the columns by lane reads from the
// column below (lane - 8).  Every sum is formed in the order of the
// one-column-at-a-time form above, so both give the same bits.  The reverse
// pass uses one depth slot (lanes w .. 7 of a column idle).
constexpr int kHPar = 8;

struct Par {
  int c, q, sz, src;             // column, member slot, group size, body lane of the slot
  int s, w, ns;                  // depth slot, slot width, depth slots per attempt
  bool on;                       // the slot holds a member
  double m, rc;                  // its mass and radius
  double pm[kHPar], prc[kHPar];  // every slot's mass and radius
};

__device__ __forceinline__ int nth_bit64(unsigned long long M, int b) {
  for (int t = 0; t < b; ++t) M &= M - 1;
  return __builtin_ctzll(M);
}

__device__ __forceinline__ Par par_of(const Sys& S, unsigned long long M, double rc,
                                      bool depths = false) {
  Par P;
  P.c = S.lane >> 3;
  P.sz = __builtin_popcountll(M);
  P.w = P.sz > 4 ? kHPar : P.sz > 2 ? 4 : 2;
  P.ns = depths ? kHPar / P.w : 1;
  P.s = depths ? (S.lane & 7) / P.w : 0;
  P.q = (S.lane & 7) - P.s * P.w;
  P.on = P.q < P.sz;
  P.src = P.on ? nth_bit64(M, P.q) : 0;
  P.m = __shfl(S.m, P.src, 64);
  P.rc = __shfl(rc, P.src, 64);
#pragma unroll
  for (int t = 0; t < kHPar; ++t) {
    const int bl = t < P.sz ? nth_bit64(M, t) : 0;
    P.pm[t] = readlane_d(S.m, bl);
    P.prc[t] = readlane_d(rc, bl);
  }
  return P;
}

// ha_deriv for the lane's slot, partners from the lanes of its column.
__device__ __forceinline__ void ha_deriv_par(const HArgs& a, const Sys& S, const Par& P,
                                             const double y[6], double dy[6]) {
  const double r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  const double r = sqrt(r2);
  const double fs = -S.Gm0 / (r2 * r);
  double a0 = fs * y[0], a1 = fs * y[1], a2 = fs * y[2];
  const int base = (S.lane & ~7) + P.s * P.w;
#pragma unroll
  for (int t = 0; t < kHPar; ++t) {
    if (t >= P.w) break;  // the slot's lanes only (wave-uniform)
    const double xj = __shfl(y[0], base + t, 64), yj = __shfl(y[1], base + t, 64),
                 zj = __shfl(y[2], base + t, 64);
    if (t < P.sz && P.on && t != P.q) {
      const double d0 = xj - y[0], d1 = yj - y[1], d2 = zj - y[2];
      const double q2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double qq = sqrt(q2);
      const double rcij = P.rc > P.prc[t] ? P.rc : P.prc[t];
      double K, dK;
      chg(qq, rcij, K, dK);
      const double f = (1.0 - K) / (q2 * qq) + dK / q2;
      const double sj = a.G * P.pm[t] * f;
      a0 += sj * d0;
      a1 += sj * d1;
      a2 += sj * d2;
    }
  }
  dy[0] = y[3];
  dy[1] = y[4];
  dy[2] = y[5];
  dy[3] = a0;
  dy[4] = a1;
  dy[5] = a2;
}

// Rounds mfrom .. mto of the lane's column of Gragg's rule (nsub = 2 (c + 1)
// substeps of hs from y0; ym, yn: the last two points; out: the result once
// round nsub is done), a column idle once its sequence is done.  keep:
// positions to zpos.
__device__ __forceinline__ void gragg_rounds(const HArgs& a, const Sys& S, const Par& P,
                                             const double y0[6], double hs, int nsub,
                                             double ym[6], double yn[6], double out[6],
                                             bool keep, int mfrom, int mto) {
  double d[6];
  for (int m = mfrom; m <= mto; ++m) {
    ha_deriv_par(a, S, P, yn, d);
    if (m == 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) yn[c] = y0[c] + hs * d[c];
    } else if (m < nsub) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double t = ym[c] + 2.0 * hs * d[c];
        ym[c] = yn[c];
        yn[c] = t;
      }
    } else if (m == nsub) {
#pragma unroll
      for (int c = 0; c < 6; ++c) out[c] = 0.5 * (ym[c] + yn[c] + hs * d[c]);
    }
    if (keep && m < nsub) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.zpos[((size_t)(m + 1) * 3 + c) * a.nl + S.gl] = yn[c];
    }
  }
}

// The lane's column of Gragg's rule (2 (c + 1) substeps over H); rounds 0 ..
// mtop (17 for every column; fewer when only the columns with 2 (c + 1) <=
// mtop are wanted).  keep: positions to zpos.
__device__ __forceinline__ void gragg_par(const HArgs& a, const Sys& S, const Par& P,
                                          const double y0[6], double H, double out[6],
                                          bool keep, int mtop = 2 * kHPar) {
  const int nsub = 2 * (P.c + 1);
  const double hs = ldexp(H, -P.s) / nsub;  // the lane's depth slot (exact scaling)
  double ym[6], yn[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    yn[c] = y0[c];
    ym[c] = y0[c];
    out[c] = 0.0;
  }
  if (keep) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.zpos[(size_t)c * a.nl + S.gl] = y0[c];
  }
  gragg_rounds(a, S, P, y0, hs, nsub, ym, yn, out, keep, 0, mtop);
}

// The Aitken-Neville tableau of the columns 0 .. kmax from their Gragg
// results T0 (T(c, 0) in the lanes of column c): T(c, j) = T(c, j-1) +
// (T(c, j-1) - T(c-1, j-1)) / ((n_c / n_{c-j})^2 - 1), the column below read
// from lane - 8; Td, Ts receive T(c, c) and T(c, c-1) in the lanes of every
// column c <= kmax.  The same operations in the same order for any kmax.
__device__ __forceinline__ void neville_par(const Sys& S, const Par& P, const double T0[6],
                                            int kmax, double Td[6], double Ts[6]) {
  double T[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    T[c] = T0[c];
    Td[c] = T0[c];
    Ts[c] = 0.0;
  }
  for (int j = 1; j <= kmax; ++j) {
    double up[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) up[c] = __shfl(T[c], S.lane - 8, 64);  // T(c - 1, j - 1)
    if (P.c >= j) {
      const double ratio = (double)(2 * (P.c + 1)) / (double)(2 * (P.c - j + 1));
      const double den = ratio * ratio - 1.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double nw = T[c] + (T[c] - up[c]) / den;
        if (P.c == j) {
          Ts[c] = T[c];
          Td[c] = nw;
        }
        T[c] = nw;
      }
    }
  }
}

// Ballot of the leading lanes (member slot 0) of the columns 1 .. kmax of
// the depth slots below smax whose largest relative change over the slot's
// members is within tol (lane bit 8 c + w s).
__device__ __forceinline__ unsigned long long accepted_par(const HArgs& a, const Par& P,
                                                           const double Td[6],
                                                           const double Ts[6], int kmax,
                                                           int smax) {
  double err = 0.0;
  if (P.on && P.c >= 1) err = fmax(vrel3(&Td[0], &Ts[0]), vrel3(&Td[3], &Ts[3]));
  // the largest error over the slot's members (its w adjacent lanes)
  err = fmax(err, __shfl_xor(err, 1, 64));
  if (P.w >= 4) err = fmax(err, __shfl_xor(err, 2, 64));
  if (P.w >= 8) err = fmax(err, __shfl_xor(err, 4, 64));
  return __builtin_amdgcn_ballot_w64(P.q == 0 && P.c >= 1 && P.c <= kmax && P.s < smax &&
                                     err <= a.bs_tol);
}

// bs_attempt with the columns side by side and P.ns depth slots (slots from
// smax on are past the depth limit and not taken): y holds the members'
// state in their body lanes; the accepted column (>= 1) of the first slot
// that has one, its slot in *sa and its value in yout (body lanes of
// members), or -1.  The columns up to kHMid are tested when they are done
// (after round 2 (kHMid + 1)): when the first slot has an accepted column
// among them the attempt ends there; otherwise the rest of the rounds run
// and every column is tested.  Either way the result is that of testing
// every column at the end.
constexpr int kHMid = 4;
__device__ __forceinline__ int bs_attempt_par(const HArgs& a, const Sys& S,
                                              unsigned long long M, const Par& P,
                                              const double y[6], double H, double yout[6],
                                              int smax, int* sa) {
  double y0[6], ym[6], yn[6], T0[6], Td[6], Ts[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    y0[c] = __shfl(y[c], P.src, 64);
    ym[c] = y0[c];
    yn[c] = y0[c];
    T0[c] = 0.0;
  }
  const int nsub = 2 * (P.c + 1);
  const double hs = ldexp(H, -P.s) / nsub;  // the lane's depth slot (exact scaling)
  gragg_rounds(a, S, P, y0, hs, nsub, ym, yn, T0, false, 0, 2 * (kHMid + 1));  // T(c, 0), c <= kHMid
  neville_par(S, P, T0, kHMid, Td, Ts);
  unsigned long long ok = accepted_par(a, P, Td, Ts, kHMid, smax);
  const unsigned long long slot0 = 0x0101010101010101ull;  // slot 0 leads at lanes 8 c
  int s = 0;
  unsigned long long oks = ok & slot0;
  if (oks == 0ull) {
    gragg_rounds(a, S, P, y0, hs, nsub, ym, yn, T0, false, 2 * (kHMid + 1) + 1, 2 * kHPar);
    neville_par(S, P, T0, kHPar - 1, Td, Ts);
    ok = accepted_par(a, P, Td, Ts, kHPar - 1, smax);
    if (ok == 0ull) return -1;
    // the first slot with an accepted column: slot s leads at lanes 8 c + w s
    for (; s < P.ns; ++s) {
      oks = ok & (slot0 << (P.w * s));
      if (oks) break;
    }
  }
  const int k = __builtin_ctzll(oks) >> 3;
  *sa = s;
  const int qi = __builtin_popcountll(M & ((1ull << S.lane) - 1ull));  // the body lane's slot
#pragma unroll
  for (int c = 0; c < 6; ++c) yout[c] = __shfl(Td[c], 8 * k + ((P.w * s + qi) & 7), 64);
  return k;
}

// BS of one group over tau with binary refinement (as the main mode): y is
// the members' state in and out.  With REC the start of every accepted
// substep goes to the lane's leaf slots and its length and column to lh, lk
// (LDS).  Returns 0, or -1 when the depth is exhausted; *nleaf counts the
// accepted substeps.
template <bool REC>
__device__ __forceinline__ int bs_group(const HArgs& a, const Sys& S, unsigned long long M, bool mem, double rc,
                        double y[6], double* lh, int* lk, int* nleaf) {
  const Par P = par_of(S, M, rc, true);
  const int D = a.bs_depth;
  const int64_t total = (int64_t)1 << D;
  int64_t pos = 0;
  int d = 0, nl = 0;
  while (pos < total) {
    double yn[6];
    int k, sa = 0;
    const int smax = P.sz <= kHPar ? min(P.ns, D - d + 1) : 1;  // depths tried at once
    if (P.sz <= kHPar)
      k = bs_attempt_par(a, S, M, P, y, ldexp(a.dt, -d), yn, smax, &sa);
    else
      k = bs_attempt(a, S, M, mem, rc, y, ldexp(a.dt, -d), yn);
    if (k >= 1) {
      d += sa;
      const double hh = ldexp(a.dt, -d);  // the accepted substep's length
      if (REC) {
        if (nl < kHLeaf) {
#pragma unroll
          for (int c = 0; c < 6; ++c) a.leaf[((size_t)nl * 6 + c) * a.nl + S.gl] = y[c];
          if (S.lane == 0) {
            lh[nl] = hh;
            lk[nl] = k;
          }
        }
        ++nl;
      }
      if (mem) {
#pragma unroll
        for (int c = 0; c < 6; ++c) y[c] = yn[c];
      }
      pos += (int64_t)1 << (D - d);
      while (d > 0 && (pos % ((int64_t)1 << (D - d + 1))) == 0) --d;
    } else {
      d += smax;
      if (d > D) {
        if (nleaf) *nleaf = nl;
        return -1;
      }
    }
  }
  if (nleaf) *nleaf = nl;
  return 0;
}

// Intermediate values of one step kept for its reverse.
struct StepVals {
  double x0[3], v0[3];  // start
  double rc;            // radii of the step (Eq. 6 at the start)
  double x1[3], v1[3];  // after the opening kick and Sun kick: the drift's start
  double s;             // universal anomaly of the Kepler drift
  double x2[3], v2[3];  // after the drift (BS for group members)
  double x3[3];         // after the second Sun kick: the closing kick's positions
  int label;            // group label (the smallest member), or -1
};

// Encounters among the candidate pairs j > i (Hermite test of the drift,
// Eqs. 10-12, below rc_ij^2), then the groups: every lane takes the smallest
// label of its neighbours until nothing changes (the components of the
// encounter graph, labelled by their smallest member).
__device__ __forceinline__ int groups(const HArgs& a, const Sys& S, unsigned long long cand, const double xa[3],
                      const double va[3], const double xb[3], const double vb[3], double rc) {
  unsigned long long E = 0ull;
  for (int j = 0; j < S.n; ++j) {
    const double x0j = readlane_d(xa[0], j), y0j = readlane_d(xa[1], j), z0j = readlane_d(xa[2], j);
    const double u0j = readlane_d(va[0], j), w0j = readlane_d(va[1], j), q0j = readlane_d(va[2], j);
    const double x1j = readlane_d(xb[0], j), y1j = readlane_d(xb[1], j), z1j = readlane_d(xb[2], j);
    const double u1j = readlane_d(vb[0], j), w1j = readlane_d(vb[1], j), q1j = readlane_d(vb[2], j);
    const double rcj = readlane_d(rc, j);
    if (S.act && j > S.lane && ((cand >> j) & 1ull)) {
      const double d2 = hermite_dmin2(a.dt, x0j - xa[0], y0j - xa[1], z0j - xa[2], u0j - va[0],
                                      w0j - va[1], q0j - va[2], x1j - xb[0], y1j - xb[1],
                                      z1j - xb[2], u1j - vb[0], w1j - vb[1], q1j - vb[2]);
      const double rcij = rc > rcj ? rc : rcj;
      if (d2 < rcij * rcij) E |= 1ull << j;
    }
  }
  // neighbours: the lane's pairs and those of lower lanes that name it
  unsigned long long nbr = E;
  for (int j = 0; j < S.n; ++j) {
    const unsigned long long Ej = readlane_u64(E, j);
    if ((Ej >> S.lane) & 1ull) nbr |= 1ull << j;
  }
  int label = nbr ? S.lane : 64;
  for (int it = 0; it < 64; ++it) {
    int nw = label;
    for (int j = 0; j < S.n; ++j) {
      const int lj = __builtin_amdgcn_readlane(label, j);
      if ((nbr >> j) & 1ull) nw = min(nw, lj);
    }
    const bool ch = nw != label;
    label = nw;
    if (__builtin_amdgcn_ballot_w64(ch) == 0ull) break;
  }
  return nbr ? label : -1;
}

// The precheck (Sec. 2.2): partners j > i closer than pf rc_ij.
__device__ __forceinline__ unsigned long long precheck(const HArgs& a, const Sys& S, const double x[3], double rc) {
  unsigned long long c = 0ull;
  for (int j = 0; j < S.n; ++j) {
    const double xj = readlane_d(x[0], j), yj = readlane_d(x[1], j), zj = readlane_d(x[2], j);
    const double rcj = readlane_d(rc, j);
    if (S.act && j > S.lane) {
      const double d0 = xj - x[0], d1 = yj - x[1], d2 = zj - x[2];
      const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double rcij = rc > rcj ? rc : rcj;
      if (r < a.pf * rcij) c |= 1ull << j;
    }
  }
  return c;
}

__device__ __forceinline__ double radius(const HArgs& a, const Sys& S, const double x[3],
                                         const double v[3]) {
  return S.act ? rcrit(x[0], x[1], x[2], v[0], v[1], v[2], S.m, S.Gm0, S.m0, a.n1, a.n2, a.absdt)
               : 0.0;
}

// One hybrid step of the lane's system: x, v and the candidate bits in and
// out; R keeps the intermediate values.
__device__ __forceinline__ void hyb_step(const HArgs& a, const Sys& S, double x[3], double v[3],
                         unsigned long long& cand, StepVals& R, unsigned& fl) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R.x0[c] = x[c];
    R.v0[c] = v[c];
  }
  const double rc = radius(a, S, x, v);
  R.rc = rc;
  double acc[3], P[3];
  accel_B(a, S, x, rc, acc);
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] += a.h * acc[c];
  momentum(S, v, P);
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] += a.h * P[c] / S.m0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R.x1[c] = x[c];
    R.v1[c] = v[c];
  }
  double s = 0.0;
  if (S.act && kepler_drift(S.Gm0, a.dt, x[0], x[1], x[2], v[0], v[1], v[2], a.max_iter, &s) < 0)
    fl |= F_KEPLER;
  R.s = s;
  const int label = groups(a, S, cand, R.x1, R.v1, x, v, rc);
  R.label = label;
  // BS of each group from the pre-drift state, groups by ascending label
  unsigned long long roots = __builtin_amdgcn_ballot_w64(label == S.lane);
  for (; roots; roots &= roots - 1) {
    const int g = __builtin_ctzll(roots);
    const bool mem = label == g;
    const unsigned long long M = __builtin_amdgcn_ballot_w64(mem);
    double y[6] = {R.x1[0], R.x1[1], R.x1[2], R.v1[0], R.v1[1], R.v1[2]};
    if (bs_group<false>(a, S, M, mem, rc, y, nullptr, nullptr, nullptr) < 0) fl |= F_BS;
    if (mem) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[c] = y[c];
        v[c] = y[3 + c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R.x2[c] = x[c];
    R.v2[c] = v[c];
  }
  momentum(S, v, P);
#pragma unroll
  for (int c = 0; c < 3; ++c) x[c] += a.h * P[c] / S.m0;
#pragma unroll
  for (int c = 0; c < 3; ++c) R.x3[c] = x[c];
  accel_B(a, S, x, rc, acc);
#pragma unroll
  for (int c = 0; c < 3; ++c) v[c] += a.h * acc[c];
  cand = precheck(a, S, x, rc);
}

// ---- reverse pieces --------------------------------------------------------
// Pair terms over the partners in P (bits of lanes) at positions x for the
// acceleration adjoint w: out += A^T w, with the mass and radius adjoints of
// the lane's body.  HA: H_A's 1 - K weighting (g = 1/r^3 - f).  The radius
// of a pair is the larger of the two (the first when neither is larger, as
// the term of the first body sees it), so each term's radius adjoint goes
// to the body whose radius it used.
template <bool HA>
__device__ __forceinline__ void pair_vjp(const HArgs& a, const Sys& S, unsigned long long Pm, bool on, double rc,
                         const double x[3], const double w[3], double out[3], double& mb,
                         double& rcb) {
  for (unsigned long long q = Pm; q; q &= q - 1) {
    const int j = __builtin_ctzll(q);
    const double xj = readlane_d(x[0], j), yj = readlane_d(x[1], j), zj = readlane_d(x[2], j);
    const double wx = readlane_d(w[0], j), wy = readlane_d(w[1], j), wz = readlane_d(w[2], j);
    const double mj = readlane_d(S.m, j), rcj = readlane_d(rc, j);
    if (on && j != S.lane) {
      const double d0 = xj - x[0], d1 = yj - x[1], d2 = zj - x[2];
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double ir = rsqrt_nr(r2), ir2 = ir * ir, ir3 = ir2 * ir, ir4 = ir2 * ir2;
      const double r = r2 * ir;
      const double rcij = rc > rcj ? rc : rcj;
      double K, Kr, Krr, Kc, Krc;
      chg2(r, rcij, K, Kr, Krr, Kc, Krc);
      double f = K * ir3 - Kr * ir2;
      double fr = 3.0 * Kr * ir3 - 3.0 * K * ir4 - Krr * ir2;
      double fc = Kc * ir3 - Krc * ir2;
      if (HA) {
        f = ir3 - f;
        fr = -3.0 * ir4 - fr;
        fc = -fc;
      }
      const double u0 = S.m * wx - mj * w[0], u1 = S.m * wy - mj * w[1], u2 = S.m * wz - mj * w[2];
      const double du = d0 * u0 + d1 * u1 + d2 * u2;
      const double c = fr * ir * du;
      out[0] += a.G * (f * u0 + c * d0);
      out[1] += a.G * (f * u1 + c * d1);
      out[2] += a.G * (f * u2 + c * d2);
      mb -= a.G * f * (d0 * wx + d1 * wy + d2 * wz);
      // the lane's term (rc_ij = rc when rc > rcj) and the partner's term
      // (rc_ij = rc when rc >= rcj)
      const double tl = a.G * fc * mj * (d0 * w[0] + d1 * w[1] + d2 * w[2]);
      const double tp = -a.G * fc * S.m * (d0 * wx + d1 * wy + d2 * wz);
      if (rc > rcj) rcb += tl;
      if (rc >= rcj) rcb += tp;
    }
  }
}

// H_A acceleration adjoint of a group member: the star's term and the pairs.
__device__ __forceinline__ void ha_vjp(const HArgs& a, const Sys& S, unsigned long long M, bool mem, double rc,
                       const double z[3], const double w[3], double out[3], double& mb,
                       double& rcb) {
  out[0] = out[1] = out[2] = 0.0;
  const double r2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
  const double ir = rsqrt_nr(r2), ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
  const double xw = z[0] * w[0] + z[1] * w[1] + z[2] * w[2];
  if (mem) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = -S.Gm0 * (w[c] * ir3 - 3.0 * xw * z[c] * ir5);
  }
  pair_vjp<true>(a, S, M, mem, rc, z, w, out, mb, rcb);
}

// yb += G^T ob for the Gragg sequence of nsub substeps over H from y0: the
// sequence recomputed keeping its positions, then reversed from the
// smoothing step (out = (z_{n-1} + z_n + hs F(z_n)) / 2) through the
// midpoint steps (z_{m+1} = z_{m-1} + 2 hs F(z_m)) to the first Euler step
// (z_1 = z_0 + hs F(z_0)); P and Q hold the adjoints of z_{m+1} and z_m.
__device__ __forceinline__ void gragg_vjp(const HArgs& a, const Sys& S, unsigned long long M,
                                          bool mem, double rc, const double y0[6], double H,
                                          int nsub, const double ob[6], double yb[6], double& mb,
                                          double& rcb) {
  const double hs = H / nsub;
  double tmp[6];
  gragg(a, S, M, mem, rc, y0, H, nsub, tmp, true);
  double Pa[6], Qa[6];
  for (int m = nsub; m >= 0; --m) {
    double z[3], w[3], o[3];
    const double cw = m == nsub ? 0.5 * hs : (m == 0 ? hs : 2.0 * hs);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c] = a.zpos[((size_t)m * 3 + c) * a.nl + S.gl];
      w[c] = cw * (m == nsub ? ob[3 + c] : Pa[3 + c]);
    }
    ha_vjp(a, S, M, mem, rc, z, w, o, mb, rcb);
    if (m == nsub) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Pa[c] = 0.5 * ob[c] + o[c];
        Pa[3 + c] = 0.5 * ob[3 + c] + 0.5 * hs * ob[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) Qa[c] = 0.5 * ob[c];
    } else if (m > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Qa[c] += o[c];
        Qa[3 + c] += 2.0 * hs * Pa[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double t = Pa[c];
        Pa[c] = Qa[c];
        Qa[c] = t;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Qa[c] += Pa[c] + o[c];
        Qa[3 + c] += Pa[3 + c] + hs * Pa[c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) yb[c] += Qa[c];
}

// ha_vjp for the lane's slot of the column-parallel layout (partners from
// the lanes of its column, in slot order).
__device__ __forceinline__ void ha_vjp_par(const HArgs& a, const Sys& S, const Par& P,
                                           const double z[3], const double w[3], double out[3],
                                           double& mb, double& rcb) {
  out[0] = out[1] = out[2] = 0.0;
  const double r2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
  const double ir = rsqrt_nr(r2), ir3 = ir * ir * ir, ir5 = ir3 * ir * ir;
  const double xw = z[0] * w[0] + z[1] * w[1] + z[2] * w[2];
  if (P.on) {
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c] = -S.Gm0 * (w[c] * ir3 - 3.0 * xw * z[c] * ir5);
  }
  const int base = S.lane & ~7;
#pragma unroll
  for (int t = 0; t < kHPar; ++t) {
    if (t >= P.w) break;  // the group's lanes only (wave-uniform)
    const double xj = __shfl(z[0], base + t, 64), yj = __shfl(z[1], base + t, 64),
                 zj = __shfl(z[2], base + t, 64);
    const double wx = __shfl(w[0], base + t, 64), wy = __shfl(w[1], base + t, 64),
                 wz = __shfl(w[2], base + t, 64);
    if (t < P.sz && P.on && t != P.q) {
      const double mj = P.pm[t], rcj = P.prc[t];
      const double d0 = xj - z[0], d1 = yj - z[1], d2 = zj - z[2];
      const double q2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double iq = rsqrt_nr(q2), iq2 = iq * iq, iq3 = iq2 * iq, iq4 = iq2 * iq2;
      const double q = q2 * iq;
      const double rcij = P.rc > rcj ? P.rc : rcj;
      double K, Kr, Krr, Kc, Krc;
      chg2(q, rcij, K, Kr, Krr, Kc, Krc);
      const double f = iq3 - (K * iq3 - Kr * iq2);
      const double fr = -3.0 * iq4 - (3.0 * Kr * iq3 - 3.0 * K * iq4 - Krr * iq2);
      const double fc = -(Kc * iq3 - Krc * iq2);
      const double u0 = P.m * wx - mj * w[0], u1 = P.m * wy - mj * w[1], u2 = P.m * wz - mj * w[2];
      const double du = d0 * u0 + d1 * u1 + d2 * u2;
      const double cc = fr * iq * du;
      out[0] += a.G * (f * u0 + cc * d0);
      out[1] += a.G * (f * u1 + cc * d1);
      out[2] += a.G * (f * u2 + cc * d2);
      mb -= a.G * f * (d0 * wx + d1 * wy + d2 * wz);
      const double tl = a.G * fc * mj * (d0 * w[0] + d1 * w[1] + d2 * w[2]);
      const double tp = -a.G * fc * P.m * (d0 * wx + d1 * wy + d2 * wz);
      if (P.rc > rcj) rcb += tl;
      if (P.rc >= rcj) rcb += tp;
    }
  }
}

// gragg_vjp for the lane's column of the column-parallel layout: reverse
// rounds from mtop = 2 (kk + 1) down, kk the last column with a weight (the
// columns past it have a zero adjoint and are left out), a column idle
// above its own sequence.
__device__ __forceinline__ void gragg_vjp_par(const HArgs& a, const Sys& S, const Par& P,
                                              const double y0[6], double H, const double ob[6],
                                              double yb[6], double& mb, double& rcb, int mtop) {
  const int nsub = 2 * (P.c + 1);
  const double hs = H / nsub;
  double tmp[6];
  gragg_par(a, S, P, y0, H, tmp, true, mtop);
  double Pa[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, Qa[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int m = mtop; m >= 0; --m) {
    const bool act = m <= nsub;
    const int mz = act ? m : nsub;
    double z[3], w[3], o[3];
    const double cw = m == nsub ? 0.5 * hs : (m == 0 ? hs : 2.0 * hs);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      z[c] = a.zpos[((size_t)mz * 3 + c) * a.nl + S.gl];
      w[c] = act ? cw * (m == nsub ? ob[3 + c] : Pa[3 + c]) : 0.0;
    }
    double mbl = 0.0, rcbl = 0.0;
    ha_vjp_par(a, S, P, z, w, o, mbl, rcbl);
    if (!act) continue;
    mb += mbl;
    rcb += rcbl;
    if (m == nsub) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Pa[c] = 0.5 * ob[c] + o[c];
        Pa[3 + c] = 0.5 * ob[3 + c] + 0.5 * hs * ob[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) Qa[c] = 0.5 * ob[c];
    } else if (m > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Qa[c] += o[c];
        Qa[3 + c] += 2.0 * hs * Pa[c];
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double t = Pa[c];
        Pa[c] = Qa[c];
        Qa[c] = t;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Qa[c] += Pa[c] + o[c];
        Qa[3 + c] += Pa[3 + c] + hs * Pa[c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) yb[c] += Qa[c];
}

// Adjoint of one group's BS over tau from y1 (the members' pre-drift
// state): yb holds the adjoint of the BS result in and that of y1 out.
__device__ __forceinline__ void bs_group_vjp(const HArgs& a, const Sys& S, unsigned long long M, bool mem,
                             double rc, const double y1[6], double yb[6], double& mb, double& rcb,
                             double* lh, int* lk, unsigned& fl) {
  double y[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) y[c] = y1[c];
  int nleaf = 0;
  const int rcode = bs_group<true>(a, S, M, mem, rc, y, lh, lk, &nleaf);
  __syncthreads();  // the substeps' lengths and columns (LDS) for every lane
  if (rcode < 0) {
    fl |= F_BS;
    return;
  }
  if (nleaf > kHLeaf) {
    fl |= F_ADJ_LEAF;
    return;
  }
  const Par P = par_of(S, M, rc);
  const int qi = __builtin_popcountll(M & ((1ull << S.lane) - 1ull)) & 7;  // body lane's slot
  for (int l = nleaf - 1; l >= 0; --l) {
    const double hh = lh[l];
    const int kk = lk[l];
    double yin[6], acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 6; ++c) yin[c] = a.leaf[((size_t)l * 6 + c) * a.nl + S.gl];
    if (P.sz <= kHPar) {
      // the columns side by side, then each member's columns added in order
      double y0[6], ob[6], col[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      const double wq = P.c <= kk ? kNW.w[kk][P.c] : 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        y0[c] = __shfl(yin[c], P.src, 64);
        ob[c] = wq * __shfl(yb[c], P.src, 64);
      }
      double mbl = 0.0, rcbl = 0.0;
      gragg_vjp_par(a, S, P, y0, hh, ob, col, mbl, rcbl, 2 * (kk + 1));
      double msum = 0.0, rsum = 0.0;
      for (int c8 = 0; c8 < kHPar; ++c8) {
        double v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = __shfl(col[c], 8 * c8 + qi, 64);
        const double mv = __shfl(mbl, 8 * c8 + qi, 64), rv = __shfl(rcbl, 8 * c8 + qi, 64);
        if (c8 <= kk) {
#pragma unroll
          for (int c = 0; c < 6; ++c) acc[c] += v[c];
          msum += mv;
          rsum += rv;
        }
      }
      if (mem) {
        mb += msum;
        rcb += rsum;
#pragma unroll
        for (int c = 0; c < 6; ++c) yb[c] = acc[c];
      }
      continue;
    }
    for (int q = 0; q <= kk; ++q) {
      const double wq = kNW.w[kk][q];
      double ob[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) ob[c] = wq * yb[c];
      gragg_vjp(a, S, M, mem, rc, yin, hh, 2 * (q + 1), ob, acc, mb, rcb);
    }
    if (mem) {
#pragma unroll
      for (int c = 0; c < 6; ++c) yb[c] = acc[c];
    }
  }
  __syncthreads();  // lh, lk are rewritten by the next group
}

// Radius adjoint (Eq. 6, the branch taken) into x^, v^, m^.
__device__ __forceinline__ void radius_vjp(const HArgs& a, const Sys& S, const double x[3], const double v[3],
                           double rcb, double xb[3], double vb[3], double& mb) {
  if (!S.act) return;
  const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  const double r = sqrt(r2);
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double inva = 2.0 / r - vv / S.Gm0;
  const double am = inva > 0.0 ? 1.0 / inva : r;
  const double cb = cbrt(S.m / (3.0 * S.m0));
  const double r1 = a.n1 * (am * cb);
  const double rv = a.n2 * a.absdt * sqrt(vv);
  if (r1 > rv) {
    const double k = rcb * a.n1 * cb;
    if (inva > 0.0) {
      const double a2 = am * am;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xb[c] += k * 2.0 * a2 * x[c] / (r2 * r);
        vb[c] += k * 2.0 * a2 * v[c] / S.Gm0;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) xb[c] += k * x[c] / r;
    }
    mb += rcb * a.n1 * am * cb / (3.0 * S.m);
  } else {
    const double k = rcb * a.n2 * a.absdt / sqrt(vv);
#pragma unroll
    for (int c = 0; c < 3; ++c) vb[c] += k * v[c];
  }
}

__device__ __forceinline__ Sys sys_of(const HArgs& a) {
  Sys S;
  S.lane = threadIdx.x & 63;
  const int s = blockIdx.x;
  S.n = a.off[s + 1] - a.off[s];
  S.act = S.lane < S.n;
  S.row = a.off[s] + (S.act ? S.lane : 0);
  S.gl = (size_t)s * 64 + S.lane;
  S.m0 = a.m0[s];
  S.Gm0 = a.G * S.m0;
  S.m = S.act ? a.xm[S.row].w : 0.0;
  S.all = S.n >= 64 ? ~0ull : ((1ull << S.n) - 1ull);
  return S;
}

__device__ __forceinline__ void load_body(const HArgs& a, const Sys& S, double x[3], double v[3]) {
  x[0] = 1.0e3 + S.lane;  // lanes past the system: far away, massless, never read
  x[1] = x[2] = v[0] = v[1] = v[2] = 0.0;
  if (S.act) {
    const double4 p = a.xm[S.row], q = a.vv[S.row];
    x[0] = p.x;
    x[1] = p.y;
    x[2] = p.z;
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
  }
}

__global__ __launch_bounds__(64) void k_hadj_fwd(HArgs a) {
  const Sys S = sys_of(a);
  double x[3], v[3];
  load_body(a, S, x, v);
  unsigned long long cand = precheck(a, S, x, radius(a, S, x, v));
  unsigned fl = 0u;
  for (int t = 0; t < a.T; ++t) {
    if (t % a.K == 0 && S.act) {
      double* c = a.ckpt + (size_t)(t / a.K) * 7 * a.nb;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        c[k * a.nb + S.row] = x[k];
        c[(3 + k) * a.nb + S.row] = v[k];
      }
      c[6 * a.nb + S.row] = __longlong_as_double((long long)cand);
    }
    StepVals R;
    hyb_step(a, S, x, v, cand, R, fl);
  }
  if (S.act) {
    a.xm[S.row] = make_double4(x[0], x[1], x[2], S.m);
    a.vv[S.row] = make_double4(v[0], v[1], v[2], 0.0);
  }
  if (fl) atomicOr(a.flags, fl);
}

__global__ __launch_bounds__(64) void k_hadj_bwd(HArgs a) {
  __shared__ double lh[kHLeaf];
  __shared__ int lk[kHLeaf];
  const Sys S = sys_of(a);
  double lx[3] = {0.0, 0.0, 0.0}, lv[3] = {0.0, 0.0, 0.0}, lm = 0.0;
  if (S.act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lx[c] = a.gxT[3 * (size_t)S.row + c];
      lv[c] = a.gvT[3 * (size_t)S.row + c];
    }
  }
  unsigned fl = 0u;
  for (int cseg = a.C - 1; cseg >= 0; --cseg) {
    const int t0 = cseg * a.K, t1 = min(a.T, t0 + a.K);
    double x[3], v[3];
    unsigned long long cand = 0ull;
    load_body(a, S, x, v);
    if (S.act) {
      const double* cp = a.ckpt + (size_t)cseg * 7 * a.nb;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        x[k] = cp[k * a.nb + S.row];
        v[k] = cp[(3 + k) * a.nb + S.row];
      }
      cand = (unsigned long long)__double_as_longlong(cp[6 * a.nb + S.row]);
    }
    // the segment replayed keeping every step's start, then its steps in
    // reverse, each recomputed from its start (one loop, so that the step's
    // code appears once)
    const int ns = t1 - t0;
    for (int it = 0; it < 2 * ns; ++it) {
      const bool rev = it >= ns;
      const int t = rev ? t1 - 1 - (it - ns) : t0 + it;
      double* tp = a.tape + (size_t)(t - t0) * 7 * a.nl;
      if (!rev) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tp[k * a.nl + S.gl] = x[k];
          tp[(3 + k) * a.nl + S.gl] = v[k];
        }
        tp[6 * a.nl + S.gl] = __longlong_as_double((long long)cand);
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          x[k] = tp[k * a.nl + S.gl];
          v[k] = tp[(3 + k) * a.nl + S.gl];
        }
        cand = (unsigned long long)__double_as_longlong(tp[6 * a.nl + S.gl]);
      }
      StepVals R;
      hyb_step(a, S, x, v, cand, R, fl);
      if (!rev) continue;
      const double rc = R.rc;
      double rcb = 0.0;
      // closing kick: v4 = v2 + h a_B(x3)
      double w[3] = {a.h * lv[0], a.h * lv[1], a.h * lv[2]};
      double xb[3] = {lx[0], lx[1], lx[2]}, vb[3] = {lv[0], lv[1], lv[2]};
      pair_vjp<false>(a, S, S.all, S.act, rc, R.x3, w, xb, lm, rcb);
      // second Sun kick: x3 = x2 + h P(v2)/m0
      double Sx[3];
      lane_sum3(S, xb, Sx);
      const double hm = a.h / S.m0;
#pragma unroll
      for (int c = 0; c < 3; ++c) vb[c] += hm * S.m * Sx[c];
      lm += hm * (R.v2[0] * Sx[0] + R.v2[1] * Sx[1] + R.v2[2] * Sx[2]);
      // drift: Kepler for bodies outside the groups, BS for each group
      double xb1[3] = {xb[0], xb[1], xb[2]}, vb1[3] = {vb[0], vb[1], vb[2]};
      if (S.act && R.label < 0) {
        const double lx2[3] = {xb[0], xb[1], xb[2]}, lv2[3] = {vb[0], vb[1], vb[2]};
        kepler_vjp(S.Gm0, a.dt, R.x1, R.v1, R.s, lx2, lv2, xb1, vb1);
      }
      unsigned long long roots = __builtin_amdgcn_ballot_w64(R.label == S.lane);
      for (; roots; roots &= roots - 1) {
        const int g = __builtin_ctzll(roots);
        const bool mem = R.label == g;
        const unsigned long long M = __builtin_amdgcn_ballot_w64(mem);
        const double y1[6] = {R.x1[0], R.x1[1], R.x1[2], R.v1[0], R.v1[1], R.v1[2]};
        double yb[6] = {xb[0], xb[1], xb[2], vb[0], vb[1], vb[2]};
        bs_group_vjp(a, S, M, mem, rc, y1, yb, lm, rcb, lh, lk, fl);
        if (mem) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            xb1[c] = yb[c];
            vb1[c] = yb[3 + c];
          }
        }
      }
      // first Sun kick: x1 = x0 + h P(v1)/m0
      lane_sum3(S, xb1, Sx);
#pragma unroll
      for (int c = 0; c < 3; ++c) vb1[c] += hm * S.m * Sx[c];
      lm += hm * (R.v1[0] * Sx[0] + R.v1[1] * Sx[1] + R.v1[2] * Sx[2]);
      // opening kick: v1 = v0 + h a_B(x0)
#pragma unroll
      for (int c = 0; c < 3; ++c) w[c] = a.h * vb1[c];
      pair_vjp<false>(a, S, S.all, S.act, rc, R.x0, w, xb1, lm, rcb);
      // radii of the step
      radius_vjp(a, S, R.x0, R.v0, rcb, xb1, vb1, lm);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        lx[c] = S.act ? xb1[c] : 0.0;
        lv[c] = S.act ? vb1[c] : 0.0;
      }
      if (!S.act) lm = 0.0;
    }
  }
  if (S.act) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.gx0[3 * (size_t)S.row + c] = lx[c];
      a.gv0[3 * (size_t)S.row + c] = lv[c];
    }
    a.gm[S.row] = lm;
  }
  if (fl) atomicOr(a.flags, fl);
}

HArgs hargs(const BatchWs& b, const StepConsts& c, int T, int K) {
  HArgs a{};
  a.xm = b.xm;
  a.vv = b.vv;
  a.off = b.off;
  a.m0 = b.m0;
  a.flags = &b.st->flags;
  a.nsys = b.nsys;
  a.T = T;
  a.K = K;
  a.C = (T + K - 1) / K;
  a.nl = b.nsys * 64;
  a.nb = b.nb;
  a.G = c.G;
  a.dt = c.dt;
  a.h = c.h;
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.pf = c.pf;
  a.absdt = fabs(c.dt);
  a.bs_tol = c.bs_tol;
  a.bs_depth = c.bs_max_depth;
  a.max_iter = c.kepler_max_iter;
  return a;
}

}  // namespace

size_t hadj_ckpt_bytes(int64_t nb, int T, int K) {
  return (size_t)((T + K - 1) / K) * 7 * (size_t)nb * sizeof(double);
}

size_t hadj_work_bytes(int nsys, int K) {
  const size_t nl = (size_t)nsys * 64;
  return nl * sizeof(double) * (7 * (size_t)K + 6 * kHLeaf + 3 * kHPos);
}

hipError_t hadj_forward(const BatchWs& b, const StepConsts& c, int T, int K, double* ckpt,
                        hipStream_t s) {
  HArgs a = hargs(b, c, T, K);
  a.ckpt = ckpt;
  hipLaunchKernelGGL(k_hadj_fwd, dim3(b.nsys), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t hadj_backward(const BatchWs& b, const StepConsts& c, int T, int K, double* ckpt,
                         double* work, const double* gxT, const double* gvT, double* gx0,
                         double* gv0, double* gm, hipStream_t s) {
  HArgs a = hargs(b, c, T, K);
  a.ckpt = ckpt;
  const size_t nl = (size_t)b.nsys * 64;
  a.tape = work;
  a.leaf = a.tape + nl * 7 * (size_t)K;
  a.zpos = a.leaf + nl * 6 * (size_t)kHLeaf;
  a.gxT = gxT;
  a.gvT = gvT;
  a.gx0 = gx0;
  a.gv0 = gv0;
  a.gm = gm;
  hipLaunchKernelGGL(k_hadj_bwd, dim3(b.nsys), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace genga
