// Device code of the Bulirsch-Stoer integration of H_A (Eq. 1) for one
// close-encounter group (Sec. 3.2.6), shared by the main-mode and the
// test-particle kernels.  One wave integrates one group.
#pragma once

#include <climits>

#include "device_math.h"

namespace genga {

constexpr int kBsCols = 8;
constexpr int kBsMaxAttempts = 1 << 16;  // substep attempts per group and step

// dv/dt of H_A for the lane's body: the fixed star plus the (1-K) part of the
// group's pair terms (Eq. 1 gradient); other members' data by lane reads.
__device__ __forceinline__ void ha_accel(int sz, int lane, double x, double y,
                                         double z, double m, double rc,
                                         double G, double Gm0, double& ax,
                                         double& ay, double& az) {
  const double r2 = x * x + y * y + z * z;
  const double ir = rsqrt_nr(r2);
  const double fs = -Gm0 * (ir * ir * ir);
  ax = fs * x;
  ay = fs * y;
  az = fs * z;
  for (int j = 0; j < sz; ++j) {
    const double xj = readlane_d(x, j), yj = readlane_d(y, j), zj = readlane_d(z, j);
    const double mj = readlane_d(m, j), rcj = readlane_d(rc, j);
    const double dx = xj - x, dy = yj - y, dz = zj - z;
    const double q2 = dx * dx + dy * dy + dz * dz;
    const double rij = fmax(rc, rcj);
    // the term vanishes exactly beyond rc_ij (K = 1, K' = 0)
    if (j != lane && q2 < rij * rij * (1.0 + 1e-12)) {
      const double iq = rsqrt_nr(q2);
      const double iq2 = iq * iq;
      double K, dK;
      changeover(q2 * iq, rij, K, dK);
      const double s = G * mj * ((1.0 - K) * iq2 * iq + dK * iq2);
      ax += s * dx;
      ay += s * dy;
      az += s * dz;
    }
  }
}

// Gragg's modified midpoint rule over H with nsub substeps (one wave, one
// body per lane).
__device__ __forceinline__ void mmid(int sz, int lane, const double y0[6], double H, int nsub,
                     double m, double rc, double G, double Gm0, double out[6]) {
  const double hs = H / nsub;
  double ym[6], yn[6], d[6];
  ha_accel(sz, lane, y0[0], y0[1], y0[2], m, rc, G, Gm0, d[3], d[4], d[5]);
  d[0] = y0[3];
  d[1] = y0[4];
  d[2] = y0[5];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    ym[c] = y0[c];
    yn[c] = y0[c] + hs * d[c];
  }
  for (int s = 1; s < nsub; ++s) {
    ha_accel(sz, lane, yn[0], yn[1], yn[2], m, rc, G, Gm0, d[3], d[4], d[5]);
    d[0] = yn[3];
    d[1] = yn[4];
    d[2] = yn[5];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double t = ym[c] + 2.0 * hs * d[c];
      ym[c] = yn[c];
      yn[c] = t;
    }
  }
  ha_accel(sz, lane, yn[0], yn[1], yn[2], m, rc, G, Gm0, d[3], d[4], d[5]);
  d[0] = yn[3];
  d[1] = yn[4];
  d[2] = yn[5];
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c] = 0.5 * (ym[c] + yn[c] + hs * d[c]);
}

__device__ __forceinline__ double relerr3(const double* A, const double* B) {
  const double d0 = A[0] - B[0], d1 = A[1] - B[1], d2 = A[2] - B[2];
  const double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  const double den = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
  return den > 0.0 ? num / den : num;
}

// One BS attempt over H: columns n_k = 2k (k = 1..8), Aitken-Neville
// extrapolation in h^2 kept in LDS (R[col][comp][lane]), accepted at the first
// column k >= 2 whose per-body relative error (max over the group) is within
// tol.  Returns true and the extrapolated state in y on success.
__device__ __forceinline__ bool bs_attempt(int sz, int lane, double y[6], double H, double m,
                           double rc, double G, double Gm0, double tol,
                           double (*R)[6][64]) {
  for (int k = 0; k < kBsCols; ++k) {
    const int nk = 2 * (k + 1);
    double t[6];
    mmid(sz, lane, y, H, nk, m, rc, G, Gm0, t);
    for (int j = 1; j <= k; ++j) {
      const double ratio = (double)nk / (double)(2 * (k - j + 1));
      const double den = ratio * ratio - 1.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double u = t[c] + (t[c] - R[j - 1][c][lane]) / den;
        R[j - 1][c][lane] = t[c];
        t[c] = u;
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) R[k][c][lane] = t[c];
    if (k >= 1) {
      double A[6], B[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        A[c] = R[k][c][lane];
        B[c] = R[k - 1][c][lane];
      }
      double e = fmax(relerr3(A, B), relerr3(A + 3, B + 3));
      if (lane >= sz) e = 0.0;
      e = wave_max(e);
      if (e <= tol) {
#pragma unroll
        for (int c = 0; c < 6; ++c) y[c] = A[c];
        return true;
      }
    }
  }
  return false;
}

// Collision of two massive members over an accepted substep (Sec. 3.2.7,
// the encounter test of Eqs. 10-12 reused between BS steps): the relative
// states of the pair at its start (o) and end (e), the substep length h and
// the sum of the radii Rs; true when the separation dips below Rs.
__device__ __forceinline__ bool pair_touches(double h, const double o[6], const double e[6],
                                             double Rs) {
  if (!(Rs > 0.0)) return false;
  return hermite_dmin2(h, o[0], o[1], o[2], o[3], o[4], o[5], e[0], e[1], e[2], e[3], e[4],
                       e[5]) < Rs * Rs;
}

// Binary refinement over [0, H]: a failed substep is halved; after finishing
// both halves of a node the next sibling is tried at the node's length.
// With ckey (massive groups with radii; Rb the lane's member radius): after
// each accepted substep every member pair whose radii sum is positive is
// tested over the substep; at the first pair (a, b), a < b in member order,
// that touches, the integration stops at the start of that substep and
// returns 1 with a * 64 + b in *ckey and the covered part of [0, H] in *cpos
// (units of H / 2^D).
__device__ __forceinline__ int bs_integrate(int sz, int lane, double y[6], double H, double m,
                            double rc, double G, double Gm0, double tol,
                            int D, double (*R)[6][64], long long* nsub, double Rb = 0.0,
                            int* ckey = nullptr, long long* cpos = nullptr) {
  long long pos = 0;
  const long long total = 1ll << D;
  int d = 0;
  int attempts = 0;
  const bool coll = ckey && __ballot(lane < sz && Rb > 0.0) != 0ull;
  while (pos < total) {
    if (++attempts > kBsMaxAttempts) return -1;
    double yt[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) yt[c] = y[c];
    if (bs_attempt(sz, lane, yt, ldexp(H, -d), m, rc, G, Gm0, tol, R)) {
      if (coll) {
        const double h = ldexp(H, -d);
        int best = INT_MAX;
        for (int j = 0; j < sz; ++j) {
          double o[6], e[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            o[c] = readlane_d(y[c], j) - y[c];
            e[c] = readlane_d(yt[c], j) - yt[c];
          }
          const double Rs = Rb + readlane_d(Rb, j);
          if (lane < sz && j > lane && pair_touches(h, o, e, Rs)) best = min(best, lane * 64 + j);
        }
        best = wave_min_i(best);
        if (best != INT_MAX) {
          *ckey = best;
          *cpos = pos;
          return 1;
        }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) y[c] = yt[c];
      ++*nsub;
      pos += 1ll << (D - d);
      while (d > 0 && (pos % (1ll << (D - d + 1))) == 0) --d;
    } else {
      ++d;
      if (d > D) return -1;
    }
  }
  return 0;
}

// ---- groups of up to 8 members: all columns, and several depths, at once ----
// A wave of 64 lanes holds S = 8/P speculative refinement depths x 8 columns
// x P member slots (P = 2, 4 or 8 >= group size); s = depth slot, c = column,
// b = member:
//   P = 2:   lane = 16 s + 2 c + b  (partner lane ^ 1: a quad permutation)
//   P >= 4:  lane = 8 P s + 8 b + c (columns adjacent)
// so that the column neighbour c - 1 of the tableau is a DPP row shift away
// (by 2 or by 1 lanes, inside the row of 16).  Column c integrates the
// modified midpoint rule with n_c = 2 (c + 1) substeps; members exchange
// positions by lane shuffles.  Slot s attempts the substep of length H / 2^s
// from the same start: exactly the attempts the sequential scheme makes
// after s failures (the first half of each halving).  The Aitken-Neville
// tableau is built across the columns (T[c][j] needs T[c-1][j-1]); column k
// is tested when it completes (after 2 k + 3 force evaluations), and each
// slot keeps its first column within tolerance.  The result is the first
// accepted slot in sequential order, so the substeps taken equal those of
// one-at-a-time evaluation.
// TP: member 0 is a massless test particle and the other members feel only
// the star (a test-particle encounter, Sec. 3.3).
constexpr int kBsPar = 8;

template <int P>
__device__ __forceinline__ int par_lane(int s, int c, int b) {
  return P == 2 ? 16 * s + 2 * c + b : 8 * P * s + 8 * b + c;
}
template <int P>
__device__ __forceinline__ int par_col(int lane) {
  return P == 2 ? (lane >> 1) & 7 : lane & 7;
}
template <int P>
__device__ __forceinline__ int par_memb(int lane) {
  return P == 2 ? lane & 1 : (lane >> 3) & (P - 1);
}
// ballot bits of the P members of slot s, column c
template <int P>
__device__ __forceinline__ unsigned long long par_members(int s, int c) {
  constexpr unsigned long long kStride = P == 2 ? 3ull : (P == 4 ? 0x01010101ull : 0x0101010101010101ull);
  return kStride << par_lane<P>(s, c, 0);
}

template <int P>
struct ParBody {
  int lane[P];     // lane of partner q (member (b + q) mod sz), q >= 1
  double m[P];     // partner mass
  double rcij[P];  // pair radius max(rc_b, rc_j)
  double i09[P];   // 1 / (0.9 rc_ij), 0 when rc_ij = 0
  double near2[P]; // rc_ij^2 (1 + 1e-12): beyond it the pair's H_A term is 0
  int lback[P];    // lane of member (b - q) mod sz
  double mback[P]; // its mass
};

// Lane shuffles of a double: generic (ds_bpermute) or, for a source lane a
// fixed distance away inside the same row of 16 lanes, a DPP move.
__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, 64); }

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int2 p = *reinterpret_cast<int2*>(&v);
  int2 q;
  q.x = __builtin_amdgcn_update_dpp(0, p.x, CTRL, 0xF, 0xF, true);
  q.y = __builtin_amdgcn_update_dpp(0, p.y, CTRL, 0xF, 0xF, true);
  return *reinterpret_cast<double*>(&q);
}
constexpr int kDppQuadSwap1 = 0xB1;     // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppQuadSwap2 = 0x4E;     // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppRowHalfMirror = 0x141;  // lane 7 - i inside each 8 lanes
constexpr int kDppRowMirror = 0x140;      // lane 15 - i inside each row
constexpr int kDppRowShr2 = 0x112;      // row_shr:2: lane - 2 inside the row
constexpr int kDppRowShr1 = 0x111;      // row_shr:1: lane - 1 inside the row

// (1-K)-weighted pair factor f of H_A (Eq. 1 gradient, without the partner's
// mass) times d = x_j - x_b, or 0 where use is false.  Beyond rc_ij
// (q2 >= near2, a margin far above the rounding of y) the term is exactly 0
// (y clamps to 1: K = 1, K' = 0), and it is 0 for rc_ij = 0 (near2 = 0).
// Branch-free, so that the compiler can interleave independent terms.
__device__ __forceinline__ void ha_pair(double dx, double dy, double dz, double rc, double i09,
                                        double near2, double G, bool use, double& fx,
                                        double& fy, double& fz) {
  const double q2 = dx * dx + dy * dy + dz * dz;
  const double iq = rsqrt_nr(q2);
  const double iq2 = iq * iq;
  double K, dK;
  changeover_clamped(q2 * iq, rc, i09, K, dK);
  double f = G * ((1.0 - K) * iq2 * iq + dK * iq2);
  f = (use && q2 < near2) ? f : 0.0;
  fx = f * dx;
  fy = f * dy;
  fz = f * dz;
}

// dv/dt of H_A for member b of a group of sz members, P/2 < sz <= P (P = 2,
// 4, 8): the fixed star plus the group's pair terms.
template <int P, bool TP>
__device__ __forceinline__ void ha_accel_par(int sz, int b, double x, double y,
                                             double z, const ParBody<P>& Q,
                                             double G, double Gm0, double& ax,
                                             double& ay, double& az) {
  const double r2 = x * x + y * y + z * z;
  const double ir = rsqrt_nr(r2);
  const double fs = -Gm0 * (ir * ir * ir);
  ax = fs * x;
  ay = fs * y;
  az = fs * z;
  if (!TP && P == 2) {  // the partner is lane ^ 1
    const double dx = dpp_d<kDppQuadSwap1>(x) - x, dy = dpp_d<kDppQuadSwap1>(y) - y,
                 dz = dpp_d<kDppQuadSwap1>(z) - z;
    double fx, fy, fz;
    ha_pair(dx, dy, dz, Q.rcij[1], Q.i09[1], Q.near2[1], G, true, fx, fy, fz);
    ax += Q.m[1] * fx;
    ay += Q.m[1] * fy;
    az += Q.m[1] * fz;
    return;
  }
  if (!TP) {
    // Each unordered pair once: member b takes partners b + q (mod sz) for
    // 2 q <= sz (at 2 q = sz only b < q does) and receives the reaction of
    // the pair that member b - q took, scaled by that member's mass.  With
    // P/2 < sz the offsets q <= P/4 always exist, so their terms need no
    // test and form one block of independent work.
#pragma unroll
    for (int q = 1; q <= P / 2; ++q) {
      if (q > P / 4 && 2 * q > sz) break;
      const bool half = 2 * q == sz;
      const double dx = shfl_d(x, Q.lane[q]) - x, dy = shfl_d(y, Q.lane[q]) - y,
                   dz = shfl_d(z, Q.lane[q]) - z;
      double fx, fy, fz;
      ha_pair(dx, dy, dz, Q.rcij[q], Q.i09[q], Q.near2[q], G, !half || b < q, fx, fy, fz);
      ax += Q.m[q] * fx;
      ay += Q.m[q] * fy;
      az += Q.m[q] * fz;
      const double rx = shfl_d(fx, Q.lback[q]), ry = shfl_d(fy, Q.lback[q]),
                   rz = shfl_d(fz, Q.lback[q]);
      const double mb = (!half || b >= q) ? Q.mback[q] : 0.0;
      ax -= mb * rx;
      ay -= mb * ry;
      az -= mb * rz;
    }
    return;
  }
  // test-particle group: member 0 is the massless particle, the planets
  // (b >= 1) feel only the star
#pragma unroll
  for (int q = 1; q < P; ++q) {
    if (q >= sz) break;
    double xj, yj, zj;
    if (P == 2) {
      xj = dpp_d<kDppQuadSwap1>(x);
      yj = dpp_d<kDppQuadSwap1>(y);
      zj = dpp_d<kDppQuadSwap1>(z);
    } else {
      xj = shfl_d(x, Q.lane[q]);
      yj = shfl_d(y, Q.lane[q]);
      zj = shfl_d(z, Q.lane[q]);
    }
    double fx, fy, fz;
    ha_pair(xj - x, yj - y, zj - z, Q.rcij[q], Q.i09[q], Q.near2[q], G, b == 0, fx, fy, fz);
    ax += Q.m[q] * fx;
    ay += Q.m[q] * fy;
    az += Q.m[q] * fz;
  }
}

// |A - B| <= tol |A| (|A - B| <= tol when A = 0), squared: the per-body
// relative-change test without square roots or divisions.
__device__ __forceinline__ bool within3(const double* A, const double* B, double tol2) {
  const double d0 = A[0] - B[0], d1 = A[1] - B[1], d2 = A[2] - B[2];
  const double n2 = d0 * d0 + d1 * d1 + d2 * d2;
  const double a2 = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
  return n2 <= tol2 * (a2 > 0.0 ? a2 : 1.0);
}

// One speculative round: returns the accepted depth offset (0..S-1), with the
// accepted state in y, or -1 when every slot failed.
template <int P, bool TP>
__device__ __forceinline__ int bs_round_par(int sz, double y[6], double H,
                                            const ParBody<P>& Q, double G,
                                            double Gm0, double tol) {
  const int lane = threadIdx.x & 63;
  const int s = lane / (kBsPar * P);
  const int c = par_col<P>(lane);
  const int b = par_memb<P>(lane);
  const int nsub = 2 * (c + 1);
  const double hs = ldexp(H, -s) / nsub;
  const double tol2 = tol >= 0.0 ? tol * tol : -1.0;  // a negative tolerance accepts nothing
  // Gragg states in two buffers used in turn: A holds the even-numbered
  // points z_0, z_2, ..., B the odd ones, so no copies are needed per substep
  double A[6], B[6], T0[6], yacc[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    A[q] = y[q];
    B[q] = y[q];
    T0[q] = y[q];
    yacc[q] = y[q];
  }
  // Neville weights of this lane's column: 1/((n_c/n_{c-j})^2 - 1) =
  // (c-j+1)^2 / ((c+1)^2 - (c-j+1)^2), j = 1..c
  double wj[kBsCols];
#pragma unroll
  for (int j = 1; j < kBsCols; ++j) {
    const int pp = c + 1, qq = c - j + 1;
    wj[j] = j <= c ? (double)(qq * qq) / (double)(pp * pp - qq * qq) : 0.0;
  }
  unsigned accm = 0u;  // slots that have accepted a column (bit s)
  // Evaluation e is at z_e: z_1 = z_0 + hs f(z_0), z_{e+1} = z_{e-1} +
  // 2 hs f(z_e) while e < nsub; the lane's points stay fixed after z_nsub
  // (step 0), and T0 = (z_{nsub-1} + z_nsub + hs f(z_nsub)) / 2.
  for (int e = 0; e <= 2 * kBsCols; e += 2) {
    double d[6];
    ha_accel_par<P, TP>(sz, b, A[0], A[1], A[2], Q, G, Gm0, d[3], d[4], d[5]);
    d[0] = A[3];
    d[1] = A[4];
    d[2] = A[5];
    if (e == nsub) {
#pragma unroll
      for (int q = 0; q < 6; ++q) T0[q] = 0.5 * (B[q] + A[q] + hs * d[q]);
    }
    {
      const double hf = e < nsub ? (e == 0 ? hs : 2.0 * hs) : 0.0;
#pragma unroll
      for (int q = 0; q < 6; ++q) B[q] = B[q] + hf * d[q];
    }
    if (e >= 4) {
      const int k = e / 2 - 1;  // column completed by this evaluation
      // Aitken-Neville across the columns: T[c][j] needs T[c-1][j-1] (lane - P).
      // Only column k's lanes are read: after j steps lane k holds T[k][j],
      // built from lane k-1 after j-1 steps, ..., lane k-j's T0, all of
      // them inside their own row (j <= c).  Lanes past their row (w = 0)
      // keep computing, and whatever they hold never reaches lane k.
      double cur[6], sub[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        cur[q] = T0[q];
        sub[q] = T0[q];
      }
#pragma unroll
      for (int j = 1; j < kBsCols; ++j) {
        if (j > k) break;
        if (j == k) {
#pragma unroll
          for (int q = 0; q < 6; ++q) sub[q] = cur[q];  // T[k][k-1] in lane k
        }
        const double w = wj[j];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const double nb = P == 2 ? dpp_d<kDppRowShr2>(cur[q]) : dpp_d<kDppRowShr1>(cur[q]);
          cur[q] = fma(cur[q] - nb, w, cur[q]);
        }
      }
      const double* diag = cur;  // T[k][k] in lane k
      // column k of every slot: accepted unless one of its members fails
      const bool bad = c == k && b < sz && !(within3(diag, sub, tol2) && within3(diag + 3, sub + 3, tol2));
      const unsigned long long badm = __ballot(bad);
      unsigned now = 0u;
#pragma unroll
      for (int t = 0; t < kBsPar / P; ++t)
        if (!((accm >> t) & 1u) && (badm & par_members<P>(t, k)) == 0ull)
          now |= 1u << t;
      if (now) {
        // the accepted state of this slot's column k, for every lane of the slot
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const double g = shfl_d(diag[q], par_lane<P>(s, k, b));
          if ((now >> s) & 1u) yacc[q] = g;
        }
        accm |= now;
      }
      // slot 0 decided: nothing can precede it
      if (accm & 1u) break;
    }
    if (e == 2 * kBsCols) break;
    ha_accel_par<P, TP>(sz, b, B[0], B[1], B[2], Q, G, Gm0, d[3], d[4], d[5]);
    d[0] = B[3];
    d[1] = B[4];
    d[2] = B[5];
    const double hf = e + 1 < nsub ? 2.0 * hs : 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) A[q] = A[q] + hf * d[q];
  }
  // first accepted slot in sequential order
  if (accm == 0u) return -1;
  const int sacc = __ffs(accm) - 1;
#pragma unroll
  for (int q = 0; q < 6; ++q) y[q] = shfl_d(yacc[q], par_lane<P>(sacc, 0, b));
  return sacc;
}

// Test-particle groups (TP) with R2 >= 0 in some lane: after each accepted
// substep, lane b (a planet member) tests its separation from member 0 over
// the substep with the Hermite rule; below sqrt(R2) (the sum of the radii)
// the integration stops at the start of that substep and returns 1, with the
// lowest such member in *cb and the covered part of [0, H] in *cpos (units of
// H / 2^D).  Returns 0 when H is covered, -1 when the depth is exhausted.
// Massive groups (!TP) with mR (the members' physical radii, any memory):
// every member pair with a positive radius sum is tested the same way, and
// the first pair (a, b), a < b, that touches stops the integration with
// a * 64 + b in *cb.
template <int P, bool TP>
__device__ __forceinline__ int bs_integrate_par(int sz, double y[6], double H,
                                                const ParBody<P>& Q, double G,
                                                double Gm0, double tol, int D,
                                                long long* nsub, double R2 = -1.0,
                                                int* cb = nullptr,
                                                long long* cpos = nullptr,
                                                const double* mR = nullptr) {
  constexpr int S = kBsPar / P;
  const int lane = threadIdx.x & 63;
  const int b = par_memb<P>(lane);
  const bool coll = TP && __ballot(R2 >= 0.0) != 0ull;
  const double Rb = (!TP && mR && b < sz) ? mR[b] : 0.0;
  const bool mcoll = !TP && mR && __ballot(Rb > 0.0) != 0ull;
  long long pos = 0;
  const long long total = 1ll << D;
  int d = 0;
  int attempts = 0;
  while (pos < total) {
    if (++attempts > kBsMaxAttempts) return -1;
    const int smax = min(S, D - d + 1);  // never beyond the depth limit
    double yt[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) yt[q] = y[q];
    int sa = bs_round_par<P, TP>(sz, yt, ldexp(H, -d), Q, G, Gm0, tol);
    if (sa >= smax) sa = -1;
    if (sa >= 0) {
      d += sa;
      if (coll) {
        const int l0 = par_lane<P>(lane / (kBsPar * P), par_col<P>(lane), 0);
        double o[6], e[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          o[q] = y[q] - __shfl(y[q], l0, 64);
          e[q] = yt[q] - __shfl(yt[q], l0, 64);
        }
        const double d2 = hermite_dmin2(ldexp(H, -d), o[0], o[1], o[2], o[3], o[4], o[5],
                                        e[0], e[1], e[2], e[3], e[4], e[5]);
        const bool hit = b >= 1 && b < sz && R2 >= 0.0 && d2 < R2;
        const unsigned long long hm = __ballot(hit) & par_members<P>(0, 0);
        if (hm != 0ull) {
          *cb = par_memb<P>(__ffsll((long long)hm) - 1);
          *cpos = pos;
          return 1;
        }
      }
      if (mcoll) {
        const double h = ldexp(H, -d);
        int best = INT_MAX;
#pragma unroll
        for (int q = 1; q < P; ++q) {
          if (q >= sz) break;
          const int j = b + q < sz ? b + q : b + q - sz;  // member (b + q) mod sz
          double o[6], e[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            o[c] = shfl_d(y[c], Q.lane[q]) - y[c];
            e[c] = shfl_d(yt[c], Q.lane[q]) - yt[c];
          }
          const double Rs = b < sz ? Rb + mR[j] : 0.0;
          if (b < sz && b < j && pair_touches(h, o, e, Rs)) best = min(best, b * 64 + j);
        }
        if (!((par_members<P>(0, 0) >> lane) & 1ull)) best = INT_MAX;
        best = wave_min_i(best);
        if (best != INT_MAX) {
          *cb = best;
          *cpos = pos;
          return 1;
        }
      }
#pragma unroll
      for (int q = 0; q < 6; ++q) y[q] = yt[q];
      ++*nsub;
      pos += 1ll << (D - d);
      while (d > 0 && (pos % (1ll << (D - d + 1))) == 0) --d;
    } else {
      d += smax;
      if (d > D) return -1;
    }
  }
  return 0;
}

// The per-lane view of a group of sz members (P the smallest of 2, 4, 8
// not below sz) that the force evaluations use: each partner's lane, mass,
// critical radius and changeover constants, and the member whose reaction
// this lane receives; mm[] and mrc[] (any memory) hold every member's mass
// and critical radius.
template <int P>
__device__ __forceinline__ ParBody<P> par_body(int sz, const double* mm, const double* mrc) {
  const int lane = threadIdx.x & 63;
  const int b = par_memb<P>(lane);
  const double rcb = b < sz ? mrc[b] : 0.0;
  ParBody<P> Q;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    int j = b + q;
    j = j >= sz ? j - sz : j;
    j = j >= sz ? j - sz : j;  // dummy slots (b >= sz) wrap twice at most
    Q.lane[q] = lane + par_lane<P>(0, 0, j) - par_lane<P>(0, 0, b);
    const int jb = ((b - q) % sz + sz) % sz;  // member (b - q) mod sz (dummies too)
    Q.lback[q] = lane + par_lane<P>(0, 0, jb) - par_lane<P>(0, 0, b);
    Q.mback[q] = q < sz ? mm[jb] : 0.0;
    Q.m[q] = 0.0;
    Q.rcij[q] = 0.0;
    Q.i09[q] = 0.0;
    Q.near2[q] = 0.0;
    if (q < sz) {
      Q.m[q] = mm[j];
      Q.rcij[q] = fmax(rcb, mrc[j]);
      Q.i09[q] = Q.rcij[q] > 0.0 ? 1.0 / (0.9 * Q.rcij[q]) : 0.0;
      Q.near2[q] = Q.rcij[q] > 0.0 ? Q.rcij[q] * Q.rcij[q] * (1.0 + 1e-12) : 0.0;
    }
  }
  return Q;
}

// One group of sz members over H, P the smallest of 2, 4, 8 not below sz
// (so P/2 < sz <= P; the pair terms rely on it).  Every lane of member b =
// par_memb<P>(lane) holds the member's start state in y (dummy state for
// b >= sz); mm[] and mrc[] (any memory) give every member's mass and critical
// radius.  On return y holds member b's state after H in each of its lanes
// (par_lane<P>(0, 0, b) among them).
template <int P, bool TP>
__device__ __forceinline__ int bs_group(int sz, double y[6], const double* mm,
                                        const double* mrc, double H, double G,
                                        double Gm0, double tol, int D,
                                        long long* nsub, double R2 = -1.0,
                                        int* cb = nullptr, long long* cpos = nullptr,
                                        const double* mR = nullptr) {
  const ParBody<P> Q = par_body<P>(sz, mm, mrc);
  return bs_integrate_par<P, TP>(sz, y, H, Q, G, Gm0, tol, D, nsub, R2, cb, cpos, mR);
}

// The merger of Sec. 3.2.7 of survivor s and absorbed body g (states ys, yg:
// x then v): mass and momentum add up, the new body sits at the centre of
// mass with its velocity, its spin is both spins plus the pair's orbital
// angular momentum about that centre, its radius that of the summed volume.
// Returns the internal energy U = 1/2 m_s m_g/(m_s+m_g) v_sg^2 - G m_s m_g/r_sg.
__device__ __forceinline__ double merge_bodies(double G, double ms, double mg, const double* ys,
                                               const double* yg, double Rs, double Rg,
                                               const double* ss, const double* sg, double& M,
                                               double* y, double& R, double* S) {
  M = ms + mg;
#pragma unroll
  for (int k = 0; k < 6; ++k) y[k] = (ms * ys[k] + mg * yg[k]) / M;
  double di[3], ui[3], dj[3], uj[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    di[k] = ys[k] - y[k];
    ui[k] = ys[3 + k] - y[3 + k];
    dj[k] = yg[k] - y[k];
    uj[k] = yg[3 + k] - y[3 + k];
  }
  const double li[3] = {di[1] * ui[2] - di[2] * ui[1], di[2] * ui[0] - di[0] * ui[2],
                        di[0] * ui[1] - di[1] * ui[0]};
  const double lj[3] = {dj[1] * uj[2] - dj[2] * uj[1], dj[2] * uj[0] - dj[0] * uj[2],
                        dj[0] * uj[1] - dj[1] * uj[0]};
#pragma unroll
  for (int k = 0; k < 3; ++k) S[k] = ss[k] + sg[k] + ms * li[k] + mg * lj[k];
  R = cbrt(Rs * Rs * Rs + Rg * Rg * Rg);
  const double dv0 = ys[3] - yg[3], dv1 = ys[4] - yg[4], dv2 = ys[5] - yg[5];
  const double dx0 = ys[0] - yg[0], dx1 = ys[1] - yg[1], dx2 = ys[2] - yg[2];
  return 0.5 * ms * mg / M * (dv0 * dv0 + dv1 * dv1 + dv2 * dv2) -
         G * ms * mg / sqrt(dx0 * dx0 + dx1 * dx1 + dx2 * dx2);
}

}  // namespace genga
