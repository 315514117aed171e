// Test-particle mode (Sec. 3.3): massless particles feel at most 32 massive
// bodies and nothing else.  The massive bodies take the main-mode step; then
// one lane per particle runs the particle's whole step in one pass:
//   k_tp_main  opening kick (planets at the start of the step), Sun kick with
//              the planets' momentum, Kepler drift, Hermite test against the
//              particle's candidate planets; particles without an encounter
//              finish the step here (second Sun kick, closing kick, new
//              candidate mask); the others are compacted into a list.  One
//              more block, beside the particles' blocks: each planet's
//              Gragg sequences and extrapolation over the whole step (it
//              feels only the star inside a particle's group), the same for
//              every particle that meets it
//   k_tp_scan  offsets of each block's listed particles (one workgroup)
//   k_tp_bs1   eight lanes (one per extrapolation column) per particle
//              meeting one planet: the BS attempt over the whole step with
//              the planet taken from that table; most passages end here
//   k_tp_bs    one wave per remaining particle: BS of the particle with the
//              planets it encounters (planets feel only the star there) with
//              binary refinement, then the rest of its step
// A particle that comes closer to a planet than the sum of their physical
// radii during a BS substep is removed there and reported (Sec. 3.3).
// Counters are kept per block or wave (no same-address atomics on the step
// path) and summed when read.
// Particle state is stored as SoA (x[3][ntp], v[3][ntp]) plus a 32-bit
// candidate mask: 52 bytes read and written per particle and step.  A removed
// particle's x and v are NaN; every kernel skips it.
#include <algorithm>
#include <climits>
#include <vector>

#include "bs_device.h"
#include "device_math.h"
#include "genga_impl.h"

namespace genga {
namespace {

inline int ceil_div64(int64_t a, int b) { return (int)((a + b - 1) / b); }



__device__ __forceinline__ unsigned lanemask_count_tp(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

struct TpArgs {
  double* __restrict__ x;        // [3][ntp]
  double* __restrict__ v;        // [3][ntp]
  unsigned* __restrict__ mask;   // candidate planets of each particle
  const double4* __restrict__ px0;    // planets at the start of the step (w = m)
  const double4* __restrict__ ppre;   // planets before the drift
  const double4* __restrict__ vpre;
  const double4* __restrict__ ppost;  // planets after the drift, before BS
  const double4* __restrict__ vpost;
  const double4* __restrict__ pfin;   // planets at the end of the step
  const double* __restrict__ rc;      // planets' radii of the step
  const double* __restrict__ partP;   // planets' momentum partials (opening kick)
  DevStat* __restrict__ st;
  int* __restrict__ bs_idx;           // listed particles
  unsigned* __restrict__ bs_mask;     // their encounter planets
  unsigned* __restrict__ bs_emask;    // the same, kept for the encounter report
  double* __restrict__ enc_d2;        // Hermite minimum per encounter [nm][ntp]
  double* __restrict__ enc_rc2;       // its threshold [nm][ntp]
  double* __restrict__ bs_rct;        // their radii
  double* __restrict__ bs_y;          // their pre-drift state [6][cap]
  const double* __restrict__ rad;     // radii: planets [32], particles [ntp]
  CollRec* __restrict__ coll;         // removal reports
  int* __restrict__ blk_cnt;          // listed particles of each 256-particle block
  int* __restrict__ blk_off;          // their exclusive prefix sum [nb + 1]
  int* __restrict__ blk_enc;          // encounters of each block, last step
  unsigned long long* __restrict__ blk_enc_tot;
  int* __restrict__ blk_kit;          // largest Kepler iteration count per block
  unsigned long long* __restrict__ khist;  // Kepler iterations per block [nb][bins]
  unsigned long long* __restrict__ sub;  // accepted BS substeps per block / wave
  double* __restrict__ pl;            // planets' full-step BS table
  int64_t* __restrict__ rq;           // entries left to the wave path
  int* __restrict__ rq_cnt;           // their count
  int64_t ntp, cap, nb;
  int nm, nblk, enc_free, max_iter;
  double G, h, m0, mu, dt, absdt, n2, pf2, tol;
  int max_depth;
};

// Kick of H_B on a particle from the planets (Eq. 2 gradient, K from the pair
// radius max(rct, rc_j)); positions from p (w = mass).
__device__ __forceinline__ void tp_kick_acc(const TpArgs& a, const double4* __restrict__ p,
                                            const double* __restrict__ prc, double x, double y,
                                            double z, double rct, double& ax, double& ay,
                                            double& az) {
  ax = ay = az = 0.0;
  for (int j = 0; j < a.nm; ++j) {
    const double4 pj = p[j];
    const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt_nr(r2);
    const double ir2 = ir * ir;
    double K = 1.0, dK = 0.0;
    if (!a.enc_free) {
      const double rcij = fmax(rct, prc[j]);
      if (r2 < rcij * rcij) changeover(r2 * ir, rcij, K, dK);
    }
    const double s = pj.w * (K * ir2 * ir - dK * ir2);
    ax += s * dx;
    ay += s * dy;
    az += s * dz;
  }
  ax *= a.G;
  ay *= a.G;
  az *= a.G;
}

// Second Sun kick, closing kick, new candidate mask; writes the particle.
// pfin, prc: the planets at the end of the step and their radii.
__device__ __forceinline__ void tp_finish(const TpArgs& a, const double4* __restrict__ pfin,
                                          const double* __restrict__ prc, int64_t k, double x,
                                          double y, double z, double vx, double vy, double vz,
                                          double rct, double P2x, double P2y, double P2z) {
  x += a.h * P2x / a.m0;
  y += a.h * P2y / a.m0;
  z += a.h * P2z / a.m0;
  double ax, ay, az;
  tp_kick_acc(a, pfin, prc, x, y, z, rct, ax, ay, az);
  vx += a.h * ax;
  vy += a.h * ay;
  vz += a.h * az;
  unsigned msk = 0u;
  if (!a.enc_free) {
    for (int j = 0; j < a.nm; ++j) {
      const double4 pj = pfin[j];
      const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
      const double rcij = fmax(rct, prc[j]);
      if (dx * dx + dy * dy + dz * dz < a.pf2 * rcij * rcij) msk |= 1u << j;
    }
  }
  a.x[k] = x;
  a.x[a.ntp + k] = y;
  a.x[2 * a.ntp + k] = z;
  a.v[k] = vx;
  a.v[a.ntp + k] = vy;
  a.v[2 * a.ntp + k] = vz;
  a.mask[k] = msk;
}

__device__ void tp_plan(const TpArgs& a);

// The planets' arrays come as kernel arguments of their own: as noalias
// parameters their wave-uniform loads become scalar loads.  A block past
// the particles' nb blocks (launched with encounters) builds the planets'
// whole-step table instead, beside the particles' work.
__global__ __launch_bounds__(256) void k_tp_main(TpArgs a, const double4* __restrict__ px0,
                                                 const double4* __restrict__ pfin,
                                                 const double4* __restrict__ ppre,
                                                 const double4* __restrict__ vpre,
                                                 const double4* __restrict__ ppost,
                                                 const double4* __restrict__ vpost,
                                                 const double* __restrict__ prc) {
  if ((int64_t)blockIdx.x >= a.nb) {  // the extra block (uniform over the workgroup)
    tp_plan(a);
    return;
  }
  __shared__ unsigned kh[kKepBins];  // this block's drifts by iteration count
  if (threadIdx.x < kKepBins) kh[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  double P1x = 0.0, P1y = 0.0, P1z = 0.0;
  for (int b = 0; b < a.nblk; ++b) {
    P1x += a.partP[4 * b + 0];
    P1y += a.partP[4 * b + 1];
    P1z += a.partP[4 * b + 2];
  }
  const double P2x = a.st->P2[0], P2y = a.st->P2[1], P2z = a.st->P2[2];
  bool listed = false;
  unsigned emask = 0u;
  double xm0 = 0, ym0 = 0, zm0 = 0, vxm = 0, vym = 0, vzm = 0, rct = 0;
  int it = 0;
  double x = 0.0;
  if (k < a.ntp) x = a.x[k];
  if (k < a.ntp && !isnan(x)) {
    double y = a.x[a.ntp + k], z = a.x[2 * a.ntp + k];
    double vx = a.v[k], vy = a.v[a.ntp + k], vz = a.v[2 * a.ntp + k];
    const unsigned cmask = a.mask[k];
    rct = a.n2 * a.absdt * sqrt(vx * vx + vy * vy + vz * vz);
    double ax, ay, az;
    tp_kick_acc(a, px0, prc, x, y, z, rct, ax, ay, az);
    vx += a.h * ax;
    vy += a.h * ay;
    vz += a.h * az;
    x += a.h * P1x / a.m0;
    y += a.h * P1y / a.m0;
    z += a.h * P1z / a.m0;
    xm0 = x;
    ym0 = y;
    zm0 = z;
    vxm = vx;
    vym = vy;
    vzm = vz;
    it = kepler_drift(a.mu, a.dt, x, y, z, vx, vy, vz, a.max_iter);
    if (it < 0) atomicOr(&a.st->flags, F_KEPLER);
    atomicAdd(&kh[min(abs(it), kKepBins - 1)], 1u);
    if (!a.enc_free && cmask) {
      for (int j = 0; j < a.nm; ++j) {
        if (!(cmask & (1u << j))) continue;
        const double4 p0 = ppre[j], q0 = vpre[j], p1 = ppost[j], q1 = vpost[j];
        const double d2 = hermite_dmin2(a.dt, p0.x - xm0, p0.y - ym0, p0.z - zm0,
                                        q0.x - vxm, q0.y - vym, q0.z - vzm,
                                        p1.x - x, p1.y - y, p1.z - z,
                                        q1.x - vx, q1.y - vy, q1.z - vz);
        const double rcij = fmax(rct, prc[j]);
        if (d2 < rcij * rcij) {
          emask |= 1u << j;
          a.enc_d2[(size_t)j * a.ntp + k] = d2;
          a.enc_rc2[(size_t)j * a.ntp + k] = rcij * rcij;
        }
      }
    }
    if (emask) {
      listed = true;
    } else {
      tp_finish(a, pfin, prc, k, x, y, z, vx, vy, vz, rct, P2x, P2y, P2z);
    }
  }
  // block-level compaction of the particles with an encounter into this
  // block's region of the list, and block counters
  __shared__ int s_cnt[4], s_enc[4], s_kit[4];
  const int w = threadIdx.x >> 6;
  const unsigned long long lm = __ballot(listed);
  int nen = listed ? __popc(emask) : 0;
  for (int o = 32; o > 0; o >>= 1) nen += __shfl_xor(nen, o, 64);
  const int itm = wave_max_i(abs(it));
  if (lane == 0) {
    s_cnt[w] = __popcll(lm);
    s_enc[w] = nen;
    s_kit[w] = itm;
  }
  __syncthreads();
  int base = 0;
  for (int q = 0; q < w; ++q) base += s_cnt[q];
  if (threadIdx.x == 0) {
    const int b = blockIdx.x;
    a.blk_cnt[b] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
    const int ne = s_enc[0] + s_enc[1] + s_enc[2] + s_enc[3];
    a.blk_enc[b] = ne;
    a.blk_enc_tot[b] += (unsigned long long)ne;
    a.blk_kit[b] = max(a.blk_kit[b], max(max(s_kit[0], s_kit[1]), max(s_kit[2], s_kit[3])));
  }
  if (threadIdx.x < kKepBins)
    a.khist[(size_t)blockIdx.x * kKepBins + threadIdx.x] += kh[threadIdx.x];
  if (listed) {
    const int64_t pos = (int64_t)blockIdx.x * 256 + base + (int)lanemask_count_tp(lm);
    a.bs_idx[pos] = (int)k;
    a.bs_mask[pos] = emask;
    a.bs_emask[pos] = emask;
    a.bs_rct[pos] = rct;
    a.bs_y[pos] = xm0;
    a.bs_y[a.cap + pos] = ym0;
    a.bs_y[2 * a.cap + pos] = zm0;
    a.bs_y[3 * a.cap + pos] = vxm;
    a.bs_y[4 * a.cap + pos] = vym;
    a.bs_y[5 * a.cap + pos] = vzm;
  }
}

// Exclusive prefix sum of the blocks' list counts (one workgroup of 1024).
__global__ __launch_bounds__(1024) void k_tp_scan(TpArgs a) {
  __shared__ int sh[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (a.nb + 1023) / 1024;
  const int64_t lo = min(a.nb, t * chunk), hi = min(a.nb, lo + chunk);
  int sum = 0;
  for (int64_t b = lo; b < hi; ++b) sum += a.blk_cnt[b];
  sh[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int run = sh[t] - sum;
  for (int64_t b = lo; b < hi; ++b) {
    a.blk_off[b] = run;
    run += a.blk_cnt[b];
  }
  if (t == 1023) a.blk_off[a.nb] = sh[1023];
  if (t == 0) *a.rq_cnt = 0;  // the wave path's queue of this step
}

// List entry of the d-th listed particle: the block whose region holds it
// (largest b with blk_off[b] <= d), then the slot inside the region.
__device__ __forceinline__ int64_t tp_entry(const TpArgs& a, int64_t d) {
  int64_t lo = 0, hi = a.nb;  // blk_off[lo] <= d < blk_off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (a.blk_off[mid] <= d) lo = mid;
    else hi = mid;
  }
  return lo * 256 + (d - a.blk_off[lo]);
}

// One wave per listed particle: its group is the particle (member 0) and the
// planets it encounters in ascending order, started from the pre-drift state.
// rtp: the particle's physical radius; a planet member with a nonzero sum
// of radii gets the collision test.
template <int P>
__device__ __forceinline__ int tp_group(const TpArgs& a, int64_t e, int sz, unsigned em,
                                        const double* mm, const double* mrc, double rtp,
                                        long long* nsub, double y[6], int* cb,
                                        long long* cpos) {
  const int lane = threadIdx.x & 63;
  const int b = par_memb<P>(lane);
  double R2 = -1.0;
  y[0] = 1.0;
  y[1] = y[2] = y[3] = y[4] = y[5] = 0.0;
  if (b == 0) {
#pragma unroll
    for (int q = 0; q < 6; ++q) y[q] = a.bs_y[q * a.cap + e];
  } else if (b < sz) {
    // b-th set bit of em
    unsigned mm2 = em;
    for (int t = 1; t < b; ++t) mm2 &= mm2 - 1u;
    const int j = __ffs(mm2) - 1;
    const double4 p = a.ppre[j], q = a.vpre[j];
    y[0] = p.x;
    y[1] = p.y;
    y[2] = p.z;
    y[3] = q.x;
    y[4] = q.y;
    y[5] = q.z;
    const double R = rtp + a.rad[j];
    if (R > 0.0) R2 = R * R;
  }
  return bs_group<P, true>(sz, y, mm, mrc, a.dt, a.G, a.mu, a.tol, a.max_depth, nsub, R2, cb,
                           cpos);
}

// Removal of listed particle e after a collision with its member cb, at the
// start of the substep that covers [cpos, ...) of the step (units 2^-D).
__device__ void tp_remove(const TpArgs& a, int64_t e, unsigned em, int cb, long long cpos,
                          const double y[6]) {
  const int64_t k = a.bs_idx[e];
  unsigned mm2 = em;
  for (int t = 1; t < cb; ++t) mm2 &= mm2 - 1u;
  const unsigned long long slot = atomicAdd(&a.st->tp_removed, 1ull);
  if ((int64_t)slot < a.ntp) {
    CollRec r;
    r.tp = k;
    r.step = (long long)a.st->nstep - 1;
    r.planet = __ffs(mm2) - 1;
    r.pad = 0;
    r.frac = ldexp((double)cpos, -a.max_depth);
#pragma unroll
    for (int q = 0; q < 6; ++q) r.xv[q] = y[q];
    a.coll[slot] = r;
  }
  const double nan = __builtin_nan("");
  a.x[k] = a.x[a.ntp + k] = a.x[2 * a.ntp + k] = nan;
  a.v[k] = a.v[a.ntp + k] = a.v[2 * a.ntp + k] = nan;
  a.mask[k] = 0u;
}

// ---- the whole-step BS attempt of a particle meeting one planet -------------
// Table per planet j (kPlStride doubles): the planet's positions after each
// midpoint substep of column k (k = 0..7, n_k = 2(k+1) substeps, column k at
// offset 3 k (k+1)), then its extrapolated state T[k][k] (6 per column), then
// its error estimate per column.
constexpr int kPlPos = 3 * 72;
constexpr int kPlDiag = kPlPos;
constexpr int kPlErr = kPlDiag + 48;
constexpr int kPlStride = kPlErr + 8;

// Star-only derivative of a planet's state.
__device__ __forceinline__ void star_acc(double Gm0, double x, double y, double z, double& ax,
                                         double& ay, double& az) {
  const double ir = rsqrt_nr(x * x + y * y + z * z);
  const double fs = -Gm0 * (ir * ir * ir);
  ax = fs * x;
  ay = fs * y;
  az = fs * z;
}

// One thread per (planet, column): the planet's Gragg sequence over the whole
// step from its pre-drift state; then one thread per planet extrapolates.
__device__ void tp_plan(const TpArgs& a) {
  __shared__ double sT0[kTpMaxPlanets * 8][6];
  const int j = threadIdx.x >> 3, k = threadIdx.x & 7;
  if (j < a.nm) {
    const double4 p = a.ppre[j], q = a.vpre[j];
    const double y0[6] = {p.x, p.y, p.z, q.x, q.y, q.z};
    const int n = 2 * (k + 1);
    const double hs = a.dt / n;
    double ym[6], yn[6], d[6];
    star_acc(a.mu, y0[0], y0[1], y0[2], d[3], d[4], d[5]);
    d[0] = y0[3];
    d[1] = y0[4];
    d[2] = y0[5];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ym[c] = y0[c];
      yn[c] = y0[c] + hs * d[c];
    }
    double* pos = a.pl + (size_t)j * kPlStride + 3 * k * (k + 1);
    for (int m = 1; m <= n; ++m) {
      pos[3 * (m - 1) + 0] = yn[0];
      pos[3 * (m - 1) + 1] = yn[1];
      pos[3 * (m - 1) + 2] = yn[2];
      star_acc(a.mu, yn[0], yn[1], yn[2], d[3], d[4], d[5]);
      d[0] = yn[3];
      d[1] = yn[4];
      d[2] = yn[5];
      if (m < n) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double t = ym[c] + 2.0 * hs * d[c];
          ym[c] = yn[c];
          yn[c] = t;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) sT0[threadIdx.x][c] = 0.5 * (ym[c] + yn[c] + hs * d[c]);
  }
  __syncthreads();
  if (threadIdx.x < a.nm) {
    const int jj = threadIdx.x;
    double R[8][6];
    double* tab = a.pl + (size_t)jj * kPlStride;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      double cur[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) cur[c] = sT0[jj * 8 + kk][c];
#pragma unroll
      for (int jn = 1; jn <= kk; ++jn) {
        const double ratio = (double)(2 * (kk + 1)) / (double)(2 * (kk - jn + 1));
        const double den = ratio * ratio - 1.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double old = R[jn - 1][c];
          R[jn - 1][c] = cur[c];
          cur[c] = cur[c] + (cur[c] - old) / den;
        }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        R[kk][c] = cur[c];
        tab[kPlDiag + 6 * kk + c] = cur[c];
      }
      tab[kPlErr + kk] =
          kk == 0 ? 0.0 : fmax(relerr3(R[kk], R[kk - 1]), relerr3(R[kk] + 3, R[kk - 1] + 3));
    }
  }
}

// Particle derivative in its group with planet position (qx, qy, qz).
struct PairK {
  double Gm, rcij, i09, near2;  // near2: rc_ij^2 (1 + 1e-12), 0 when rc_ij = 0
};
__device__ __forceinline__ void tp_pair_acc(double Gm0, const PairK& Q, double x, double y,
                                            double z, double qx, double qy, double qz,
                                            double& ax, double& ay, double& az) {
  const double ir = rsqrt_nr(x * x + y * y + z * z);
  const double fs = -Gm0 * (ir * ir * ir);
  ax = fs * x;
  ay = fs * y;
  az = fs * z;
  const double dx = qx - x, dy = qy - y, dz = qz - z;
  const double q2 = dx * dx + dy * dy + dz * dz;
  // beyond rc_ij the H_A pair term is exactly 0 (K = 1, K' = 0)
  if (q2 < Q.near2) {
    const double iq = rsqrt_nr(q2);
    const double iq2 = iq * iq;
    double K, dK;
    changeover_clamped(q2 * iq, Q.rcij, Q.i09, K, dK);
    const double sc = Q.Gm * ((1.0 - K) * iq2 * iq + dK * iq2);
    ax += sc * dx;
    ay += sc * dy;
    az += sc * dz;
  }
}

// Whole-step BS attempt of the passages that meet one planet, eight lanes per
// passage: lane c integrates column c (n_c = 2 (c + 1) Gragg substeps, the
// planet's positions from its table), the Aitken-Neville tableau is built
// across the eight lanes by row shifts, and the first column k >= 1 whose
// relative change, and the planet's own, are within tolerance is taken.
// Passages that need refinement or meet several planets are queued for the
// wave path (one atomic per wave), which spreads them evenly over its waves.
__global__ __launch_bounds__(256) void k_tp_bs1(TpArgs a) {
  const int64_t nl = a.blk_off[a.nb];
  const double P2x = a.st->P2[0], P2y = a.st->P2[1], P2z = a.st->P2[2];
  unsigned long long nsub = 0;
  const int lane = threadIdx.x & 63;
  const int c = lane & 7;  // column of this lane
  const int g0 = lane & ~7;
  const int nsubs = 2 * (c + 1);
  // Neville weights of the lane's column: 1/((n_c/n_{c-j})^2 - 1), 0 past c
  double wj[8];
#pragma unroll
  for (int j = 1; j < 8; ++j) {
    const int pp = c + 1, qq = c - j + 1;
    wj[j] = j <= c ? (double)(qq * qq) / (double)(pp * pp - qq * qq) : 0.0;
  }
  const int64_t stride = (int64_t)gridDim.x * 256 / 8;
  for (int64_t d = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 8; d < nl; d += stride) {
    const int64_t e = tp_entry(a, d);
    const unsigned em = a.bs_mask[e];
    bool wave = true;  // left to the wave path
    if (__popc(em) == 1) {
      const int j = __ffs(em) - 1;
      const double rct = a.bs_rct[e];
      PairK Q;
      Q.Gm = a.G * a.px0[j].w;
      Q.rcij = fmax(rct, a.rc[j]);
      Q.i09 = Q.rcij > 0.0 ? 1.0 / (0.9 * Q.rcij) : 0.0;
      Q.near2 = Q.rcij > 0.0 ? Q.rcij * Q.rcij * (1.0 + 1e-12) : 0.0;
      const double* tab = a.pl + (size_t)j * kPlStride;
      const double4 pp = a.ppre[j];
      double y0[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) y0[q] = a.bs_y[q * a.cap + e];
      double f0[6];
      tp_pair_acc(a.mu, Q, y0[0], y0[1], y0[2], pp.x, pp.y, pp.z, f0[3], f0[4], f0[5]);
      f0[0] = y0[3];
      f0[1] = y0[4];
      f0[2] = y0[5];
      // Gragg's modified midpoint rule for this lane's column: z_1 = z_0 +
      // hs f(z_0), z_{m+1} = z_{m-1} + 2 hs f(z_m), T0 = (z_{n-1} + z_n +
      // hs f(z_n)) / 2, the points in two buffers used in turn
      const double hs = a.dt / nsubs;
      const double* pos = tab + 3 * c * (c + 1);
      double Z0[6], Z1[6], dd[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        Z0[q] = y0[q];
        Z1[q] = y0[q] + hs * f0[q];
      }
      for (int m = 1; m < 16; m += 2) {
        // odd m: evaluate at z_m (Z1), z_{m+1} into Z0
        if (m <= nsubs) {
          tp_pair_acc(a.mu, Q, Z1[0], Z1[1], Z1[2], pos[3 * (m - 1)], pos[3 * (m - 1) + 1],
                      pos[3 * (m - 1) + 2], dd[3], dd[4], dd[5]);
          dd[0] = Z1[3];
          dd[1] = Z1[4];
          dd[2] = Z1[5];
          if (m < nsubs) {
#pragma unroll
            for (int q = 0; q < 6; ++q) Z0[q] = Z0[q] + 2.0 * hs * dd[q];
          }
        }
        // even m + 1: evaluate at z_{m+1} (Z0), z_{m+2} into Z1
        if (m + 1 <= nsubs) {
          tp_pair_acc(a.mu, Q, Z0[0], Z0[1], Z0[2], pos[3 * m], pos[3 * m + 1], pos[3 * m + 2],
                      dd[3], dd[4], dd[5]);
          dd[0] = Z0[3];
          dd[1] = Z0[4];
          dd[2] = Z0[5];
          if (m + 1 < nsubs) {
#pragma unroll
            for (int q = 0; q < 6; ++q) Z1[q] = Z1[q] + 2.0 * hs * dd[q];
          }
        }
      }
      // n is even: z_n is in Z0 and z_{n-1} in Z1; dd = f(z_n)
      double cur[6], sub[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        cur[q] = 0.5 * (Z1[q] + Z0[q] + hs * dd[q]);
        sub[q] = cur[q];
      }
      // tableau across the columns: after j steps lane c holds T[c][min(j, c)]
#pragma unroll
      for (int jn = 1; jn < 8; ++jn) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          sub[q] = jn == c ? cur[q] : sub[q];  // T[c][c-1]
          const double nb = dpp_d<kDppRowShr1>(cur[q]);
          cur[q] = fma(cur[q] - nb, wj[jn], cur[q]);
        }
      }
      const double err = fmax(fmax(relerr3(cur, sub), relerr3(cur + 3, sub + 3)), tab[kPlErr + c]);
      const unsigned okm = (unsigned)(__ballot(c >= 1 && err <= a.tol) >> g0) & 0xFFu;
      if (okm != 0u) {
        wave = false;
        const int kacc = __ffs(okm) - 1;
        double y1[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) y1[q] = shfl_d(cur[q], g0 + kacc);
        if (c == 0) {
          ++nsub;
          const int64_t ip = a.bs_idx[e];
          const double Rs = a.rad[kTpMaxPlanets + ip] + a.rad[j];
          bool hit = false;
          if (Rs > 0.0) {
            const double4 pv = a.vpre[j];
            const double* q1 = tab + kPlDiag + 6 * kacc;
            const double d2 = hermite_dmin2(a.dt, pp.x - y0[0], pp.y - y0[1], pp.z - y0[2],
                                            pv.x - y0[3], pv.y - y0[4], pv.z - y0[5],
                                            q1[0] - y1[0], q1[1] - y1[1], q1[2] - y1[2],
                                            q1[3] - y1[3], q1[4] - y1[4], q1[5] - y1[5]);
            hit = d2 < Rs * Rs;
          }
          if (hit) {
            tp_remove(a, e, em, 1, 0, y0);
          } else {
            tp_finish(a, a.pfin, a.rc, ip, y1[0], y1[1], y1[2], y1[3], y1[4], y1[5], rct, P2x,
                      P2y, P2z);
          }
          a.bs_mask[e] = 0u;  // done
        }
      }
    }
    // passages left to the wave path: one queue slot each (lane c = 0)
    const bool q0 = wave && c == 0;
    const unsigned long long qm = __ballot(q0);
    if (qm) {
      const int leader = __ffsll((long long)qm) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(a.rq_cnt, __popcll(qm));
      base = __shfl(base, leader, 64);
      if (q0) a.rq[base + (int)lanemask_count_tp(qm)] = e;
    }
  }
  for (int o = 32; o > 0; o >>= 1) nsub += __shfl_xor(nsub, o, 64);
  __shared__ unsigned long long s_sub[4];
  if ((threadIdx.x & 63) == 0) s_sub[threadIdx.x >> 6] = nsub;
  __syncthreads();
  if (threadIdx.x == 0) a.sub[blockIdx.x] += s_sub[0] + s_sub[1] + s_sub[2] + s_sub[3];
}

__global__ __launch_bounds__(64) void k_tp_bs(TpArgs a) {
  __shared__ double mm[kBsPar], mrc[kBsPar];
  const int lane = threadIdx.x;
  const int nq = *a.rq_cnt;
  long long nsub = 0;
  const double P2x = a.st->P2[0], P2y = a.st->P2[1], P2z = a.st->P2[2];
  for (int q = blockIdx.x; q < nq; q += gridDim.x) {
    const int64_t e = a.rq[q];
    const unsigned em = a.bs_mask[e];
    if (em == 0u) continue;  // finished by the whole-step attempt
    const int sz = 1 + __popc(em);
    const double rct = a.bs_rct[e];
    if (sz > kBsPar) {
      if (lane == 0) atomicOr(&a.st->flags, F_GROUP);
      continue;
    }
    __syncthreads();
    if (lane == 0) {
      mm[0] = 0.0;
      mrc[0] = rct;
      unsigned mm2 = em;
      for (int t = 1; t < sz; ++t) {
        const int j = __ffs(mm2) - 1;
        mm2 &= mm2 - 1u;
        mm[t] = a.px0[j].w;
        mrc[t] = a.rc[j];
      }
    }
    __syncthreads();
    double y[6];
    const double rtp = a.rad[kTpMaxPlanets + a.bs_idx[e]];
    int r, cb = 0;
    long long cpos = 0;
    if (sz <= 2)
      r = tp_group<2>(a, e, sz, em, mm, mrc, rtp, &nsub, y, &cb, &cpos);
    else if (sz <= 4)
      r = tp_group<4>(a, e, sz, em, mm, mrc, rtp, &nsub, y, &cb, &cpos);
    else
      r = tp_group<8>(a, e, sz, em, mm, mrc, rtp, &nsub, y, &cb, &cpos);
    if (r < 0 && lane == 0) atomicOr(&a.st->flags, F_BS);
    if (r == 1) {
      if (lane == 0) tp_remove(a, e, em, cb, cpos, y);
    } else if (lane == 0) {
      tp_finish(a, a.pfin, a.rc, a.bs_idx[e], y[0], y[1], y[2], y[3], y[4], y[5], rct, P2x, P2y,
                P2z);
    }
  }
  if (lane == 0 && nsub > 0) a.sub[kTpBs1Grid + blockIdx.x] += (unsigned long long)nsub;
}

// Rows [nm, nm + ntp) of the caller's n x 3 arrays into SoA; heliocentric
// velocities become barycentric with the planets' shift in mom.
__global__ void k_tp_pack(const double* __restrict__ x, const double* __restrict__ v,
                          const double* __restrict__ mom, double* __restrict__ tx,
                          double* __restrict__ tv, int64_t ntp, int nm, int helio,
                          double m0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntp) return;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    const double den = m0 + mom[3];
    sx = mom[0] / den;
    sy = mom[1] / den;
    sz = mom[2] / den;
  }
  const int64_t r = nm + k;
  tx[k] = x[3 * r];
  tx[ntp + k] = x[3 * r + 1];
  tx[2 * ntp + k] = x[3 * r + 2];
  tv[k] = v[3 * r] - sx;
  tv[ntp + k] = v[3 * r + 1] - sy;
  tv[2 * ntp + k] = v[3 * r + 2] - sz;
}

__global__ void k_tp_unpack(const double* __restrict__ tx, const double* __restrict__ tv,
                            const double* __restrict__ mom, double* __restrict__ x,
                            double* __restrict__ v, int64_t ntp, int nm, int helio,
                            double m0) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntp) return;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    sx = mom[0] / m0;
    sy = mom[1] / m0;
    sz = mom[2] / m0;
  }
  const int64_t r = nm + k;
  x[3 * r] = tx[k];
  x[3 * r + 1] = tx[ntp + k];
  x[3 * r + 2] = tx[2 * ntp + k];
  v[3 * r] = tv[k] + sx;
  v[3 * r + 1] = tv[ntp + k] + sy;
  v[3 * r + 2] = tv[2 * ntp + k] + sz;
}

// Candidate masks of the first step: r < pf max(rct, rc_j) at the start.
__global__ void k_tp_prime(TpArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.ntp) return;
  const double x = a.x[k], y = a.x[a.ntp + k], z = a.x[2 * a.ntp + k];
  const double vx = a.v[k], vy = a.v[a.ntp + k], vz = a.v[2 * a.ntp + k];
  const double rct = a.n2 * a.absdt * sqrt(vx * vx + vy * vy + vz * vz);
  unsigned msk = 0u;
  if (!a.enc_free) {
    for (int j = 0; j < a.nm; ++j) {
      const double4 pj = a.pfin[j];
      const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
      const double rcij = fmax(rct, a.rc[j]);
      if (dx * dx + dy * dy + dz * dz < a.pf2 * rcij * rcij) msk |= 1u << j;
    }
  }
  a.mask[k] = msk;
}

// Test-particle rows of the caller's state: each row is finite, or all six
// values are NaN (a removed particle).
__global__ void k_tp_validate(const double* __restrict__ x, const double* __restrict__ v,
                              int64_t ntp, int nm, int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ntp) return;
  const int64_t r = nm + k;
  int fin = 0, nan = 0;
  for (int q = 0; q < 3; ++q) {
    const double a = x[3 * r + q], b = v[3 * r + q];
    fin += isfinite(a) + isfinite(b);
    nan += isnan(a) + isnan(b);
  }
  if (fin != 6 && nan != 6) atomicOr(bad, 1);
}

__global__ void k_tp_radii(const double* __restrict__ r, double* __restrict__ rad, int64_t ntp,
                           int nm, int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kTpMaxPlanets) rad[k] = k < nm ? r[k] : 0.0;
  if (k < ntp) rad[kTpMaxPlanets + k] = r[nm + k];
  if (k < nm + ntp) {
    const double q = r[k];
    if (!(q >= 0.0) || !isfinite(q)) atomicOr(bad, 1);
  }
}

TpArgs tp_args(const MassiveWs& w, const TpWs& t, const StepConsts& c) {
  TpArgs a;
  a.x = t.x;
  a.v = t.v;
  a.mask = t.mask;
  a.px0 = w.xstart;
  a.ppre = w.xpre;
  a.vpre = w.vpre;
  a.ppost = w.xpost;
  a.vpost = w.vpost;
  a.pfin = w.xs;
  a.rc = w.rc_cur;
  a.partP = w.partP;
  a.st = w.st;
  a.bs_idx = t.bs_idx;
  a.bs_mask = t.bs_mask;
  a.bs_emask = t.bs_emask;
  a.enc_d2 = t.enc_d2;
  a.enc_rc2 = t.enc_rc2;
  a.bs_rct = t.bs_rct;
  a.bs_y = t.bs_y;
  a.rad = t.rad;
  a.coll = t.coll;
  a.blk_cnt = t.blk_cnt;
  a.blk_off = t.blk_off;
  a.blk_enc = t.blk_enc;
  a.blk_enc_tot = t.blk_enc_tot;
  a.blk_kit = t.blk_kit;
  a.khist = t.khist;
  a.sub = t.sub;
  a.pl = t.pl;
  a.rq = t.rq;
  a.rq_cnt = t.rq_cnt;
  a.ntp = t.ntp;
  a.cap = t.cap;
  a.nb = t.nb;
  a.nm = w.n;
  a.nblk = w.nblk;
  a.enc_free = c.encounter_free;
  a.max_iter = c.kepler_max_iter;
  a.G = c.G;
  a.h = c.h;
  a.m0 = c.m0;
  a.mu = c.mu;
  a.dt = c.dt;
  a.absdt = fabs(c.dt);
  a.n2 = c.n2;
  a.pf2 = c.pf2;
  a.tol = c.bs_tol;
  a.max_depth = c.bs_max_depth;
  return a;
}

}  // namespace

size_t tp_carve(TpWs& t, int64_t ntp, int nm, void* base) {
  t.ntp = ntp;
  t.nm = nm;
  t.nb = std::max<int64_t>((ntp + 255) / 256, 1);
  t.cap = t.nb * 256;  // one 256-entry region of the list per block
  const size_t n = (size_t)std::max<int64_t>(ntp, 1);
  const size_t nc = (size_t)t.cap, nb = (size_t)t.nb;
  size_t off = 0;
  auto take = [&](size_t sz) -> void* {
    const size_t o = off;
    off += (sz + 255) & ~size_t(255);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  t.x = (double*)take(3 * n * sizeof(double));
  t.v = (double*)take(3 * n * sizeof(double));
  t.mask = (unsigned*)take(n * sizeof(unsigned));
  t.bs_idx = (int*)take(nc * sizeof(int));
  t.bs_mask = (unsigned*)take(nc * sizeof(unsigned));
  t.bs_emask = (unsigned*)take(nc * sizeof(unsigned));
  t.enc_d2 = (double*)take((size_t)nm * n * sizeof(double));
  t.enc_rc2 = (double*)take((size_t)nm * n * sizeof(double));
  t.bs_rct = (double*)take(nc * sizeof(double));
  t.bs_y = (double*)take(6 * nc * sizeof(double));
  t.rad = (double*)take((kTpMaxPlanets + n) * sizeof(double));
  t.coll = (CollRec*)take(n * sizeof(CollRec));
  t.blk_cnt = (int*)take(nb * sizeof(int));
  t.blk_off = (int*)take((nb + 1) * sizeof(int));
  t.blk_enc = (int*)take(nb * sizeof(int));
  // cumulative counters, cleared at init: enc totals, Kepler maxima, substeps
  t.cum = base ? (char*)base + off : nullptr;
  const size_t cum0 = off;
  t.blk_enc_tot = (unsigned long long*)take(nb * sizeof(unsigned long long));
  t.blk_kit = (int*)take(nb * sizeof(int));
  t.khist = (unsigned long long*)take(nb * kKepBins * sizeof(unsigned long long));
  t.sub = (unsigned long long*)take(kTpSubSlots * sizeof(unsigned long long));
  t.cum_bytes = off - cum0;
  t.pl = (double*)take((size_t)kTpMaxPlanets * kPlStride * sizeof(double));
  t.rq = (int64_t*)take(nc * sizeof(int64_t));
  t.rq_cnt = (int*)take(sizeof(int));
  return off;
}

hipError_t tp_read_counters(const TpWs& t, TpCounters* h, hipStream_t s) {
  h->enc = 0;
  h->enc_total = 0;
  h->kit = 0;
  h->sub = 0;
  for (int q = 0; q < kKepBins; ++q) h->khist[q] = 0;
  if (t.ntp <= 0) return hipSuccess;
  std::vector<int> enc(t.nb), kit(t.nb);
  std::vector<unsigned long long> tot(t.nb), sub(kTpSubSlots), kh((size_t)t.nb * kKepBins);
  hipError_t e = hipMemcpyAsync(enc.data(), t.blk_enc, t.nb * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(kit.data(), t.blk_kit, t.nb * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(tot.data(), t.blk_enc_tot, t.nb * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sub.data(), t.sub, kTpSubSlots * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(kh.data(), t.khist, kh.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int64_t b = 0; b < t.nb; ++b) {
    h->enc += enc[b];
    h->enc_total += tot[b];
    h->kit = std::max(h->kit, kit[b]);
  }
  for (int q = 0; q < kTpSubSlots; ++q) h->sub += sub[q];
  for (size_t q = 0; q < kh.size(); ++q) h->khist[q % kKepBins] += kh[q];
  return hipSuccess;
}

// Copies of the list (per block region: its particles and their encounter
// planets) and of the stored minima; no arithmetic.
hipError_t tp_read_encounters(const TpWs& t, std::vector<TpEnc>* out, hipStream_t s) {
  out->clear();
  if (t.ntp <= 0) return hipSuccess;
  std::vector<int> cnt(t.nb), idx(t.cap);
  std::vector<unsigned> em(t.cap);
  std::vector<double> d2((size_t)t.nm * t.ntp), rc2((size_t)t.nm * t.ntp);
  hipError_t e = hipMemcpyAsync(cnt.data(), t.blk_cnt, t.nb * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(idx.data(), t.bs_idx, t.cap * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(em.data(), t.bs_emask, t.cap * sizeof(unsigned), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d2.data(), t.enc_d2, d2.size() * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rc2.data(), t.enc_rc2, rc2.size() * sizeof(double), hipMemcpyDeviceToHost,
                       s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int64_t b = 0; b < t.nb; ++b)
    for (int q = 0; q < cnt[b]; ++q) {
      const int64_t pos = b * 256 + q;
      const long long k = idx[pos];
      for (unsigned m = em[pos]; m; m &= m - 1u) {
        const int j = __builtin_ctz(m);
        const size_t at = (size_t)j * t.ntp + k;
        out->push_back(TpEnc{k, j, d2[at], rc2[at]});
      }
    }
  return hipSuccess;
}

hipError_t tp_validate(const TpWs& t, int nm, const double* x, const double* v, int* dbad,
                       hipStream_t s) {
  if (t.ntp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tp_validate, dim3(ceil_div64(t.ntp, 256)), dim3(256), 0, s, x, v, t.ntp,
                     nm, dbad);
  return hipGetLastError();
}

hipError_t tp_set_radii(const TpWs& t, int nm, const double* r, int* dbad, hipStream_t s) {
  const int64_t n = std::max<int64_t>(t.ntp + nm, kTpMaxPlanets);
  hipLaunchKernelGGL(k_tp_radii, dim3(ceil_div64(n, 256)), dim3(256), 0, s, r, t.rad, t.ntp, nm,
                     dbad);
  return hipGetLastError();
}

hipError_t tp_pack(const MassiveWs& w, const TpWs& t, const StepConsts& c, const double* x,
                   const double* v, int coords_in, hipStream_t s) {
  if (t.ntp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tp_pack, dim3(ceil_div64(t.ntp, 256)), dim3(256), 0, s, x, v, w.red,
                     t.x, t.v, t.ntp, w.n, coords_in == GENGA_HELIO, c.m0);
  return hipGetLastError();
}

hipError_t tp_unpack(const MassiveWs& w, const TpWs& t, const StepConsts& c, double* x,
                     double* v, int coords_out, hipStream_t s) {
  if (t.ntp <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tp_unpack, dim3(ceil_div64(t.ntp, 256)), dim3(256), 0, s, t.x, t.v,
                     w.red, x, v, t.ntp, w.n, coords_out == GENGA_HELIO, c.m0);
  return hipGetLastError();
}

hipError_t tp_prime(const MassiveWs& w, const TpWs& t, const StepConsts& c, hipStream_t s) {
  if (t.ntp <= 0) return hipSuccess;
  TpArgs a = tp_args(w, t, c);
  hipLaunchKernelGGL(k_tp_prime, dim3(ceil_div64(t.ntp, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t tp_step(const MassiveWs& w, const TpWs& t, const StepConsts& c, hipStream_t s) {
  if (t.ntp <= 0) return hipSuccess;
  TpArgs a = tp_args(w, t, c);
  // with encounters, one block more: the planets' whole-step table
  hipLaunchKernelGGL(k_tp_main, dim3((unsigned)(t.nb + (c.encounter_free ? 0 : 1))), dim3(256), 0, s, a,
                     (const double4*)a.px0, (const double4*)a.pfin, (const double4*)a.ppre,
                     (const double4*)a.vpre, (const double4*)a.ppost, (const double4*)a.vpost,
                     (const double*)a.rc);
  if (!c.encounter_free) {
    hipLaunchKernelGGL(k_tp_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_tp_bs1, dim3(kTpBs1Grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_tp_bs, dim3(kTpBsGrid), dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace genga
