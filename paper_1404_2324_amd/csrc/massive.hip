// Main-mode kernels of the hybrid symplectic step (Grimm & Stadel,
// arXiv:1404.2324, Sec. 2.2 step recipe and Sec. 3.2 kernels), for gfx950.
//
// One step is five launches on one stream (captured once into a HIP graph;
// a sixth, the compaction, when bodies can leave):
//   k_open_drift   opening kick: cached non-candidate acceleration + candidate
//                  pairs recomputed with the new radii (KickA/KickB, Sec 3.2.3);
//                  Sun kick tau/2 (Eq. 3) + pre-drift copy + Kepler drift
//                  (Eq. 9) + momentum partials for the second Sun kick
//   k_encounter    Hermite test of every candidate (Eqs. 10-12), ballot
//                  compaction of the confirmed pairs
//   k_group_bs     equivalence classes of the pairs in LDS (App. A), formed
//                  by every workgroup for itself, then Bulirsch-Stoer
//                  integration of H_A per group, one workgroup of four waves
//                  each (speculative halving depths)
//   k_pair_part    closing kick: all pairs and the prechecker, partial sums
//                  per split of the partners
//   k_pair_finish  per body: the splits added, the second Sun kick tau/2,
//                  v += tau/2 a and the next radii
// Between steps the positions live in xs (the closing kick's output); x
// holds them while a step runs.
#include <hip/hip_ext.h>

#include <climits>
#include <cstddef>
#include <mutex>

#include "bs_device.h"
#include "device_math.h"
#include "genga_impl.h"

namespace genga {

namespace {

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

__device__ __forceinline__ unsigned lanemask_count(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Deterministic sum over a block of NT threads; every thread gets the total.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) t += sh[k];
  return t;
}

// Three such sums with one pair of barriers; sh holds 3 NT/64 doubles.
template <int NT>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* sh) {
  constexpr int NW = NT / 64;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[w] = a;
    sh[NW + w] = b;
    sh[2 * NW + w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    a += sh[k];
    b += sh[NW + k];
    c += sh[2 * NW + k];
  }
}

// ---------------------------------------------------------------------------
// The pair kernel: all pairs of H_B (the gradient of Eq. 2, Sec. 3.2.3) with
// the prechecker (Sec. 2.2), as per-split partial sums; a second kernel
// adds the splits of each body in a fixed order and applies the per-body
// epilogue.
// Two shapes (waves per workgroup, splits x padded bodies aimed for), chosen
// by size (measured): below kPairBigN 16 waves and 16384 (2048 bodies: 8
// splits, 4096 waves; the launch floor dominates there), from kPairBigN on 8
// waves and 65536 (16384 bodies: 4 splits, 1024 workgroups of 8 waves,
// 21.1 against 18.6 TFLOP/s with the small-system shape).
constexpr int kPairW = 16;                     // waves per workgroup, small systems
constexpr int kPairTarget = 16384;
constexpr int kPairWBig = 8;                   // waves per workgroup, large systems
constexpr int kPairTargetBig = 65536;
constexpr int kPairBigN = 8192;                // padded bodies from which the large shape runs
constexpr int kPairBlock = 64;                 // i-bodies per workgroup (one per lane)
constexpr int kPairU = 2;                      // partners per prefetched batch
constexpr int kFinThreads = 64;                // threads of the finishing kernel

struct PairArgs {
  const double* __restrict__ rc;      // radii of the step
  int* __restrict__ ccnt;             // candidate table (appended)
  int* __restrict__ ctab;
  double* __restrict__ cr2;
  double* __restrict__ pp;            // partial sums [njs][6][np]: far x y z, near x y z
  double4* __restrict__ xs;           // positions at the end of the step (out)
  double4* __restrict__ vv;
  double4* __restrict__ afar;         // non-candidate acceleration (x G), reused next step
  double* __restrict__ rc_next;
  double* __restrict__ acc_out;
  const double* __restrict__ partP2;  // momentum partials after the drift
  const double* __restrict__ dP;      // momentum change of each BS group
  DevStat* __restrict__ st;
  int n, np, cpb, nblk, njs, jl, encounter_free;  // jl = np / (16 njs) partners per wave
  double G, h, m0, mu, n1, n2, absdt, pf;
};

enum { KICK_CLOSE = 0, KICK_INIT = 1, KICK_ACC = 2 };

// Workgroup (s, b) takes the 64 bodies i = 64 b + lane and the partners of
// split s; each of its 16 waves a contiguous range of L = np / (16 njs)
// partners j (L is even: np is a multiple of 32 njs), the same j for every lane, so the partner data
// (x, y, z, m) comes through the scalar cache into SGPRs, two partners ahead
// of their use: the pair loop issues no vector memory instruction.  The
// bodies are padded to a multiple of 256 with massless bodies at the origin,
// whose terms are exact zeros (a lane's own j and padded pairs at r = 0 are
// excluded by the candidate test below).
// A pair with r^2 < max(thr_i, thr_j), thr = max((pf rc)^2, tiny), is a
// candidate: its K-weighted term is summed apart ("near") and, outside the
// accumulation mode, appended to the body's candidate table; every other
// pair has K = 1 and joins the "far" sum that the next opening kick reuses
// (KickB).  The common test is one compare against the wave's largest
// threshold T (over its 64 bodies and its partner range, from the 64-body
// chunk maxima): below it the term is held out of the far sum by a select,
// and a wave with any such lane takes the exact test for those lanes.  The
// W waves' sums are added in LDS in wave order; the split's sums go to pp.
template <int MODE, int W>
__global__ __launch_bounds__(W * 64) void k_pair_part(PairArgs a,
                                                            const double4* __restrict__ x,
                                                            const double* __restrict__ thr,
                                                            const double* __restrict__ tmx) {
  __shared__ double red[6][W][kPairBlock];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ib = blockIdx.y, sp = blockIdx.x;
  // a context's step: a stopped run appends nothing (its partial sums are
  // written and ignored by the finishing kernel), and rows past the live
  // count are padding (bodies that left); the acceleration form has no
  // status word (st may be null) and takes every body.  The status word is
  // loaded here and first read in the rare candidate branch, so that no
  // wave waits for it before its pair loop.
  int nl = a.n, stopped = 0;
  if (MODE != KICK_ACC) {
    nl = a.st->nlive;
    stopped = a.st->stopped;
  }
  const int i = ib * kPairBlock + lane;
  const int L = a.jl;
  const int j0 = __builtin_amdgcn_readfirstlane((sp * W + wave) * L);
  const double4* xj = x + j0;
  double4 cur[kPairU], nxt[kPairU];
#pragma unroll
  for (int q = 0; q < kPairU; ++q) nxt[q] = xj[q];
  const double4 pi = x[i];
  const double ti = thr[i];
  // T = the largest threshold of the wave's bodies and of the 64-body chunk
  // of partners in use, from the chunk maxima (wave-uniform, through the
  // scalar cache); the next chunk's maximum is loaded a chunk ahead, so that
  // every load of the prologue is issued before the first wait
  const double Ti = tmx[ib];
  const int clast = (j0 + L - 1) >> 6;
  int cn = j0 >> 6;
  double tn = tmx[cn], T = 0.0;
  double fx = 0.0, fy = 0.0, fz = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  // the series constants of m_rinv3 in registers for the whole loop (an
  // empty asm statement hides their values, so that they are not re-made
  // from literals for every pair)
  double c1875 = 1.875, c15 = 1.5;
  asm volatile("" : "+v"(c1875), "+v"(c15));
  int k = 0;
  do {  // L >= 2: no test before the first batch, so that the prologue's loads go out together
    // partner ranges and kPairU-partner batches are aligned so that a batch
    // never straddles two chunks
    if (((j0 + k) >> 6) == cn) {
      T = fmax(Ti, tn);
      ++cn;
      tn = tmx[min(cn, clast)];
    }
#pragma unroll
    for (int q = 0; q < kPairU; ++q) cur[q] = nxt[q];
    if (k + kPairU < L) {
#pragma unroll
      for (int q = 0; q < kPairU; ++q) nxt[q] = xj[k + kPairU + q];
    }
#pragma unroll
    for (int q = 0; q < kPairU; ++q) {
      const double4 pj = cur[q];
      const double dx = pj.x - pi.x, dy = pj.y - pi.y, dz = pj.z - pi.z;
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double s = m_rinv3(pj.w, r2, c1875, c15);
      const bool c = r2 < T;
      const double sf = c ? 0.0 : s;
      fx = fma(sf, dx, fx);
      fy = fma(sf, dy, fy);
      fz = fma(sf, dz, fz);
      if (__builtin_expect(__builtin_amdgcn_ballot_w64(c) != 0ull, 0)) {
        const int j = j0 + k + q;
        const double tj = thr[j];
        // (an empty asm statement keeps the status word's use, and its
        // wait, inside this branch)
        int nlv = nl, stv = stopped;
        asm volatile("" : "+s"(nlv), "+s"(stv));
        if (c) {
          if (!(r2 < ti || r2 < tj)) {
            fx = fma(s, dx, fx);
            fy = fma(s, dy, fy);
            fz = fma(s, dz, fz);
          } else if (i < nlv && j != i && j < nlv) {
            const double ir = rsqrt_nr(r2);
            const double ir2 = ir * ir;
            double K = 1.0, dK = 0.0;
            if (!a.encounter_free) changeover(r2 * ir, fmax(a.rc[i], a.rc[j]), K, dK);
            const double sn = pj.w * (K * ir2 * ir - dK * ir2);
            nx += sn * dx;
            ny += sn * dy;
            nz += sn * dz;
            if (MODE != KICK_ACC && !a.encounter_free && !stv) {
              const int slot = atomicAdd(&a.ccnt[i], 1);
              if (slot < a.cpb) {
                a.ctab[(size_t)i * a.cpb + slot] = j;
                a.cr2[(size_t)i * a.cpb + slot] = r2;
              } else {
                atomicOr(&a.st->flags, F_CAND_OVF);
              }
            }
          }
        }
      }
    }
    k += kPairU;
  } while (k < L);
  red[0][wave][lane] = fx;
  red[1][wave][lane] = fy;
  red[2][wave][lane] = fz;
  red[3][wave][lane] = nx;
  red[4][wave][lane] = ny;
  red[5][wave][lane] = nz;
  __syncthreads();
  if (threadIdx.x < 6 * kPairBlock) {
    const int cpt = threadIdx.x >> 6, q = threadIdx.x & 63;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[cpt][w][q];
    a.pp[((size_t)sp * 6 + cpt) * a.np + ib * kPairBlock + q] = t;
  }
}

// Per body: the splits' partial sums added in split order, then
//   CLOSE  second Sun kick (x += tau/2 P/m0, P from the drift's momentum
//          partials and each BS group's change, added in the same order by
//          every workgroup), v += tau/2 a, next radii (Eq. 6) and the reuse
//          check; the cached far sum; the shifted positions to xs
//   INIT   the far sum and xs = x (the first step's opening kick)
//   ACC    the acceleration out
template <int MODE>
__global__ __launch_bounds__(kFinThreads) void k_pair_finish(PairArgs a,
                                                             const double4* __restrict__ x) {
  const int lane = threadIdx.x;
  const int i = blockIdx.x * kFinThreads + lane;  // < np: pp and x hold np rows
  // Every load that does not depend on the status word goes out before it
  // is read: the status word (the ACC form has none), the momentum partials
  // and the first 64 groups' momentum changes (dP holds more than 64), and
  // the splits' partial sums.
  int stopped = 0, nl = a.n, ng = 0;
  if (MODE != KICK_ACC) {
    stopped = a.st->stopped;
    nl = a.st->nlive;
    ng = a.encounter_free ? 0 : a.st->ngroups;
  }
  double Px = 0.0, Py = 0.0, Pz = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  if (MODE == KICK_CLOSE) {
    if (lane < a.nblk) {
      Px = a.partP2[4 * lane + 0];
      Py = a.partP2[4 * lane + 1];
      Pz = a.partP2[4 * lane + 2];
    }
    for (int b = lane + 64; b < a.nblk; b += 64) {
      Px += a.partP2[4 * b + 0];
      Py += a.partP2[4 * b + 1];
      Pz += a.partP2[4 * b + 2];
    }
    gx = a.dP[4 * lane + 0];
    gy = a.dP[4 * lane + 1];
    gz = a.dP[4 * lane + 2];
  }
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0), vi = p;
  double rci = 0.0;
  if (MODE != KICK_ACC) {
    p = x[i];
    rci = a.rc[i];
  }
  if (MODE == KICK_CLOSE) vi = a.vv[i];
  double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // eight splits' loads in flight at a time, added in split order (past
  // the last split the load repeats it and the value is dropped)
  for (int s0 = 0; s0 < a.njs; s0 += 8) {
    double v[8][6];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const size_t su = (size_t)min(s0 + u, a.njs - 1);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const double t = a.pp[(su * 6 + c) * a.np + i];
        v[u][c] = s0 + u < a.njs ? t : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < 6; ++c) S[c] += v[u][c];
  }
  if (stopped) return;
  if (MODE == KICK_CLOSE) {
    if (lane < ng) {
      Px += gx;
      Py += gy;
      Pz += gz;
    }
    for (int g = lane + 64; g < ng; g += 64) {
      Px += a.dP[4 * g + 0];
      Py += a.dP[4 * g + 1];
      Pz += a.dP[4 * g + 2];
    }
    Px = wave_sum(Px);
    Py = wave_sum(Py);
    Pz = wave_sum(Pz);
    // bodies ejected after BS take their momentum with them (0 otherwise)
    Px -= a.st->Pej[0];
    Py -= a.st->Pej[1];
    Pz -= a.st->Pej[2];
    if (blockIdx.x == 0 && lane == 0) {
      a.st->P2[0] = Px;
      a.st->P2[1] = Py;
      a.st->P2[2] = Pz;
    }
  }
  if (MODE == KICK_INIT && blockIdx.x == 0 && lane == 0) a.st->ctl = 0u;
  if (i >= nl) return;
  const double G = a.G;
  if (MODE == KICK_ACC) {
    a.acc_out[3 * (size_t)i + 0] = G * (S[0] + S[3]);
    a.acc_out[3 * (size_t)i + 1] = G * (S[1] + S[4]);
    a.acc_out[3 * (size_t)i + 2] = G * (S[2] + S[5]);
    return;
  }
  a.afar[i] = make_double4(G * S[0], G * S[1], G * S[2], 0.0);
  if (MODE == KICK_INIT) {
    a.rc_next[i] = rci;
    a.xs[i] = p;
    return;
  }
  p.x += a.h * Px / a.m0;
  p.y += a.h * Py / a.m0;
  p.z += a.h * Pz / a.m0;
  a.xs[i] = p;
  double4 v = vi;
  v.x += a.h * (G * (S[0] + S[3]));
  v.y += a.h * (G * (S[1] + S[4]));
  v.z += a.h * (G * (S[2] + S[5]));
  a.vv[i] = v;
  const double rcn =
      rcrit(p.x, p.y, p.z, v.x, v.y, v.z, p.w, a.mu, a.m0, a.n1, a.n2, a.absdt);
  a.rc_next[i] = rcn;
  if (!a.encounter_free && rcn > a.pf * rci) atomicOr(&a.st->ctl, C_FULLKICK);
}

// Largest threshold of the 64 bodies i0 .. i0 + 63 of a wave (lanes past
// the bodies hold kTiny), written to tmax64[i0 / 64]: the pair kernel's
// common candidate test.
__device__ __forceinline__ void chunk_tmax(double t, int i0, double* tmax64) {
  t = wave_max(t);
  if ((threadIdx.x & 63) == 0) tmax64[i0 >> 6] = t;
}

// ---------------------------------------------------------------------------
struct OpenArgs {
  const double4* __restrict__ xs;  // start positions (with mass): partners are read here
  double4* __restrict__ xm;        // drifted positions out
  double4* __restrict__ xstart;    // snapshot of the start positions (or null)
  double4* __restrict__ vv;
  double4* __restrict__ xpre;
  double4* __restrict__ vpre;
  double4* __restrict__ xpost;     // snapshot after the drift (or null)
  double4* __restrict__ vpost;
  const double4* __restrict__ afar;
  const double* __restrict__ rc_next;
  double* __restrict__ rc_cur;
  double* __restrict__ thr;
  double* __restrict__ tmax64;
  const int* __restrict__ ccnt;
  const int* __restrict__ ctab;
  double* __restrict__ partP;
  double* __restrict__ partP2;
  unsigned long long* __restrict__ khist;
  DevStat* __restrict__ st;
  int n, cpb, encounter_free, max_iter;
  double G, h, pf2, m0, mu, dt;
};

__device__ __forceinline__ void pair_hb(double xi, double yi, double zi,
                                        double rci, const double4 pj,
                                        double rcj, int enc_free, double& ax,
                                        double& ay, double& az) {
  const double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double ir = rsqrt_nr(r2);
  const double ir2 = ir * ir;
  double K = 1.0, dK = 0.0;
  if (!enc_free) changeover(r2 * ir, fmax(rci, rcj), K, dK);
  const double s = pj.w * (K * ir2 * ir - dK * ir2);
  ax += s * dx;
  ay += s * dy;
  az += s * dz;
}

constexpr int kPre = 8;       // partners fetched per batch of loads
constexpr int kRowSort = 32;  // longest candidate row sorted in registers

// Ascending sort of N (a power of two) values in registers: bitonic network.
template <int N>
__device__ __forceinline__ void bitonic_sort(int (&v)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int u = 0; u < N; ++u) {
        const int l = u ^ j;
        if (l > u) {
          const int lo = min(v[u], v[l]), hi = max(v[u], v[l]);
          const bool up = (u & k) == 0;
          v[u] = up ? lo : hi;
          v[l] = up ? hi : lo;
        }
      }
}

// Pair terms of the sorted partners jj[c0 .. min(c0 + B, cnt) - 1] of body i,
// in that order; all B partner loads are issued before the first use.
template <int B, int N>
__device__ __forceinline__ void sum_partners(const int (&jj)[N], int c0, int cnt, int i,
                                             const double4& p, double rci, const OpenArgs& a,
                                             double& cx, double& cy, double& cz) {
  double4 pj[B];
  double rj[B];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int jl = c0 + u < cnt ? jj[c0 + u] : i;  // padded slots read a valid index
    pj[u] = a.xs[jl];
    rj[u] = a.rc_next[jl];
  }
#pragma unroll
  for (int u = 0; u < B; ++u)
    if (c0 + u < cnt) pair_hb(p.x, p.y, p.z, rci, pj[u], rj[u], a.encounter_free, cx, cy, cz);
}

// Opening kick (KickA/KickB, Sec. 3.2.3), first Sun kick tau/2 (H_C flow,
// Eq. 3), pre-drift copy and Kepler drift (Eq. 9) in one pass per body.
// Kick: the closing kick's non-candidate sum is reused; candidate pairs are
// recomputed with this step's radii in ascending partner order, partners
// read from the start positions xs (xm receives the drifted positions).
// When some radius grew beyond pf times the radius that formed the
// candidate table the reuse is not exact and the full pair sum is taken.
// Sun kick: the momentum P = sum m v is the one the previous step's second
// Sun kick used (or that of the initial state); the kicks in between change
// it by tau/2 sum m a = 0 (pair terms cancel), so it equals the momentum
// after this opening kick up to rounding.  Also installs the step's radii
// and thresholds, leaves per-block momentum partials after the kick and
// after the drift, and resets the step's encounter counters.
__global__ __launch_bounds__(kOpenBlock) void k_open_drift(OpenArgs a) {
  __shared__ double sh[3 * (kOpenBlock / 64)];
  __shared__ unsigned kh[kKepBins];  // this block's drifts by iteration count
  double tloc = kTiny;               // the lane's candidate threshold
  const int i = blockIdx.x * kOpenBlock + threadIdx.x;  // < np: every per-body array has np rows
  // Every load that does not depend on the status word is issued before the
  // word is read: the body's state, cached far sum and radius, its row count
  // and the first kPre entries of its candidate row (entries past the count
  // are read and dropped), this block's Kepler histogram row, and the
  // running iteration maximum.
  const double4 p0 = a.xs[i];
  const double rc0 = a.rc_next[i];
  const double4 af0 = a.afar[i];
  const double4 v0 = a.vv[i];
  const int cnt0 = a.ccnt[i];
  const int* row = a.ctab + (size_t)i * a.cpb;
  int r8[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) r8[u] = u < a.cpb ? row[u] : INT_MAX;
  const unsigned long long kh0 =
      threadIdx.x < kKepBins ? a.khist[(size_t)blockIdx.x * kKepBins + threadIdx.x] : 0ull;
  const int itmax0 = a.st->kep_itmax;
  if (threadIdx.x < kKepBins) kh[threadIdx.x] = 0u;
  __syncthreads();
  if (a.st->flags & F_NMIN) {
    // fewer than nmin bodies left after the last step: the run has stopped
    if (blockIdx.x == 0 && threadIdx.x == 0) a.st->stopped = 1;
    return;
  }
  const bool iv = i < a.st->nlive;
  const bool full = (__builtin_amdgcn_readfirstlane(a.st->ctl) & C_FULLKICK) != 0;
  const double Ps = a.h / a.m0;
  const double sx = Ps * a.st->P2[0], sy = Ps * a.st->P2[1], sz = Ps * a.st->P2[2];
  double m = 0.0, kx = 0.0, ky = 0.0, kz = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
  int it = 0;
  if (iv) {
    const double4 p = p0;
    const double rci = rc0;
    if (a.xstart) a.xstart[i] = p;
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (full) {
      for (int j = 0; j < a.n; ++j)
        if (j != i) pair_hb(p.x, p.y, p.z, rci, a.xs[j], a.rc_next[j], a.encounter_free, ax, ay, az);
      ax *= a.G;
      ay *= a.G;
      az *= a.G;
    } else {
      const double4 af = af0;
      const int cnt = min(cnt0, a.cpb);
      double cx = 0.0, cy = 0.0, cz = 0.0;
      // Partners are summed in ascending order (deterministic).  Rows of up
      // to 8 (nearly all), 16 or kRowSort partners are sorted by a bitonic
      // network of that width in registers; partner data is then fetched 8
      // at a time with independent loads.  Longer rows fall back to an
      // ordered scan.
      if (cnt <= kPre) {
        int jj[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) jj[u] = u < cnt ? r8[u] : INT_MAX;
        bitonic_sort(jj);
        sum_partners<kPre>(jj, 0, cnt, i, p, rci, a, cx, cy, cz);
      } else if (cnt <= 2 * kPre) {
        int jj[2 * kPre];
#pragma unroll
        for (int u = 0; u < 2 * kPre; ++u) jj[u] = u < cnt ? row[u] : INT_MAX;
        bitonic_sort(jj);
        sum_partners<kPre>(jj, 0, cnt, i, p, rci, a, cx, cy, cz);
        sum_partners<kPre>(jj, kPre, cnt, i, p, rci, a, cx, cy, cz);
      } else if (cnt <= kRowSort) {
        int jj[kRowSort];
#pragma unroll
        for (int u = 0; u < kRowSort; ++u) jj[u] = u < cnt ? row[u] : INT_MAX;
        bitonic_sort(jj);
#pragma unroll
        for (int c0 = 0; c0 < kRowSort; c0 += kPre) {
          if (c0 >= cnt) break;
          sum_partners<kPre>(jj, c0, cnt, i, p, rci, a, cx, cy, cz);
        }
      } else {
        int prev = -1;
        for (int t = 0; t < cnt; ++t) {
          int jm = INT_MAX;
          for (int u = 0; u < cnt; ++u) {
            const int j = row[u];
            jm = (j > prev && j < jm) ? j : jm;
          }
          if (jm == INT_MAX) break;
          prev = jm;
          pair_hb(p.x, p.y, p.z, rci, a.xs[jm], a.rc_next[jm], a.encounter_free, cx, cy, cz);
        }
      }
      ax = af.x + a.G * cx;
      ay = af.y + a.G * cy;
      az = af.z + a.G * cz;
    }
    double4 v = v0;
    v.x += a.h * ax;
    v.y += a.h * ay;
    v.z += a.h * az;
    a.rc_cur[i] = rci;
    tloc = a.encounter_free ? kTiny : fmax(a.pf2 * rci * rci, kTiny);
    a.thr[i] = tloc;
    m = p.w;
    kx = v.x;
    ky = v.y;
    kz = v.z;
    double x = p.x + sx, y = p.y + sy, z = p.z + sz;
    a.xpre[i] = make_double4(x, y, z, 0.0);
    a.vpre[i] = make_double4(v.x, v.y, v.z, 0.0);
    dx = v.x;
    dy = v.y;
    dz = v.z;
    it = kepler_drift(a.mu, a.dt, x, y, z, dx, dy, dz, a.max_iter);
    if (it < 0) atomicOr(&a.st->flags, F_KEPLER);
    atomicAdd(&kh[min(abs(it), kKepBins - 1)], 1u);
    a.xm[i] = make_double4(x, y, z, p.w);
    a.vv[i] = make_double4(dx, dy, dz, 0.0);
    if (a.xpost) {
      a.xpost[i] = make_double4(x, y, z, p.w);
      a.vpost[i] = make_double4(dx, dy, dz, 0.0);
    }
  }
  // the running maximum rarely grows: read it first, so that waves do not
  // queue on one address every step
  const int itm = wave_max_i(abs(it));
  if ((threadIdx.x & 63) == 0 && itm > itmax0) atomicMax(&a.st->kep_itmax, itm);
  double Px = m * kx, Py = m * ky, Pz = m * kz;
  block_sum3<kOpenBlock>(Px, Py, Pz, sh);
  double Qx = m * dx, Qy = m * dy, Qz = m * dz;
  block_sum3<kOpenBlock>(Qx, Qy, Qz, sh);  // its barriers also order kh
  if (threadIdx.x < kKepBins)
    a.khist[(size_t)blockIdx.x * kKepBins + threadIdx.x] = kh0 + kh[threadIdx.x];
  chunk_tmax(tloc, i & ~63, a.tmax64);
  if (threadIdx.x == 0) {
    a.partP[4 * blockIdx.x + 0] = Px;
    a.partP[4 * blockIdx.x + 1] = Py;
    a.partP[4 * blockIdx.x + 2] = Pz;
    a.partP2[4 * blockIdx.x + 0] = Qx;
    a.partP2[4 * blockIdx.x + 1] = Qy;
    a.partP2[4 * blockIdx.x + 2] = Qz;
    if (blockIdx.x == 0) {
      if (full) a.st->fullkicks += 1ull;
      a.st->nenc = 0;
      a.st->ncand = 0;
      a.st->ngroups = 0;
      a.st->maxg = 0;
      a.st->nstep += 1ull;
    }
  }
}

// ---------------------------------------------------------------------------
struct EncArgs {
  const double4* __restrict__ xm;
  const double4* __restrict__ vv;
  const double4* __restrict__ xpre;
  const double4* __restrict__ vpre;
  const double* __restrict__ rc;
  int* __restrict__ ccnt;
  const int* __restrict__ ctab;
  int2* __restrict__ encij;
  double* __restrict__ encd2;
  double* __restrict__ encrc2;
  int* __restrict__ goff;
  int* __restrict__ gmem;
  DevStat* __restrict__ st;
  int n, cpb, enc_cap;
  double dt;
};

constexpr int kEncThreads = 1024;

// Exclusive scan over a block of NT threads; returns the prefix and puts the
// total in *total.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* shw, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  __syncthreads();
  if (lane == 63) shw[w] = incl;
  __syncthreads();
  int base = 0, tot = 0;
  for (int k = 0; k < NT / 64; ++k) {
    if (k < w) base += shw[k];
    tot += shw[k];
  }
  *total = tot;
  return base + incl - v;
}

// Encounter search (Sec. 3.2.4): one lane per candidate slot (body i, slot
// k) over all workgroups, so the candidates' loads overlap across the chip.
// The Hermite minimum of Eqs. (10)-(12) is taken for pairs i < j; confirmed
// pairs are appended with a ballot compaction (one atomic per wave that has
// any; the candidate count is taken by the grouping kernel instead, since
// an atomic on one address from every wave serialises them).
__global__ __launch_bounds__(kVecBlock) void k_encounter(EncArgs a) {
  if (a.st->flags & F_NMIN) return;  // the run stopped below nmin bodies
  const int t = blockIdx.x * kVecBlock + threadIdx.x;
  const int i = t / a.cpb, k = t - i * a.cpb;
  const int lane = threadIdx.x & 63;
  bool enc = false;
  int j = -1;
  double d2 = 0.0, rc2 = 0.0;
  if (i < a.n && k < min(a.ccnt[i], a.cpb)) {
    j = a.ctab[(size_t)i * a.cpb + k];
    if (j > i) {
      const double4 xi0 = a.xpre[i], xj0 = a.xpre[j], vi0 = a.vpre[i], vj0 = a.vpre[j];
      const double4 xi1 = a.xm[i], xj1 = a.xm[j], vi1 = a.vv[i], vj1 = a.vv[j];
      d2 = hermite_dmin2(a.dt, xj0.x - xi0.x, xj0.y - xi0.y, xj0.z - xi0.z,
                         vj0.x - vi0.x, vj0.y - vi0.y, vj0.z - vi0.z,
                         xj1.x - xi1.x, xj1.y - xi1.y, xj1.z - xi1.z,
                         vj1.x - vi1.x, vj1.y - vi1.y, vj1.z - vi1.z);
      const double rcij = fmax(a.rc[i], a.rc[j]);
      rc2 = rcij * rcij;
      enc = d2 < rc2;
    }
  }
  const unsigned long long msk = __ballot(enc);
  int b0 = 0;
  if (lane == 0 && msk) b0 = atomicAdd(&a.st->nenc, __popcll(msk));
  b0 = __shfl(b0, 0, 64);
  if (enc) {
    const int pos = b0 + (int)lanemask_count(msk);
    if (pos < a.enc_cap) {
      a.encij[pos] = make_int2(i, j);
      a.encd2[pos] = d2;
      a.encrc2[pos] = rc2;
    }
  }
}

// Encounter search over every pair i < j (the composed steps, Sec. 2.3: no
// prechecker).  Workgroup (ti, tj), tj >= ti, takes i in tile ti and j in
// tile tj (64 bodies each); the j tile's states before and after the drift
// and radii sit in LDS; lane l serves i = 64 ti + l over the 16 partners of
// its quarter, and confirmed pairs are appended as in k_encounter.
constexpr int kEncTile = 64;
__global__ __launch_bounds__(256) void k_encounter_all(EncArgs a) {
  __shared__ double sj[13][kEncTile];
  const int ti = blockIdx.x, tj = blockIdx.y;
  if (tj < ti) return;  // upper triangle of tiles (uniform over the workgroup)
  const int tid = threadIdx.x, lane = tid & 63, q = tid >> 6;
  if (tid < kEncTile) {
    const int j = tj * kEncTile + tid;
    double4 p0 = make_double4(0, 0, 0, 0), v0 = p0, p1 = p0, v1 = p0;
    double rc = 0.0;
    if (j < a.n) {
      p0 = a.xpre[j];
      v0 = a.vpre[j];
      p1 = a.xm[j];
      v1 = a.vv[j];
      rc = a.rc[j];
    }
    sj[0][tid] = p0.x;
    sj[1][tid] = p0.y;
    sj[2][tid] = p0.z;
    sj[3][tid] = v0.x;
    sj[4][tid] = v0.y;
    sj[5][tid] = v0.z;
    sj[6][tid] = p1.x;
    sj[7][tid] = p1.y;
    sj[8][tid] = p1.z;
    sj[9][tid] = v1.x;
    sj[10][tid] = v1.y;
    sj[11][tid] = v1.z;
    sj[12][tid] = rc;
  }
  __syncthreads();
  const int i = ti * kEncTile + lane;
  const bool iv = i < a.n;
  double4 xi0 = make_double4(0, 0, 0, 0), vi0 = xi0, xi1 = xi0, vi1 = xi0;
  double rci = 0.0;
  if (iv) {
    xi0 = a.xpre[i];
    vi0 = a.vpre[i];
    xi1 = a.xm[i];
    vi1 = a.vv[i];
    rci = a.rc[i];
  }
  for (int t = 0; t < kEncTile / 4; ++t) {
    const int k = q * (kEncTile / 4) + t;
    const int j = tj * kEncTile + k;
    bool enc = false;
    double d2 = 0.0, rc2 = 0.0;
    if (iv && j < a.n && j > i) {
      d2 = hermite_dmin2(a.dt, sj[0][k] - xi0.x, sj[1][k] - xi0.y, sj[2][k] - xi0.z,
                         sj[3][k] - vi0.x, sj[4][k] - vi0.y, sj[5][k] - vi0.z,
                         sj[6][k] - xi1.x, sj[7][k] - xi1.y, sj[8][k] - xi1.z,
                         sj[9][k] - vi1.x, sj[10][k] - vi1.y, sj[11][k] - vi1.z);
      const double rcij = fmax(rci, sj[12][k]);
      rc2 = rcij * rcij;
      enc = d2 < rc2;
    }
    const unsigned long long msk = __ballot(enc);
    if (msk) {
      int b0 = 0;
      if (lane == 0) b0 = atomicAdd(&a.st->nenc, __popcll(msk));
      b0 = __shfl(b0, 0, 64);
      if (enc) {
        const int pos = b0 + (int)lanemask_count(msk);
        if (pos < a.enc_cap) {
          a.encij[pos] = make_int2(i, j);
          a.encd2[pos] = d2;
          a.encrc2[pos] = rc2;
        }
      }
    }
  }
}

// Equivalence classes of the encounter pairs (App. A), one workgroup: LINK
// starts as the identity on the pairs' bodies, every pair lowers both ends
// to the smaller link (LDS atomic min), links are shortened by LINK[i] =
// LINK[LINK[i]], and both sweeps repeat until nothing changes.  Groups are
// numbered by their smallest member (the rank of each component's root
// among the roots); offsets and members go to global memory for the BS
// kernel (and, with gm, to LDS).  Every loop of the grouping runs over the
// pairs or their ends, not over the bodies: a step has tens of pairs among
// thousands of bodies.  The writing workgroup also clears the candidate
// table for the closing kick (a loop over the bodies), counts its pairs and
// sets the step's group statistics.
// The first kEncLds pairs are held in LDS; pairs beyond (many-pair regimes,
// up to the list capacity) are read from the encounter list in place, so
// the workgroup's LINK array, not the pair count, bounds the grouping.
template <int NT>
struct GroupLds {
  int link[kGroupMaxN];
  int first[kGroupMaxN];  // the first end (2 e or 2 e + 1) naming each body
  int gid[kGroupMaxN];    // group of each root
  int2 pr[kEncLds];
  int gsz[kGroupMaxN / 2 + 1];
  int gof[kGroupMaxN / 2 + 1];  // group offsets, gof[ng] = the member count
  int roots[kGroupMaxN / 2];
  int nroot;
  int shw[NT / 64];
  int chg[2];
};

// The grouping of ne_all encounter pairs by one workgroup of NT threads;
// returns the number of groups.  gm (LDS, or null): the members by group at
// the offsets gof.  writer: this workgroup writes the global results.  pf
// (or null): the list's entry tid, already loaded by the caller.
template <int NT>
__device__ __forceinline__ int group_phase(const EncArgs& a, int ne_all, GroupLds<NT>& L,
                                           int* gm, bool writer,
                                           const int2* pf = nullptr) {
  int* link = L.link;
  int* first = L.first;
  int* gid = L.gid;
  int2* pr = L.pr;
  int* gsz = L.gsz;
  int* gof = L.gof;
  int* shw = L.shw;
  int* chg = L.chg;
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = a.n;
  const int ne = min(ne_all, a.enc_cap);
  const int nl = min(ne, kEncLds);  // pairs held in LDS
  auto pair_at = [&](int e) { return e < nl ? pr[e] : a.encij[e]; };
  auto end_at = [&](int t) {  // end t of the pairs: pair t / 2, first or second body
    const int2 q = pair_at(t >> 1);
    return (t & 1) ? q.y : q.x;
  };
  // the opening kick has read the reuse flag; this step's closing kick sets
  // it again for the next one
  if (writer && tid == 0) a.st->ctl = 0u;
  if (tid == 0) {
    L.nroot = 0;
    chg[0] = chg[1] = 0;
  }
  for (int e = tid; e < nl; e += NT) pr[e] = (pf && e == tid) ? *pf : a.encij[e];
  __syncthreads();
  // candidate pairs i < j: every pair sits in both rows (the test is
  // symmetric), so half the sum of the row lengths
  int rows = 0;
  if (writer)
    for (int i = tid; i < n; i += NT) {
      rows += min(a.ccnt[i], a.cpb);
      a.ccnt[i] = 0;
    }
  for (int t = tid; t < 2 * ne; t += NT) {
    const int i = end_at(t);
    link[i] = i;
    first[i] = INT_MAX;
  }
  // equivalence classes; the change flag of sweep k is chg[k & 1], the
  // other one cleared for the next sweep once every thread is past the
  // barrier before which it was last read.  The first sweep also notes each
  // body's first end.
  __syncthreads();
  for (int it = 0;; ++it) {
    bool ch = false;
    for (int e = tid; e < ne; e += NT) {
      const int2 q = pair_at(e);
      const int p1 = q.x, p2 = q.y;
      const int l1 = link[p1], l2 = link[p2];
      if (l1 != l2) {
        atomicMin(&link[p1], l2);
        atomicMin(&link[p2], l1);
        ch = true;
      }
    }
    __syncthreads();
    // pointer jumping over the pairs' ends (links only ever name such bodies)
    for (int t = tid; t < 2 * ne; t += NT) {
      const int i = end_at(t);
      if (it == 0) atomicMin(&first[i], t);
      const int l = link[i];
      const int ll = link[l];
      if (ll < l) {
        atomicMin(&link[i], ll);
        ch = true;
      }
    }
    if (ch) chg[it & 1] = 1;
    if (tid == 0) chg[(it & 1) ^ 1] = 0;
    __syncthreads();
    if (!chg[it & 1]) break;
  }
  // each body once (at its first end), each root once
  for (int t = tid; t < 2 * ne; t += NT) {
    const int i = end_at(t);
    if (first[i] == t && link[i] == i) L.roots[atomicAdd(&L.nroot, 1)] = i;
  }
  __syncthreads();
  const int ng = L.nroot;
  // group ids in order of the smallest member: the rank among the roots
  for (int r = tid; r < ng; r += NT) {
    const int ri = L.roots[r];
    int rank = 0;
    for (int u = 0; u < ng; ++u) rank += L.roots[u] < ri ? 1 : 0;
    gid[ri] = rank;
  }
  for (int g = tid; g <= ng; g += NT) gsz[g] = 0;
  __syncthreads();
  for (int t = tid; t < 2 * ne; t += NT) {
    const int i = end_at(t);
    if (first[i] == t) atomicAdd(&gsz[gid[link[i]]], 1);
  }
  __syncthreads();
  // offsets: exclusive scan of the sizes
  constexpr int GPER = (kGroupMaxN / 2 + NT - 1) / NT;
  int loc = 0, mx = 0;
  for (int k = 0; k < GPER; ++k) {
    const int g = tid * GPER + k;
    if (g < ng) {
      loc += gsz[g];
      mx = max(mx, gsz[g]);
    }
  }
  int tot = 0;
  int o2 = block_excl_scan<NT>(loc, shw, &tot);
  for (int k = 0; k < GPER; ++k) {
    const int g = tid * GPER + k;
    if (g < ng) {
      gof[g] = o2;
      if (writer) a.goff[g] = o2;
      o2 += gsz[g];
    }
  }
  if (tid == 0) {
    gof[ng] = tot;
    if (writer) a.goff[ng] = tot;
  }
  int nrow = 0;
  if (writer) (void)block_excl_scan<NT>(rows, shw, &nrow);  // writer: the same for every thread
  mx = wave_max_i(mx);
  __syncthreads();
  if (lane == 0) shw[tid >> 6] = mx;
  for (int g = tid; g < ng; g += NT) gsz[g] = 0;
  __syncthreads();
  if (writer && tid == 0) {
    int m2 = 0;
    for (int k = 0; k < NT / 64; ++k) m2 = max(m2, shw[k]);
    a.st->maxg = m2;
    a.st->ngroups = ng;
    a.st->ncand = nrow / 2;
    a.st->enc_total += (unsigned long long)ne_all;
    if (ne_all > a.enc_cap) atomicOr(&a.st->flags, F_ENC_OVF);
  }
  for (int t = tid; t < 2 * ne; t += NT) {
    const int i = end_at(t);
    if (first[i] == t) {
      const int g = gid[link[i]];
      const int pos = gof[g] + atomicAdd(&gsz[g], 1);
      if (writer) a.gmem[pos] = i;
      if (gm) gm[pos] = i;
    }
  }
  __syncthreads();  // gof and gm for every thread
  return ng;
}

__global__ __launch_bounds__(kEncThreads) void k_group(EncArgs a) {
  __shared__ GroupLds<kEncThreads> L;
  if (a.st->flags & F_NMIN) return;  // the run stopped below nmin bodies
  (void)group_phase<kEncThreads>(a, a.st->nenc, L, nullptr, true);
}


// ---------------------------------------------------------------------------
struct BsArgs {
  double4* __restrict__ xm;
  double4* __restrict__ vv;
  double* __restrict__ dP;
  const double4* __restrict__ xpre;
  const double4* __restrict__ vpre;
  const double* __restrict__ rc;
  const int* __restrict__ goff;
  const int* __restrict__ gmem;
  double* __restrict__ big;    // per-body records of groups over 64 members
  double4* __restrict__ bpos;  // their positions and masses at a Gragg point
  int* __restrict__ bmem;      // their members, sorted, at the group's offset
  double* __restrict__ rc_w;   // this step's radii (a merged body keeps the larger)
  double* __restrict__ rad;    // physical radii (collisions)
  double4* __restrict__ sp;    // spins
  const int* __restrict__ ids; // original rows
  int* __restrict__ dead;      // absorbed bodies of this step
  genga_event* __restrict__ ev;
  DevStat* __restrict__ st;
  double G, Gm0, dt, tol;
  int max_depth, coll, ev_cap;
};

// The BS kernels (k_group_bs, and k_bs for the composed steps) run kBsWaves
// waves per workgroup.  Groups of up to kBsPar members
// without collisions take all of them (speculative depths spread over the
// waves); every other group is integrated by wave 0 alone while the others
// wait at the group's closing barrier.  The lanes of that one wave order
// their LDS and global accesses with wsync: the release and acquire fences
// of a workgroup barrier around a wave barrier, without the workgroup-wide
// s_barrier the waiting waves would have to join.
constexpr int kBsWaves = 4;
__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---- groups of more than 64 members ------------------------------------------
// One wave integrates the group with the BS scheme of the smaller paths (the
// same column sequence, Aitken-Neville tableau, error norm and halving), each
// lane taking the members lane, lane + 64, ...  The state of member id lives
// in the record big[id][kBigRec] (groups are disjoint, so records are too):
// substep start y0, the Gragg points z_{s-1} and z_s, the tableau R[8][6];
// the positions of the current Gragg point are published in bpos[id] for the
// pair sums, between barriers (a one-wave workgroup: the barrier orders the
// lanes' global stores and loads).  Members are sorted ascending, so every
// sum runs in a fixed order.  The cost grows as sz^2 per force evaluation:
// a fallback for rare large groups (the paper steers those from the CPU,
// Sec. 3.2.6), not a fast path.
constexpr int kBigRec = 66;  // y0[6], zp[6], zc[6], R[8][6]
constexpr int kBigY0 = 0, kBigZp = 6, kBigZc = 12, kBigR = 18;

// dv/dt of H_A for member m at (x, y, z): the fixed star and every other
// member's (1-K)-weighted pair term in member order (the formula of
// ha_accel).
__device__ __forceinline__ void ha_accel_big(const BsArgs& a, const int* mem, int sz, int m,
                                             double x, double y, double z, double rc,
                                             double& ax, double& ay, double& az) {
  const double r2 = x * x + y * y + z * z;
  const double ir = rsqrt_nr(r2);
  const double fs = -a.Gm0 * (ir * ir * ir);
  ax = fs * x;
  ay = fs * y;
  az = fs * z;
  for (int q = 0; q < sz; ++q) {
    const int jd = mem[q];
    const double4 pj = a.bpos[jd];
    const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
    const double q2 = dx * dx + dy * dy + dz * dz;
    const double rij = fmax(rc, a.rc[jd]);
    if (q != m && q2 < rij * rij * (1.0 + 1e-12)) {
      const double iq = rsqrt_nr(q2);
      const double iq2 = iq * iq;
      double K, dK;
      changeover(q2 * iq, rij, K, dK);
      const double sc = a.G * pj.w * ((1.0 - K) * iq2 * iq + dK * iq2);
      ax += sc * dx;
      ay += sc * dy;
      az += sc * dz;
    }
  }
}

// Positions of the Gragg point held at record offset off published to bpos.
__device__ __forceinline__ void big_publish(const BsArgs& a, const int* mem, int sz, int off) {
  for (int m = threadIdx.x; m < sz; m += 64) {
    const int id = mem[m];
    const double* r = a.big + (size_t)id * kBigRec + off;
    a.bpos[id] = make_double4(r[0], r[1], r[2], a.xm[id].w);
  }
  wsync();
}

// One attempt over H (columns n_k = 2k, k = 1..8, accepted at the first
// column k >= 2 within tol); on success y0 of every member becomes the
// accepted state.  Returns whether it was accepted (wave-uniform).
__device__ bool big_attempt(const BsArgs& a, const int* mem, int sz, double H) {
  for (int k = 0; k < kBsCols; ++k) {
    const int nk = 2 * (k + 1);
    const double hs = H / nk;
    // z_0 = y0, z_1 = z_0 + hs f(z_0)
    for (int m = threadIdx.x; m < sz; m += 64) {
      double* r = a.big + (size_t)mem[m] * kBigRec;
#pragma unroll
      for (int c = 0; c < 6; ++c) r[kBigZp + c] = r[kBigY0 + c];
    }
    big_publish(a, mem, sz, kBigY0);
    for (int m = threadIdx.x; m < sz; m += 64) {
      const int id = mem[m];
      double* r = a.big + (size_t)id * kBigRec;
      double d[6];
      d[0] = r[kBigZp + 3];
      d[1] = r[kBigZp + 4];
      d[2] = r[kBigZp + 5];
      ha_accel_big(a, mem, sz, m, r[kBigZp], r[kBigZp + 1], r[kBigZp + 2], a.rc[id], d[3], d[4], d[5]);
#pragma unroll
      for (int c = 0; c < 6; ++c) r[kBigZc + c] = r[kBigZp + c] + hs * d[c];
    }
    wsync();
    big_publish(a, mem, sz, kBigZc);
    // z_{s+1} = z_{s-1} + 2 hs f(z_s), s = 1 .. nk - 1
    for (int st = 1; st < nk; ++st) {
      for (int m = threadIdx.x; m < sz; m += 64) {
        const int id = mem[m];
        double* r = a.big + (size_t)id * kBigRec;
        double d[6];
        d[0] = r[kBigZc + 3];
        d[1] = r[kBigZc + 4];
        d[2] = r[kBigZc + 5];
        ha_accel_big(a, mem, sz, m, r[kBigZc], r[kBigZc + 1], r[kBigZc + 2], a.rc[id], d[3], d[4],
                     d[5]);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double t = r[kBigZp + c] + 2.0 * hs * d[c];
          r[kBigZp + c] = r[kBigZc + c];
          r[kBigZc + c] = t;
        }
      }
      wsync();
      big_publish(a, mem, sz, kBigZc);
    }
    // T_k0 = (z_{n-1} + z_n + hs f(z_n)) / 2, then the tableau row
    double e = 0.0;
    for (int m = threadIdx.x; m < sz; m += 64) {
      const int id = mem[m];
      double* r = a.big + (size_t)id * kBigRec;
      double d[6], t[6];
      d[0] = r[kBigZc + 3];
      d[1] = r[kBigZc + 4];
      d[2] = r[kBigZc + 5];
      ha_accel_big(a, mem, sz, m, r[kBigZc], r[kBigZc + 1], r[kBigZc + 2], a.rc[id], d[3], d[4],
                   d[5]);
#pragma unroll
      for (int c = 0; c < 6; ++c) t[c] = 0.5 * (r[kBigZp + c] + r[kBigZc + c] + hs * d[c]);
      double* R = r + kBigR;
      for (int j = 1; j <= k; ++j) {
        const double ratio = (double)nk / (double)(2 * (k - j + 1));
        const double den = ratio * ratio - 1.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double u = t[c] + (t[c] - R[6 * (j - 1) + c]) / den;
          R[6 * (j - 1) + c] = t[c];
          t[c] = u;
        }
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) R[6 * k + c] = t[c];
      if (k >= 1) e = fmax(e, fmax(relerr3(R + 6 * k, R + 6 * (k - 1)),
                                   relerr3(R + 6 * k + 3, R + 6 * (k - 1) + 3)));
    }
    e = wave_max(e);
    wsync();
    if (k >= 1 && e <= a.tol) {
      for (int m = threadIdx.x; m < sz; m += 64) {
        double* r = a.big + (size_t)mem[m] * kBigRec;
#pragma unroll
        for (int c = 0; c < 6; ++c) r[kBigY0 + c] = r[kBigR + 6 * k + c];
      }
      wsync();
      return true;
    }
  }
  return false;
}

// Group g of sz > 64 members gm[0 .. sz - 1] at offset o: members sorted
// into bmem, state from the pre-drift copy, binary refinement over tau as
// bs_integrate does, result written back; returns the BS status (0, or -1
// when the depth or the attempt cap is exhausted) and the group's momentum
// change.
__device__ int bs_group_big(const BsArgs& a, const int* gm, int o, int sz, long long* nsub,
                            double& dpx, double& dpy, double& dpz) {
  const int lane = threadIdx.x;
  int* mem = a.bmem + o;
  for (int m = lane; m < sz; m += 64) {
    const int id = gm[m];
    int rank = 0;
    for (int q = 0; q < sz; ++q) rank += gm[q] < id ? 1 : 0;
    mem[rank] = id;
  }
  wsync();
  for (int m = lane; m < sz; m += 64) {
    const int id = mem[m];
    const double4 p = a.xpre[id], q = a.vpre[id];
    double* r = a.big + (size_t)id * kBigRec;
    r[kBigY0 + 0] = p.x;
    r[kBigY0 + 1] = p.y;
    r[kBigY0 + 2] = p.z;
    r[kBigY0 + 3] = q.x;
    r[kBigY0 + 4] = q.y;
    r[kBigY0 + 5] = q.z;
  }
  wsync();
  const int D = a.max_depth;
  const long long total = 1ll << D;
  long long pos = 0;
  int d = 0, attempts = 0, status = 0;
  while (pos < total) {
    if (++attempts > kBsMaxAttempts) {
      status = -1;
      break;
    }
    if (big_attempt(a, mem, sz, ldexp(a.dt, -d))) {
      ++*nsub;
      pos += 1ll << (D - d);
      while (d > 0 && (pos % (1ll << (D - d + 1))) == 0) --d;
    } else {
      ++d;
      if (d > D) {
        status = -1;
        break;
      }
    }
  }
  dpx = dpy = dpz = 0.0;
  for (int m = lane; m < sz; m += 64) {
    const int id = mem[m];
    const double* r = a.big + (size_t)id * kBigRec;
    const double mass = a.xm[id].w;
    const double4 vo = a.vv[id];
    dpx += mass * (r[kBigY0 + 3] - vo.x);
    dpy += mass * (r[kBigY0 + 4] - vo.y);
    dpz += mass * (r[kBigY0 + 5] - vo.z);
    a.xm[id] = make_double4(r[kBigY0], r[kBigY0 + 1], r[kBigY0 + 2], mass);
    a.vv[id] = make_double4(r[kBigY0 + 3], r[kBigY0 + 4], r[kBigY0 + 5], 0.0);
  }
  return status;
}

// Depth-slot exchange of the waves integrating one group.
struct BsXchg {
  int gs[kBsWaves];         // each wave's first accepted slot (INT_MAX: none)
  double y[kBsPar][6];      // the winning slot's state per member
};

// Binary refinement over [0, H] of a group of sz <= P members by the
// kBsWaves waves of the workgroup: in each round wave w tries the depths
// d + w S .. d + w S + S - 1 (S = kBsPar / P per wave, as bs_round_par lays
// them out), so that kBsWaves S halvings of the substep are attempted at
// once from the same start.  The first accepted slot in sequential order
// wins; its state reaches every wave through LDS, and the waves, holding the
// same state, position and depth, go on together.  The substeps taken and
// their results are those of the one-wave bs_integrate_par.
template <int P>
__device__ __forceinline__ int bs_integrate_mw(int sz, double y[6], double H,
                                               const ParBody<P>& Q, double G, double Gm0,
                                               double tol, int D, long long* nsub, BsXchg& X) {
  constexpr int S = kBsPar / P;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = par_memb<P>(lane);
  long long pos = 0;
  const long long total = 1ll << D;
  int d = 0, attempts = 0;
  while (pos < total) {
    if (++attempts > kBsMaxAttempts) return -1;
    const int smax = min(kBsWaves * S, D - d + 1);  // never beyond the depth limit
    double yt[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) yt[q] = y[q];
    int gs = INT_MAX;
    if (wave * S < smax) {
      const int sa = bs_round_par<P, false>(sz, yt, ldexp(H, -(d + wave * S)), Q, G, Gm0, tol);
      if (sa >= 0 && wave * S + sa < smax) gs = wave * S + sa;
    }
    if (lane == 0) X.gs[wave] = gs;
    __syncthreads();
    int best = X.gs[0];
#pragma unroll
    for (int w = 1; w < kBsWaves; ++w) best = min(best, X.gs[w]);
    if (best != INT_MAX) {
      if (wave == best / S && lane == par_lane<P>(0, 0, b)) {
#pragma unroll
        for (int q = 0; q < 6; ++q) X.y[b][q] = yt[q];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 6; ++q) y[q] = X.y[b][q];
      d += best;
      ++*nsub;
      pos += 1ll << (D - d);
      while (d > 0 && (pos % (1ll << (D - d + 1))) == 0) --d;
    } else {
      d += smax;
    }
    // X is written again only after every wave has read it
    __syncthreads();
    if (d > D) return -1;
  }
  return 0;
}

// Main-mode group of sz <= P members without collisions (sorted indices in
// mem; masses and radii staged in mm, mrc), on all waves of the workgroup:
// start from the pre-drift copy, integrate, wave 0 writes back; returns the
// BS status and, in wave 0, per member lane, its momentum change
// m (v_BS - v_drift).
template <int P>
__device__ __forceinline__ int bs_member_group(const BsArgs& a, int sz, const int* mem,
                                               double* mm, double* mrc, BsXchg& X,
                                               long long* nsub, double& dpx, double& dpy,
                                               double& dpz) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = par_memb<P>(lane);
  const int id = b < sz ? mem[b] : -1;
  // every load the group needs is issued at once: the members' masses and
  // radii (one per lane), their pre-drift states and drifted velocities
  const int ml = lane < sz ? mem[lane] : -1;
  double mw = 0.0, rcw = 0.0;
  if (ml >= 0) {
    mw = a.xm[ml].w;
    rcw = a.rc[ml];
  }
  double y[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double4 vo = make_double4(0.0, 0.0, 0.0, 0.0);
  if (id >= 0) {
    const double4 p = a.xpre[id], q = a.vpre[id];
    vo = a.vv[id];
    y[0] = p.x;
    y[1] = p.y;
    y[2] = p.z;
    y[3] = q.x;
    y[4] = q.y;
    y[5] = q.z;
  }
  if (ml >= 0 && wave == 0) {
    mm[lane] = mw;
    mrc[lane] = rcw;
  }
  __syncthreads();
  const ParBody<P> Q = par_body<P>(sz, mm, mrc);
  const int r = bs_integrate_mw<P>(sz, y, a.dt, Q, a.G, a.Gm0, a.tol, a.max_depth, nsub, X);
  dpx = dpy = dpz = 0.0;
  if (wave == 0 && lane == par_lane<P>(0, 0, b) && id >= 0) {  // one lane per member writes
    const double m = mm[b];
    dpx = m * (y[3] - vo.x);
    dpy = m * (y[4] - vo.y);
    dpz = m * (y[5] - vo.z);
    a.xm[id] = make_double4(y[0], y[1], y[2], m);
    a.vv[id] = make_double4(y[3], y[4], y[5], 0.0);
  }
  return r;
}

// ---- groups whose members can collide (Sec. 3.2.7) ----------------------------
// Member t of the group (ascending row) sits in lane t < sz: its pre-drift
// state pre[], mass, critical and physical radius, spin and original row.
// The group is integrated by the path its size selects; when two members
// touch during a substep (the Hermite test of Eqs. 10-12 over the substep)
// the integration stops at the start of that substep, the pair merges there
// (the more massive survives, the lower row on equal masses; mass, momentum
// and orbital-plus-spin angular momentum kept, the summed volume, the larger
// critical radius for the rest of the step), the merger is recorded, the
// absorbed member leaves the lanes, and the group, one member fewer, goes on
// over the rest of the step (the batched kernel's rule).
template <int P>
__device__ __forceinline__ int coll_par(const BsArgs& a, int sz, double pre[6], double m,
                                        double rc, double Rd, double* mm, double* mrc, double* mR,
                                        long long* nsub, double H, int* key, long long* cpos) {
  const int lane = threadIdx.x & 63;
  const int b = par_memb<P>(lane);
  double y[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) y[c] = __shfl(pre[c], b < sz ? b : 0, 64);
  if (b >= sz) {
    y[0] = 1.0;
    y[1] = y[2] = y[3] = y[4] = y[5] = 0.0;
  }
  wsync();
  if (lane < sz) {
    mm[lane] = m;
    mrc[lane] = rc;
    mR[lane] = Rd;
  }
  wsync();
  const int r = bs_group<P, false>(sz, y, mm, mrc, H, a.G, a.Gm0, a.tol, a.max_depth, nsub, -1.0,
                                   key, cpos, mR);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double t = __shfl(y[c], par_lane<P>(0, 0, min(lane, P - 1)), 64);
    if (lane < sz) pre[c] = t;
  }
  return r;
}

__device__ int bs_group_coll(const BsArgs& a, int g, int sz, const int* mem, double* mm,
                             double* mrc, double* mR, double (*R)[6][64], long long* nsub,
                             double& dpx, double& dpy, double& dpz, double& Ug) {
  const int lane = threadIdx.x & 63;
  const bool act = lane < sz;  // members at the start
  int id = act ? mem[lane] : 0;
  double pre[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double m = 0.0, rc = 0.0, Rd = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
  double b0x = 0.0, b0y = 0.0, b0z = 0.0;  // momentum before, after the drift
  if (act) {
    const double4 p = a.xpre[id], q = a.vpre[id], vo = a.vv[id], sv = a.sp[id];
    pre[0] = p.x;
    pre[1] = p.y;
    pre[2] = p.z;
    pre[3] = q.x;
    pre[4] = q.y;
    pre[5] = q.z;
    m = a.xm[id].w;
    rc = a.rc_w[id];
    Rd = a.rad[id];
    S0 = sv.x;
    S1 = sv.y;
    S2 = sv.z;
    b0x = m * vo.x;
    b0y = m * vo.y;
    b0z = m * vo.z;
  }
  const long long step = (long long)a.st->nstep - 1;
  double H = a.dt, f0 = 0.0;
  Ug = 0.0;
  int status = 0;
  for (;;) {
    long long gsub = 0, cpos = 0;
    int key = -1, st;
    if (sz <= 2)
      st = coll_par<2>(a, sz, pre, m, rc, Rd, mm, mrc, mR, &gsub, H, &key, &cpos);
    else if (sz <= 4)
      st = coll_par<4>(a, sz, pre, m, rc, Rd, mm, mrc, mR, &gsub, H, &key, &cpos);
    else if (sz <= kBsPar)
      st = coll_par<8>(a, sz, pre, m, rc, Rd, mm, mrc, mR, &gsub, H, &key, &cpos);
    else
      st = bs_integrate(sz, lane, pre, H, lane < sz ? m : 0.0, lane < sz ? rc : 0.0, a.G, a.Gm0,
                        a.tol, a.max_depth, R, &gsub, lane < sz ? Rd : 0.0, &key, &cpos);
    *nsub += gsub;
    if (st != 1) {
      status = st;
      break;
    }
    // members key >> 6 < key & 63 touch: merge them at the start of that
    // substep, then the rest of the step with one member fewer
    const double fc = ldexp((double)cpos, -a.max_depth);
    const int la = key >> 6, lb = key & 63;
    const double mla = readlane_d(m, la), mlb = readlane_d(m, lb);
    const int ls = mlb > mla ? lb : la, lg = ls == la ? lb : la;
    double ys[6], yg[6], ss[3], sg[3], ym[6], sm[3], Mm, Rm;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      ys[c] = readlane_d(pre[c], ls);
      yg[c] = readlane_d(pre[c], lg);
    }
    ss[0] = readlane_d(S0, ls);
    ss[1] = readlane_d(S1, ls);
    ss[2] = readlane_d(S2, ls);
    sg[0] = readlane_d(S0, lg);
    sg[1] = readlane_d(S1, lg);
    sg[2] = readlane_d(S2, lg);
    const double ms = readlane_d(m, ls), mg = readlane_d(m, lg);
    const double Rs = readlane_d(Rd, ls), Rg = readlane_d(Rd, lg);
    const double Uc = merge_bodies(a.G, ms, mg, ys, yg, Rs, Rg, ss, sg, Mm, ym, Rm, sm);
    const double frac = f0 + (1.0 - f0) * fc;
    const int ids_s = a.ids[__builtin_amdgcn_readlane(id, ls)];
    const int idg = __builtin_amdgcn_readlane(id, lg);
    const int ids_g = a.ids[idg];
    const double rcm = fmax(readlane_d(rc, ls), readlane_d(rc, lg));
    if (lane == 0) {
      const unsigned long long k = atomicAdd(&a.st->ev_cnt, 1ull);
      if ((long long)k < a.ev_cap) {
        genga_event e;
        e.kind = GENGA_EV_MERGE;
        e.sys = 0;
        e.id_i = ids_s;
        e.id_j = ids_g;
        e.step = step;
        e.frac = frac;
        e.m_i = ms;
        e.m_j = mg;
        e.R_i = Rs;
        e.R_j = Rg;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          e.x_i[q] = ys[q];
          e.v_i[q] = ys[3 + q];
          e.s_i[q] = ss[q];
          e.x_j[q] = yg[q];
          e.v_j[q] = yg[3 + q];
          e.s_j[q] = sg[q];
        }
        e.U = Uc;
        a.ev[k] = e;
      }
      a.dead[idg] = 1;
    }
    Ug += Uc;
    if (lane == ls) {
#pragma unroll
      for (int c = 0; c < 6; ++c) pre[c] = ym[c];
      m = Mm;
      Rd = Rm;
      S0 = sm[0];
      S1 = sm[1];
      S2 = sm[2];
      rc = rcm;
    }
    // the absorbed member leaves: the lanes above it move down by one
    const int src = lane >= lg ? min(lane + 1, 63) : lane;
#pragma unroll
    for (int c = 0; c < 6; ++c) pre[c] = __shfl(pre[c], src, 64);
    m = __shfl(m, src, 64);
    rc = __shfl(rc, src, 64);
    Rd = __shfl(Rd, src, 64);
    S0 = __shfl(S0, src, 64);
    S1 = __shfl(S1, src, 64);
    S2 = __shfl(S2, src, 64);
    id = __shfl(id, src, 64);
    --sz;
    H = H * (1.0 - fc);
    f0 = frac;
  }
  // survivors written back; the group's momentum change for the second Sun
  // kick includes the absorbed members' momentum before the step
  double ax = 0.0, ay = 0.0, az = 0.0;
  if (lane < sz) {
    a.xm[id] = make_double4(pre[0], pre[1], pre[2], m);
    a.vv[id] = make_double4(pre[3], pre[4], pre[5], 0.0);
    a.rad[id] = Rd;
    a.sp[id] = make_double4(S0, S1, S2, 0.0);
    a.rc_w[id] = rc;
    ax = m * pre[3];
    ay = m * pre[4];
    az = m * pre[5];
  }
  dpx = ax - b0x;
  dpy = ay - b0y;
  dpz = az - b0z;
  return status;
}

// A group that wave 0 integrates alone (wave 0 only): members that can
// collide, or more than kBsPar members (one lane per member; more than 64
// in the per-body records).  Writes the group's momentum change and merger
// energy to dP.
__device__ __forceinline__ void bs_group_one(const BsArgs& a, const int* gmem, int g, int o,
                                             int sz, int* mem, double* mm, double* mrc,
                                             double* mR, double (*R)[6][64], long long* nsub) {
  const int lane = threadIdx.x & 63;
  if (a.coll && sz > kBsMaxGroup) {
    // collisions are tested in groups of up to 64 members only
    if (lane == 0) atomicOr(&a.st->flags, F_GROUP);
    return;
  }
  double dpx = 0.0, dpy = 0.0, dpz = 0.0, Ug = 0.0;
  if (sz > kBsMaxGroup) {
    const int r = bs_group_big(a, gmem + o, o, sz, nsub, dpx, dpy, dpz);
    if (r != 0 && lane == 0) atomicOr(&a.st->flags, F_BS);
  } else {
    const int my = lane < sz ? gmem[o + lane] : INT_MAX;
    int rank = 0;
    for (int q = 0; q < sz; ++q) rank += (__builtin_amdgcn_readlane(my, q) < my) ? 1 : 0;
    if (lane < sz) mem[rank] = my;
    wsync();
    if (a.coll) {
      const int r = bs_group_coll(a, g, sz, mem, mm, mrc, mR, R, nsub, dpx, dpy, dpz, Ug);
      if (r != 0 && lane == 0) atomicOr(&a.st->flags, F_BS);
    } else {
      const int bb = lane < sz ? mem[lane] : -1;
      double y[6] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      double m = 0.0, rc = 0.0;
      if (bb >= 0) {
        const double4 p = a.xpre[bb], q = a.vpre[bb];
        y[0] = p.x;
        y[1] = p.y;
        y[2] = p.z;
        y[3] = q.x;
        y[4] = q.y;
        y[5] = q.z;
        m = a.xm[bb].w;
        rc = a.rc[bb];
      }
      const int r = bs_integrate(sz, lane, y, a.dt, m, rc, a.G, a.Gm0, a.tol,
                                 a.max_depth, R, nsub);
      if (r != 0 && lane == 0) atomicOr(&a.st->flags, F_BS);
      if (bb >= 0) {
        const double4 vo = a.vv[bb];
        dpx = m * (y[3] - vo.x);
        dpy = m * (y[4] - vo.y);
        dpz = m * (y[5] - vo.z);
        a.xm[bb] = make_double4(y[0], y[1], y[2], m);
        a.vv[bb] = make_double4(y[3], y[4], y[5], 0.0);
      }
    }
  }
  // the group's momentum change for the second Sun kick (fixed lane order)
  dpx = wave_sum(dpx);
  dpy = wave_sum(dpy);
  dpz = wave_sum(dpz);
  if (lane == 0) {
    a.dP[4 * g + 0] = dpx;
    a.dP[4 * g + 1] = dpy;
    a.dP[4 * g + 2] = dpz;
    a.dP[4 * g + 3] = Ug;  // internal energy of the group's mergers
  }
}

// LDS of one workgroup's BS.
struct BsLds {
  double R[kBsCols][6][64];
  int mem[64];
  double mm[kBsPar], mrc[kBsPar], mR[kBsPar];
  BsXchg X;
};

// The ng groups (offsets goff[0 .. ng], members gmem at those offsets, in
// global memory or LDS) on the workgroups of the grid, one group at a time
// per workgroup (grid-stride): members sorted ascending, state reset to the
// pre-drift copy, H_A integrated over tau by BS, result written back.
// Groups of up to 8 members take the all-columns path with speculative
// depths over every wave; the others take wave 0 alone (one lane per
// member with the columns in sequence, or the collision path).
__device__ __forceinline__ void bs_groups(const BsArgs& a, int ng, const int* goff,
                                          const int* gmem, BsLds& L) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  long long nsub = 0;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    const int o = goff[g];
    const int sz = goff[g + 1] - o;
    if (!a.coll && sz <= kBsPar) {
      // every wave ranks the members; wave 0 writes them in order
      const int my = lane < sz ? gmem[o + lane] : INT_MAX;
      int rank = 0;
      for (int q = 0; q < sz; ++q) rank += (__builtin_amdgcn_readlane(my, q) < my) ? 1 : 0;
      if (wave == 0 && lane < sz) L.mem[rank] = my;
      __syncthreads();
      double dpx, dpy, dpz;
      int r;
      if (sz <= 2)
        r = bs_member_group<2>(a, sz, L.mem, L.mm, L.mrc, L.X, &nsub, dpx, dpy, dpz);
      else if (sz <= 4)
        r = bs_member_group<4>(a, sz, L.mem, L.mm, L.mrc, L.X, &nsub, dpx, dpy, dpz);
      else
        r = bs_member_group<8>(a, sz, L.mem, L.mm, L.mrc, L.X, &nsub, dpx, dpy, dpz);
      if (wave == 0) {
        if (r != 0 && lane == 0) atomicOr(&a.st->flags, F_BS);
        // the group's momentum change for the second Sun kick (fixed lane order)
        dpx = wave_sum(dpx);
        dpy = wave_sum(dpy);
        dpz = wave_sum(dpz);
        if (lane == 0) {
          a.dP[4 * g + 0] = dpx;
          a.dP[4 * g + 1] = dpy;
          a.dP[4 * g + 2] = dpz;
          a.dP[4 * g + 3] = 0.0;
        }
      }
    } else if (wave == 0) {
      bs_group_one(a, gmem, g, o, sz, L.mem, L.mm, L.mrc, L.mR, L.R, &nsub);
    }
    // the group's LDS (mem, mm, mrc, mR, R, X) is free for the next one
    __syncthreads();
  }
  if (threadIdx.x == 0 && nsub > 0) atomicAdd(&a.st->bs_sub, (unsigned long long)nsub);
}

// BS of the groups that the grouping kernel left in global memory.
__global__ __launch_bounds__(64 * kBsWaves) void k_bs(BsArgs a) {
  __shared__ BsLds L;
  if (a.st->flags & F_NMIN) return;  // the run stopped below nmin bodies
  const int ng = __builtin_amdgcn_readfirstlane(a.st->ngroups);
  bs_groups(a, ng, a.goff, a.gmem, L);
}

// Grouping (App. A) and BS (Sec. 3.2.6) in one launch: every workgroup
// forms the groups of the step's encounter pairs in its own LDS (the same
// groups, offsets and member sets in each: the labels and offsets come from
// the pairs alone), so no workgroup waits for another before its BS; one
// also writes the groups, the counts and the cleared candidate table to
// global memory.
struct GroupBsLds {
  GroupLds<64 * kBsWaves> g;
  int gm[kGroupMaxN];
  BsLds b;
};
__global__ __launch_bounds__(64 * kBsWaves) void k_group_bs(EncArgs e, BsArgs a) {
  constexpr int NT = 64 * kBsWaves;
  __shared__ GroupBsLds L;
  // the status word, the pair count and the list's first NT entries (a
  // step's pairs are fewer, as a rule) are loaded together; entries past the
  // count are dropped, and any beyond NT are read once the count is known
  const unsigned fl = a.st->flags;
  const int ne_all = e.st->nenc;
  const int2 pf = (int)threadIdx.x < e.enc_cap ? e.encij[threadIdx.x] : make_int2(0, 0);
  if (fl & F_NMIN) return;  // the run stopped below nmin bodies
  // the last workgroup, which rarely has a group of its own, writes the
  // global results
  const int ng = group_phase<NT>(e, ne_all, L.g, L.gm, blockIdx.x == gridDim.x - 1, &pf);
  bs_groups(a, ng, L.g.gof, L.gm, L.b);
}

// ---- bodies leaving the system (Sec. 3.2.7, 3.2.8, 3.4.6) ------------------
struct CompactArgs {
  double4* __restrict__ xs;
  double4* __restrict__ xm;
  double4* __restrict__ vv;
  double* __restrict__ rc;
  double* __restrict__ thr;
  double* __restrict__ tmax64;
  double* __restrict__ rad;
  double4* __restrict__ sp;
  int* __restrict__ ids;
  int* __restrict__ dead;
  const double* __restrict__ dP;
  genga_event* __restrict__ ev;
  DevStat* __restrict__ st;
  int np, nmin, ev_cap;
  double rcut, rcut_sun;
};

// After BS, in one workgroup: the groups' merger energies added in group
// order; bodies beyond rcut or inside rcut_sun of the central mass leave
// (recorded); then every freed row, in descending order, takes the last
// body (the oracle's compaction), the rows past the count become padding
// (massless at the origin), the 64-body threshold maxima are rebuilt, and
// with fewer than nmin bodies left the run stops (later steps do nothing).
__global__ __launch_bounds__(1024) void k_compact(CompactArgs a) {
  __shared__ int dl[kGroupMaxN];
  __shared__ int s_nd;
  const int tid = threadIdx.x;
  if (a.st->flags & F_NMIN) return;
  const int n = a.st->nlive;
  const long long step = (long long)a.st->nstep - 1;
  if (tid == 0) {
    s_nd = 0;
    double U = 0.0;
    for (int g = 0; g < a.st->ngroups; ++g) U += a.dP[4 * g + 3];
    a.st->U += U;
  }
  __syncthreads();
  for (int i = tid; i < n; i += 1024) {
    if (!a.dead[i] && (a.rcut > 0.0 || a.rcut_sun > 0.0)) {
      const double4 p = a.xm[i];
      const double r = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
      int kind = 0;
      if (a.rcut > 0.0 && r > a.rcut) kind = GENGA_EV_EJECT_FAR;
      if (a.rcut_sun > 0.0 && r < a.rcut_sun) kind = GENGA_EV_EJECT_SUN;
      if (kind) {
        const unsigned long long k = atomicAdd(&a.st->ev_cnt, 1ull);
        if ((long long)k < a.ev_cap) {
          const double4 q = a.vv[i], s = a.sp[i];
          genga_event e;
          e.kind = kind;
          e.sys = 0;
          e.id_i = a.ids[i];
          e.id_j = -1;
          e.step = step;
          e.frac = 1.0;
          e.m_i = p.w;
          e.m_j = 0.0;
          e.R_i = a.rad[i];
          e.R_j = 0.0;
          e.x_i[0] = p.x;
          e.x_i[1] = p.y;
          e.x_i[2] = p.z;
          e.v_i[0] = q.x;
          e.v_i[1] = q.y;
          e.v_i[2] = q.z;
          e.s_i[0] = s.x;
          e.s_i[1] = s.y;
          e.s_i[2] = s.z;
          for (int c = 0; c < 3; ++c) e.x_j[c] = e.v_j[c] = e.s_j[c] = 0.0;
          e.U = 0.0;
          a.ev[k] = e;
        }
        a.dead[i] = 2;  // ejected (1: absorbed in a merger)
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < n; i += 1024)
    if (a.dead[i]) dl[atomicAdd(&s_nd, 1)] = i;
  __syncthreads();
  const int nd = s_nd;
  if (tid == 0) {
    // freed rows in descending order: a short insertion sort of the list
    for (int k = 1; k < nd; ++k) {
      const int v = dl[k];
      int q = k - 1;
      while (q >= 0 && dl[q] < v) {
        dl[q + 1] = dl[q];
        --q;
      }
      dl[q + 1] = v;
    }
    // the ejected bodies' momentum, in that order, leaves with them: the
    // second Sun kick takes the momentum of the bodies that stay
    double ex = 0.0, ey = 0.0, ez = 0.0;
    for (int k = 0; k < nd; ++k) {
      const int h = dl[k];
      if (a.dead[h] == 2) {
        const double mh = a.xm[h].w;
        const double4 q = a.vv[h];
        ex += mh * q.x;
        ey += mh * q.y;
        ez += mh * q.z;
      }
    }
    a.st->Pej[0] = ex;
    a.st->Pej[1] = ey;
    a.st->Pej[2] = ez;
    int nn = n;
    for (int k = 0; k < nd; ++k) {
      const int h = dl[k];
      const int last = nn - 1;
      if (h != last) {
        a.xm[h] = a.xm[last];
        a.vv[h] = a.vv[last];
        a.rc[h] = a.rc[last];
        a.thr[h] = a.thr[last];
        a.rad[h] = a.rad[last];
        a.sp[h] = a.sp[last];
        a.ids[h] = a.ids[last];
      }
      a.xs[last] = make_double4(0.0, 0.0, 0.0, 0.0);
      a.xm[last] = make_double4(0.0, 0.0, 0.0, 0.0);
      a.vv[last] = make_double4(0.0, 0.0, 0.0, 0.0);
      a.rc[last] = 0.0;
      a.thr[last] = kTiny;
      a.rad[last] = 0.0;
      a.sp[last] = make_double4(0.0, 0.0, 0.0, 0.0);
      a.ids[last] = -1;
      a.dead[h] = 0;
      nn = last;
    }
    a.st->nlive = nn;
    if (nn < a.nmin) atomicOr(&a.st->flags, F_NMIN);
  }
  __syncthreads();
  if (nd > 0) {
    // the moved rows' thresholds: rebuild every 64-body chunk maximum
    const int w = tid >> 6, lane = tid & 63;
    for (int c = w; c < a.np / 64; c += 16) {
      double t = a.thr[64 * c + lane];
      t = wave_max(t);
      if (lane == 0) a.tmax64[c] = t;
    }
  }
}

// Every body present in its own row, no spins, none leaving; radii cleared
// only with clear_rad (init; a new state keeps them).
__global__ __launch_bounds__(256) void k_bodies_reset(int* __restrict__ ids,
                                                      double4* __restrict__ sp,
                                                      int* __restrict__ dead,
                                                      double* __restrict__ rad,
                                                      DevStat* __restrict__ st, int n, int np,
                                                      int clear_rad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    st->nlive = n;
    st->stopped = 0;
  }
  if (i >= np) return;
  ids[i] = i < n ? i : -1;
  sp[i] = make_double4(0.0, 0.0, 0.0, 0.0);
  dead[i] = 0;
  if (clear_rad) rad[i] = 0.0;
}

// ---------------------------------------------------------------------------
// packing, coordinates, radii, energy

// P = sum m v and M = sum m over n bodies given as n x 3 (src3) or double4.
__global__ __launch_bounds__(1024) void k_momentum(const double* __restrict__ m,
                                                   const double* __restrict__ v3,
                                                   const double4* __restrict__ xm,
                                                   const double4* __restrict__ vv,
                                                   int n, double* __restrict__ out) {
  __shared__ double sh[16];
  double px = 0.0, py = 0.0, pz = 0.0, mm = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    double mi, vx, vy, vz;
    if (v3) {
      mi = m[i];
      vx = v3[3 * i];
      vy = v3[3 * i + 1];
      vz = v3[3 * i + 2];
    } else {
      mi = xm[i].w;
      vx = vv[i].x;
      vy = vv[i].y;
      vz = vv[i].z;
    }
    px += mi * vx;
    py += mi * vy;
    pz += mi * vz;
    mm += mi;
  }
  const double Px = block_sum<1024>(px, sh);
  const double Py = block_sum<1024>(py, sh);
  const double Pz = block_sum<1024>(pz, sh);
  const double M = block_sum<1024>(mm, sh);
  if (threadIdx.x == 0) {
    out[0] = Px;
    out[1] = Py;
    out[2] = Pz;
    out[3] = M;
  }
}

// Heliocentric velocities become barycentric: v = u - sum m u / (m0 + sum m).
// Rows n..np-1 (padding) become massless bodies at the origin in x and xs:
// the pair kernel runs over them and their terms are exact zeros.
__global__ void k_pack(const double* __restrict__ m, const double* __restrict__ x,
                       const double* __restrict__ v, const double* __restrict__ mom,
                       double4* __restrict__ xm, double4* __restrict__ vv,
                       double4* __restrict__ xs, int n, int np, int helio, double m0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  if (i >= n) {
    xm[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    vv[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    xs[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    return;
  }
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    const double den = m0 + mom[3];
    sx = mom[0] / den;
    sy = mom[1] / den;
    sz = mom[2] / den;
  }
  xm[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], m[i]);
  vv[i] = make_double4(v[3 * i] - sx, v[3 * i + 1] - sy, v[3 * i + 2] - sz, 0.0);
}

// Barycentric velocities back to heliocentric: u = v + sum m v / m0.
__global__ void k_unpack(const double4* __restrict__ xm, const double4* __restrict__ vv,
                         const double* __restrict__ mom, double* __restrict__ x,
                         double* __restrict__ v, int n, int helio, double m0,
                         const DevStat* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i >= st->nlive) {  // a body that left: NaN row
    const double q = __builtin_nan("");
    for (int c = 0; c < 3; ++c) x[3 * i + c] = v[3 * i + c] = q;
    return;
  }
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    sx = mom[0] / m0;
    sy = mom[1] / m0;
    sz = mom[2] / m0;
  }
  const double4 p = xm[i], q = vv[i];
  x[3 * i] = p.x;
  x[3 * i + 1] = p.y;
  x[3 * i + 2] = p.z;
  v[3 * i] = q.x + sx;
  v[3 * i + 1] = q.y + sy;
  v[3 * i + 2] = q.z + sz;
}

// Radii of the first step (Eq. 6), thresholds, empty candidate table.
__global__ __launch_bounds__(256) void k_rcrit_init(
    const double4* __restrict__ xm, const double4* __restrict__ vv, double* __restrict__ rc,
    double* __restrict__ thr, double* __restrict__ tmax64, int* __restrict__ ccnt, int n,
    double mu, double m0, double n1, double n2, double absdt, double pf2, int enc_free) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // grid: the padded count
  double t = kTiny;
  if (i < n) {
    const double4 p = xm[i], q = vv[i];
    const double r = rcrit(p.x, p.y, p.z, q.x, q.y, q.z, p.w, mu, m0, n1, n2, absdt);
    rc[i] = r;
    t = enc_free ? kTiny : fmax(pf2 * r * r, kTiny);
    ccnt[i] = 0;
  }
  thr[i] = t;
  chunk_tmax(t, i & ~63, tmax64);
}

// Per-body energy terms and angular momentum; rows[8 i + k]:
// kinetic, -G m0 m/r, -1/2 G m sum_j m_j/r_ij, m v (3), m x x v (3) -> 9 terms
__global__ void k_energy_rows(const double4* __restrict__ xm, const double4* __restrict__ vv,
                              int n, double G, double m0, double* __restrict__ rows,
                              const DevStat* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i >= st->nlive) {  // padding rows (bodies that left) add nothing
    for (int k = 0; k < 9; ++k) rows[9 * (size_t)i + k] = 0.0;
    return;
  }
  const double4 p = xm[i], q = vv[i];
  double pp = 0.0;
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    const double4 pj = xm[j];
    const double dx = pj.x - p.x, dy = pj.y - p.y, dz = pj.z - p.z;
    pp += pj.w / sqrt(dx * dx + dy * dy + dz * dz);
  }
  double* r = rows + 9 * (size_t)i;
  r[0] = 0.5 * p.w * (q.x * q.x + q.y * q.y + q.z * q.z);
  r[1] = -G * m0 * p.w / sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  r[2] = -0.5 * G * p.w * pp;
  r[3] = p.w * q.x;
  r[4] = p.w * q.y;
  r[5] = p.w * q.z;
  r[6] = p.w * (p.y * q.z - p.z * q.y);
  r[7] = p.w * (p.z * q.x - p.x * q.z);
  r[8] = p.w * (p.x * q.y - p.y * q.x);
}

__global__ __launch_bounds__(256) void k_energy_final(const double* __restrict__ rows,
                                                       int n, double m0,
                                                       double* __restrict__ E,
                                                       double* __restrict__ L) {
  __shared__ double sh[16];
  double t[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) t[k] = 0.0;
  for (int i = threadIdx.x; i < n; i += 256)
#pragma unroll
    for (int k = 0; k < 9; ++k) t[k] += rows[9 * (size_t)i + k];
  double s[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) s[k] = block_sum<256>(t[k], sh);
  if (threadIdx.x == 0) {
    E[0] = s[0] + (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]) / (2.0 * m0) + s[1] + s[2];
    L[0] = s[6];
    L[1] = s[7];
    L[2] = s[8];
  }
}

// Candidate thresholds from given radii: max((pf rc)^2, tiny).
__global__ __launch_bounds__(256) void k_thresholds(const double* __restrict__ rc,
                                                    double* __restrict__ thr,
                                                    double* __restrict__ tmax64,
                                                    int* __restrict__ ccnt, int n, double pf2,
                                                    int enc_free) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // grid: the padded count
  double t = kTiny;
  if (i < n) {
    t = enc_free ? kTiny : fmax(pf2 * rc[i] * rc[i], kTiny);
    ccnt[i] = 0;
  }
  thr[i] = t;
  chunk_tmax(t, i & ~63, tmax64);
}

// Radii given by the caller: installed with their thresholds (zero and the
// smallest threshold when rc_in is null, the K = 1 map).
__global__ __launch_bounds__(256) void k_radii_in(const double* __restrict__ rc_in,
                                                  double* __restrict__ rc,
                                                  double* __restrict__ thr,
                                                  double* __restrict__ tmax64,
                                                  int* __restrict__ ccnt, int n, double pf2,
                                                  int enc_free) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // grid: the padded count
  double t = kTiny;
  if (i < n) {
    const double r = rc_in ? rc_in[i] : 0.0;
    rc[i] = r;
    t = enc_free ? kTiny : fmax(pf2 * r * r, kTiny);
    ccnt[i] = 0;
  }
  thr[i] = t;
  chunk_tmax(t, i & ~63, tmax64);
}

// Masses out of the packed state.
__global__ void k_masses(const double4* __restrict__ xm, double* __restrict__ m, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m[i] = xm[i].w;
}

// Every input value finite?  Sets *bad when not.
__global__ void k_validate(const double* __restrict__ a, int64_t cnt, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt && !isfinite(a[i])) atomicOr(bad, 1);
}

PairArgs pair_args(const MassiveWs& w, const StepConsts& c) {
  PairArgs a;
  a.rc = w.rc_cur;
  a.ccnt = w.ccnt;
  a.ctab = w.ctab;
  a.cr2 = w.cr2;
  a.pp = w.pp;
  a.njs = w.njs;
  a.jl = w.np / (w.njs * w.pw);
  a.xs = w.xs;
  a.vv = w.vv;
  a.afar = w.afar;
  a.rc_next = w.rc_next;
  a.acc_out = nullptr;
  a.partP2 = w.partP2;
  a.dP = w.dP;
  a.st = w.st;
  a.n = w.n;
  a.np = w.np;
  a.cpb = w.cpb;
  a.nblk = w.nblk;
  a.encounter_free = c.encounter_free;
  a.G = c.G;
  a.h = c.h;
  a.m0 = c.m0;
  a.mu = c.mu;
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.absdt = c.absdt_next;  // the next (sub-)step's radii are formed here
  a.pf = c.pf;
  return a;
}

// The pair kernel of the workspace's shape, and its workgroup size.
template <int MODE>
inline auto pair_kernel(const MassiveWs& w) {
  return w.pw == kPairWBig ? k_pair_part<MODE, kPairWBig> : k_pair_part<MODE, kPairW>;
}
inline dim3 pair_block(const MassiveWs& w) { return dim3(w.pw * 64); }

// Workgroups of the pair kernel: splits x 64-body blocks, the split fastest,
// so that consecutive workgroups (dispatched to the 8 XCDs in turn) take
// different splits: with 8 splits each XCD's L2 holds one split's partners.
inline dim3 pair_grid(const MassiveWs& w) { return dim3(w.njs, w.np / kPairBlock); }

}  // namespace

// ---------------------------------------------------------------------------
StepConsts make_consts(const genga_params& p) {
  StepConsts c;
  c.G = p.G;
  c.m0 = p.m0;
  c.mu = p.G * p.m0;
  c.dt = p.dt;
  c.h = 0.5 * p.dt;
  c.n1 = p.n1;
  c.n2 = p.n2;
  c.pf = p.pf;
  c.pf2 = p.pf * p.pf;
  c.bs_tol = p.bs_tol;
  c.bs_max_depth = p.bs_max_depth;
  c.kepler_max_iter = p.kepler_max_iter;
  c.encounter_free = p.encounter_free;
  c.absdt_next = fabs(p.dt);
  c.all_pairs = 0;
  c.rcut = p.rcut;
  c.rcut_sun = p.rcut_sun;
  c.nmin = p.nmin;
  c.coll = 0;
  c.phys = p.rcut > 0.0 || p.rcut_sun > 0.0 || p.nmin > 0;
  return c;
}

// Yoshida's symmetric compositions (fourth order; sixth order, his solution
// A), the coefficients as published.
int composition(int order, double* w) {
  if (order == 0 || order == 2) {
    w[0] = 1.0;
    return 1;
  }
  if (order == 4) {
    const double c = cbrt(2.0);
    w[0] = w[2] = 1.0 / (2.0 - c);
    w[1] = 1.0 - 2.0 * w[0];
    return 3;
  }
  if (order == 6) {
    const double w1 = -1.17767998417887, w2 = 0.235573213359357, w3 = 0.784513610477560;
    const double w0 = 1.0 - 2.0 * (w1 + w2 + w3);
    const double q[7] = {w3, w2, w1, w0, w1, w2, w3};
    for (int k = 0; k < 7; ++k) w[k] = q[k];
    return 7;
  }
  return 0;
}

genga_params accel_params(const genga_params& p) {
  genga_params q = p;
  q.cand_per_body = 1;
  q.enc_cap = 1;
  return q;
}

size_t massive_ws_bytes(int n, const genga_params& p, bool snap) {
  if (n < 1) return 0;
  MassiveWs w;
  return massive_carve(w, n, p, nullptr, snap);
}

// Lay the main-mode arrays out in the workspace starting at base (nullptr:
// only size the layout).  Returns the bytes used.
// Splits of the partner range per 64-body block of the pair kernel with W
// waves per workgroup: the largest divisor of np / (W waves x 2 partners)
// with splits x np at most target, so that small systems still spread over
// the whole chip (2048 bodies: 8 splits, 4096 waves) and every wave takes
// whole batches.
int pair_splits(int np, int W, int target) {
  const int q = np / (W * kPairU);
  int best = 1;
  for (int d = 1; d <= q; ++d)
    if (q % d == 0 && (size_t)d * np <= (size_t)target) best = d;
  return best;
}

// The pair kernel's shape for np padded bodies: waves per workgroup, splits.
void pair_shape(int np, int* pw, int* njs) {
  const bool big = np >= kPairBigN;
  *pw = big ? kPairWBig : kPairW;
  *njs = pair_splits(np, *pw, big ? kPairTargetBig : kPairTarget);
}

size_t massive_carve(MassiveWs& w, int n, const genga_params& p, void* base, bool snap) {
  w.n = n;
  w.np = ceil_div(n, 256) * 256;
  pair_shape(w.np, &w.pw, &w.njs);
  w.nblk = ceil_div(n, kOpenBlock);
  w.cpb = p.cand_per_body;
  w.enc_cap = p.enc_cap;
  const size_t np = (size_t)w.np;
  size_t off = 0;
  auto take = [&](size_t sz) -> void* {
    const size_t o = off;
    off += align256(sz);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  w.xm = (double4*)take(np * sizeof(double4));
  w.vv = (double4*)take(np * sizeof(double4));
  w.xs = (double4*)take(np * sizeof(double4));
  w.xpre = (double4*)take(np * sizeof(double4));
  w.vpre = (double4*)take(np * sizeof(double4));
  w.afar = (double4*)take(np * sizeof(double4));
  w.rc_cur = (double*)take(np * sizeof(double));
  w.rc_next = (double*)take(np * sizeof(double));
  w.thr = (double*)take(np * sizeof(double));
  w.tmax64 = (double*)take(np / 64 * sizeof(double));
  w.pp = (double*)take((size_t)w.njs * 6 * np * sizeof(double));
  w.partP = (double*)take((size_t)w.nblk * 4 * sizeof(double));
  w.partP2 = (double*)take((size_t)w.nblk * 4 * sizeof(double));
  w.dP = (double*)take((np / 2 + 1) * 4 * sizeof(double));
  w.red = (double*)take(std::max<size_t>(np * 9, 64) * sizeof(double));
  w.ccnt = (int*)take(np * sizeof(int));
  w.ctab = (int*)take(np * (size_t)std::max(1, w.cpb) * sizeof(int));
  w.cr2 = (double*)take(np * (size_t)std::max(1, w.cpb) * sizeof(double));
  w.khist = (unsigned long long*)take((size_t)w.nblk * kKepBins * sizeof(unsigned long long));
  w.encij = (int2*)take((size_t)std::max(1, w.enc_cap) * sizeof(int2));
  w.encd2 = (double*)take((size_t)std::max(1, w.enc_cap) * sizeof(double));
  w.encrc2 = (double*)take((size_t)std::max(1, w.enc_cap) * sizeof(double));
  w.goff = (int*)take((np + 1) * sizeof(int));
  w.gmem = (int*)take(np * sizeof(int));
  w.rad = (double*)take(np * sizeof(double));
  w.sp = (double4*)take(np * sizeof(double4));
  w.ids = (int*)take(np * sizeof(int));
  w.dead = (int*)take(np * sizeof(int));
  w.ev_cap = 2 * w.n + 16;  // every body leaves at most once
  w.ev = (genga_event*)take((size_t)w.ev_cap * sizeof(genga_event));
  w.bsbig = (double*)take(np * kBigRec * sizeof(double));
  w.bspos = (double4*)take(np * sizeof(double4));
  w.bsmem = (int*)take(np * sizeof(int));
  w.flag_in = (int*)take(sizeof(int));
  w.xstart = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.xpost = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.vpost = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.st = (DevStat*)take(sizeof(DevStat));
  return off;
}

hipError_t massive_reset_bodies(const MassiveWs& w, bool clear_radii, hipStream_t s) {
  hipLaunchKernelGGL(k_bodies_reset, dim3(ceil_div(w.np, 256)), dim3(256), 0, s, w.ids, w.sp,
                     w.dead, w.rad, w.st, w.n, w.np, clear_radii ? 1 : 0);
  return hipGetLastError();
}

hipError_t massive_pack(const MassiveWs& w, const StepConsts& c, const double* m,
                        const double* x, const double* v, int coords_in,
                        hipStream_t s) {
  const int helio = coords_in == GENGA_HELIO;
  if (helio) hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, m, v, nullptr, nullptr, w.n, w.red);
  hipLaunchKernelGGL(k_pack, dim3(ceil_div(w.np, 256)), dim3(256), 0, s, m, x, v, w.red,
                     w.xm, w.vv, w.xs, w.n, w.np, helio, c.m0);
  return hipGetLastError();
}

hipError_t massive_unpack(const MassiveWs& w, const StepConsts& c, double* x,
                          double* v, int coords_out, hipStream_t s) {
  const int helio = coords_out == GENGA_HELIO;
  if (helio)
    hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, nullptr, nullptr, w.xs, w.vv, w.n, w.red);
  hipLaunchKernelGGL(k_unpack, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xs, w.vv, w.red,
                     x, v, w.n, helio, c.m0, (const DevStat*)w.st);
  return hipGetLastError();
}

hipError_t massive_prime(const MassiveWs& w, const StepConsts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_rcrit_init, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xm, w.vv,
                     w.rc_cur, w.thr, w.tmax64, w.ccnt, w.n, c.mu, c.m0, c.n1, c.n2, fabs(c.dt),
                     c.pf2, c.encounter_free);
  PairArgs a = pair_args(w, c);
  hipLaunchKernelGGL(pair_kernel<KICK_INIT>(w), pair_grid(w), pair_block(w), 0, s, a,
                     (const double4*)w.xm, (const double*)w.thr, (const double*)w.tmax64);
  hipLaunchKernelGGL(k_pair_finish<KICK_INIT>, dim3(ceil_div(w.n, kFinThreads)), dim3(kFinThreads),
                     0, s, a, (const double4*)w.xm);
  // the momentum for the first step's first Sun kick
  double* P2 = reinterpret_cast<double*>(reinterpret_cast<char*>(w.st) + offsetof(DevStat, P2));
  hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, nullptr, nullptr, w.xm, w.vv, w.n, P2);
  return hipGetLastError();
}

hipError_t massive_accel(const MassiveWs& w, const StepConsts& c, const double4* x,
                         double* acc, hipStream_t s) {
  PairArgs a = pair_args(w, c);
  a.acc_out = acc;
  hipLaunchKernelGGL(pair_kernel<KICK_ACC>(w), pair_grid(w), pair_block(w), 0, s, a, x,
                     (const double*)w.thr, (const double*)w.tmax64);
  hipLaunchKernelGGL(k_pair_finish<KICK_ACC>, dim3(ceil_div(w.n, kFinThreads)), dim3(kFinThreads),
                     0, s, a, x);
  return hipGetLastError();
}

// Launch of kernel slot `slot` of the step; with kev, through hipExtLaunch so
// that the slot's two events take the dispatch's own start and end.
#define STEP_LAUNCH(slot, K, g, b, ...)                                             \
  do {                                                                              \
    if (kev)                                                                        \
      hipExtLaunchKernelGGL(K, g, b, 0, s, kev[2 * (slot)], kev[2 * (slot) + 1], 0, \
                            __VA_ARGS__);                                           \
    else                                                                            \
      hipLaunchKernelGGL(K, g, b, 0, s, __VA_ARGS__);                               \
  } while (0)

hipError_t massive_step(const MassiveWs& w, const StepConsts& c, hipStream_t s,
                        const hipEvent_t* kev) {
  OpenArgs o;
  o.xs = w.xs;
  o.xm = w.xm;
  o.xstart = w.xstart;
  o.vv = w.vv;
  o.xpre = w.xpre;
  o.vpre = w.vpre;
  o.xpost = w.xpost;
  o.vpost = w.vpost;
  o.afar = w.afar;
  o.rc_next = w.rc_next;
  o.rc_cur = w.rc_cur;
  o.thr = w.thr;
  o.tmax64 = w.tmax64;
  o.ccnt = w.ccnt;
  o.ctab = w.ctab;
  o.partP = w.partP;
  o.partP2 = w.partP2;
  o.khist = w.khist;
  o.st = w.st;
  o.n = w.n;
  o.cpb = w.cpb;
  o.encounter_free = c.encounter_free;
  o.max_iter = c.kepler_max_iter;
  o.G = c.G;
  o.h = c.h;
  o.pf2 = c.pf2;
  o.m0 = c.m0;
  o.mu = c.mu;
  o.dt = c.dt;
  STEP_LAUNCH(0, k_open_drift, dim3(w.nblk), dim3(kOpenBlock), o);

  if (!c.encounter_free) {
    EncArgs e;
    e.xm = w.xm;
    e.vv = w.vv;
    e.xpre = w.xpre;
    e.vpre = w.vpre;
    e.rc = w.rc_cur;
    e.ccnt = w.ccnt;
    e.ctab = w.ctab;
    e.encij = w.encij;
    e.encd2 = w.encd2;
    e.encrc2 = w.encrc2;
    e.goff = w.goff;
    e.gmem = w.gmem;
    e.st = w.st;
    e.n = w.n;
    e.cpb = w.cpb;
    e.enc_cap = w.enc_cap;
    e.dt = c.dt;
    BsArgs b;
    b.xm = w.xm;
    b.vv = w.vv;
    b.dP = w.dP;
    b.xpre = w.xpre;
    b.vpre = w.vpre;
    b.rc = w.rc_cur;
    b.goff = w.goff;
    b.gmem = w.gmem;
    b.big = w.bsbig;
    b.bpos = w.bspos;
    b.bmem = w.bsmem;
    b.rc_w = w.rc_cur;
    b.rad = w.rad;
    b.sp = w.sp;
    b.ids = w.ids;
    b.dead = w.dead;
    b.ev = w.ev;
    b.st = w.st;
    b.G = c.G;
    b.Gm0 = c.mu;
    b.dt = c.dt;
    b.tol = c.bs_tol;
    b.max_depth = c.bs_max_depth;
    b.coll = c.coll;
    b.ev_cap = w.ev_cap;
    const dim3 bs_grid(std::max(1, std::min(256, w.n / 2)));
    if (c.all_pairs) {
      // composed steps (not timed per kernel): every pair tested, then the
      // grouping and BS on their own
      const int nt = ceil_div(w.n, kEncTile);
      hipLaunchKernelGGL(k_encounter_all, dim3(nt, nt), dim3(256), 0, s, e);
      hipLaunchKernelGGL(k_group, dim3(1), dim3(kEncThreads), 0, s, e);
      hipLaunchKernelGGL(k_bs, bs_grid, dim3(64 * kBsWaves), 0, s, b);
    } else {
      STEP_LAUNCH(1, k_encounter, dim3(ceil_div(w.n * w.cpb, kVecBlock)), dim3(kVecBlock), e);
      STEP_LAUNCH(2, k_group_bs, bs_grid, dim3(64 * kBsWaves), e, b);
    }
    if (c.phys) {
      // bodies that merged or crossed rcut / rcut_sun leave (not timed per
      // kernel: the measurement forms run without these limits)
      CompactArgs ca;
      ca.xs = w.xs;
      ca.xm = w.xm;
      ca.vv = w.vv;
      ca.rc = w.rc_cur;
      ca.thr = w.thr;
      ca.tmax64 = w.tmax64;
      ca.rad = w.rad;
      ca.sp = w.sp;
      ca.ids = w.ids;
      ca.dead = w.dead;
      ca.dP = w.dP;
      ca.ev = w.ev;
      ca.st = w.st;
      ca.np = w.np;
      ca.nmin = c.nmin;
      ca.ev_cap = w.ev_cap;
      ca.rcut = c.rcut;
      ca.rcut_sun = c.rcut_sun;
      hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, ca);
    }
  }

  PairArgs a = pair_args(w, c);
  const auto kpair = pair_kernel<KICK_CLOSE>(w);
  STEP_LAUNCH(3, kpair, pair_grid(w), pair_block(w), a,
              (const double4*)w.xm, (const double*)w.thr, (const double*)w.tmax64);
  STEP_LAUNCH(4, k_pair_finish<KICK_CLOSE>, dim3(ceil_div(w.n, kFinThreads)), dim3(kFinThreads), a,
              (const double4*)w.xm);
  return hipGetLastError();
}

hipError_t massive_energy(const MassiveWs& w, const StepConsts& c, double* dE,
                          double* dL, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_rows, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xs, w.vv,
                     w.n, c.G, c.m0, w.red, (const DevStat*)w.st);
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, w.red, w.n, c.m0, dE, dL);
  return hipGetLastError();
}

hipError_t validate_finite(const double* a, int64_t cnt, int* dbad, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, a, cnt, dbad);
  return hipGetLastError();
}

hipError_t thresholds_from_radii(const MassiveWs& w, const StepConsts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_thresholds, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.rc_cur, w.thr,
                     w.tmax64, w.ccnt, w.n, c.pf2, c.encounter_free);
  return hipGetLastError();
}

hipError_t accel_run(const MassiveWs& w, const StepConsts& c, const double* m, const double* x,
                     const double* rc, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(ceil_div(w.np, 256)), dim3(256), 0, s, m, x, x,
                     (const double*)nullptr, w.xm, w.vv, w.xs, w.n, w.np, 0, c.m0);
  hipLaunchKernelGGL(k_radii_in, dim3(ceil_div(w.n, 256)), dim3(256), 0, s,
                     c.encounter_free ? nullptr : rc, w.rc_cur, w.thr, w.tmax64, w.ccnt, w.n, c.pf2,
                     c.encounter_free);
  return massive_accel(w, c, w.xm, acc, s);
}

// ---- the pair kernel with no workspace argument ----------------------------
// Scratch of accel_noalloc_run: the packed bodies (x, y, z, m), the velocity
// and start-position rows the packing kernel also fills, radii, thresholds
// and candidate counts of up to kNoAllocBodies bodies (116 bytes per padded
// body), the 64-body chunks' largest thresholds and the pair kernel's partial sums
// (6 doubles x splits x padded bodies, splits x padded bodies <=
// kPairTargetBig, the pair kernel's shape being the workspace path's): 5.0 MB.  Each GPU holds its own copy until the process ends;
// every call on a GPU uses that GPU's copy, so calls that overlap on one GPU
// race.  Every byte a call reads is written earlier in the same call.
constexpr int kNoAllocBodies = kAccelNoAllocMax;
static_assert(kNoAllocBodies % 256 == 0, "bodies are padded to multiples of 256");
static_assert(kNoAllocBodies <= kPairTarget && kPairTarget <= kPairTargetBig,
              "partial sums sized by kPairTargetBig");
constexpr size_t kNoAllocBytes =
    (size_t)kNoAllocBodies * (3 * sizeof(double4) + 2 * sizeof(double) + sizeof(int)) +
    (size_t)kNoAllocBodies / 64 * sizeof(double) + (size_t)kPairTargetBig * 6 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch, looked up once per
// device.  In host code the array's name is only a host-side stand-in, so
// this address is what every launch and copy uses.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

hipError_t accel_noalloc_run(const StepConsts& c, int n, const double* m, const double* x,
                             const double* rc, double* acc, hipStream_t s) {
  if (n < 1 || n > kNoAllocBodies) return hipErrorInvalidValue;
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  // the arrays the packing, radii and pair kernels of accel_run touch; the
  // pair kernel's accumulation mode reads no other workspace field
  MassiveWs w{};
  w.n = n;
  w.np = ceil_div(n, 256) * 256;
  pair_shape(w.np, &w.pw, &w.njs);  // as the workspace path, so both give the same bits
  w.nblk = ceil_div(n, kOpenBlock);
  const size_t np = (size_t)w.np;
  char* q = static_cast<char*>(base);
  w.xm = reinterpret_cast<double4*>(q);
  q += np * sizeof(double4);
  w.vv = reinterpret_cast<double4*>(q);
  q += np * sizeof(double4);
  w.xs = reinterpret_cast<double4*>(q);
  q += np * sizeof(double4);
  w.rc_cur = reinterpret_cast<double*>(q);
  q += np * sizeof(double);
  w.thr = reinterpret_cast<double*>(q);
  q += np * sizeof(double);
  w.ccnt = reinterpret_cast<int*>(q);
  q += np * sizeof(int);
  w.tmax64 = reinterpret_cast<double*>(q);
  q += np / 64 * sizeof(double);
  w.pp = reinterpret_cast<double*>(q);
  q += (size_t)w.njs * 6 * np * sizeof(double);
  if ((size_t)(q - static_cast<char*>(base)) > kNoAllocBytes) return hipErrorInvalidValue;
  return accel_run(w, c, m, x, rc, acc, s);
}

hipError_t massive_masses(const MassiveWs& w, double* m, hipStream_t s) {
  hipLaunchKernelGGL(k_masses, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xs, m, w.n);
  return hipGetLastError();
}

}  // namespace genga
