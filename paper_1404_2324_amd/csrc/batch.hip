// Batched independent systems (Sec. 3.4): each system has its own central
// mass and 1..64 bodies; systems never interact.  One wave integrates one
// system (or two systems of up to 32 bodies, one per half-wave), one lane
// per body, and runs every requested step inside a single launch with the
// state held in registers (the method's step of Sec. 2.2, as in main mode,
// with each system's own central mass):
//   radii (Eq. 6), opening kick (Eq. 2 gradient, every pair), Sun kick,
//   Kepler drift (Eq. 9), Hermite test of the prechecker's candidates
//   (Eqs. 10-12), groups (connected components, App. A), BS of each group
//   from the pre-drift state (Sec. 3.2.6), Sun kick, closing kick and the
//   next candidates.
// Partner data moves by lane reads (readlane / bpermute / DPP) and through
// LDS, so the only memory traffic of a run is loading and storing the state
// once.  The tuner picks, by timing the real systems, the register budget
// per wave (occupancy), the order in which systems are handed to waves and
// whether small systems share a wave.
#include <algorithm>
#include <climits>
#include <vector>

#include "bs_device.h"
#include "device_math.h"
#include "genga_impl.h"

namespace genga {
namespace {

constexpr size_t kBsRDoubles = (size_t)kBsCols * 6 * 64;  // one sequential-BS tableau

struct BatchArgs {
  double4* __restrict__ xm;                 // [nb] x, y, z, m (democratic)
  double4* __restrict__ vv;                 // [nb] vx, vy, vz, 0
  unsigned long long* __restrict__ cand;    // [nb] candidate partners (local bits)
  unsigned long long* __restrict__ encm;    // [nb] encounters j > i of the last step
  const int* __restrict__ off;              // [nsys + 1]
  const double* __restrict__ m0;            // [nsys]
  const int* __restrict__ order;            // [nsys] systems in hand-out order
  BatchSysStat* __restrict__ ss;            // [nsys]
  unsigned* __restrict__ flags;             // latched error bits
  double* __restrict__ rbuf;                // BS tableaux of groups over 8 members
  const int* __restrict__ rslot;            // [nsys] slice of rbuf (systems over 8 bodies)
  double* __restrict__ rad;                 // [nb] physical radii
  double4* __restrict__ sp;                 // [nb] spins
  int* __restrict__ ids;                    // [nb] original rows
  genga_event* __restrict__ ev;             // mergers and ejections
  unsigned long long* __restrict__ ev_cnt;
  long long ev_cap;
  int nsys, nsteps;
  double G, dt, h, absdt, n1, n2, pf2, tol;
  int max_depth, max_iter, enc_free;
  double rcut, rcut_sun;
  int nmin;
  int coll;    // radii are set: mergers (Sec. 3.2.7)
  int phys;    // coll, or ejection limits, or nmin: bodies can leave
  int record;  // events go to ev (not on the tuner's copies)
};

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// The halves of a double exchanged between rows 2r and 2r + 1 (W = 16) or
// between the two halves of the wave (W = 32); returns the lane's value plus
// its partner's, the pair ordered by row so that both partners hold the same
// bits.
template <int W>
__device__ __forceinline__ double swap_sum(double v) {
  const int2 p = *reinterpret_cast<int2*>(&v);
  int2 lo, hi;
  if (W == 16) {
    const auto a = __builtin_amdgcn_permlane16_swap(p.x, p.x, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(p.y, p.y, false, false);
    lo = make_int2(a[0], b[0]);
    hi = make_int2(a[1], b[1]);
  } else {
    const auto a = __builtin_amdgcn_permlane32_swap(p.x, p.x, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(p.y, p.y, false, false);
    lo = make_int2(a[0], b[0]);
    hi = make_int2(a[1], b[1]);
  }
  return *reinterpret_cast<double*>(&lo) + *reinterpret_cast<double*>(&hi);
}

// Sum over the lanes of one system, on every lane: the butterfly over lane
// distances 1, 2 (DPP quad permutes), 4, 8 (DPP half-row and row mirrors,
// which pair the same partial sums as lane ^ 4 and lane ^ 8 once those are
// uniform over their quad or half-row), 16 (row swap) and, one system per
// wave, 32.  Each step adds the same two partial sums as the xor butterfly,
// so every layout gives the same bits.  Called with the whole wave active.
template <int PK>
__device__ __forceinline__ double sys_sum(double v) {
  v += dpp_d<kDppQuadSwap1>(v);
  v += dpp_d<kDppQuadSwap2>(v);
  v += dpp_d<kDppRowHalfMirror>(v);
  v += dpp_d<kDppRowMirror>(v);
  v = swap_sum<16>(v);
  if (PK == 1) v = swap_sum<32>(v);
  return v;
}

// Integer reductions over the lanes of one system: the whole wave (PK = 1)
// or the lane's half (PK = 2, lanes 0-31 and 32-63 hold two systems).
template <int PK>
__device__ __forceinline__ int sys_max_i(int v) {
  for (int o = 32 / PK; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

template <int PK>
__device__ __forceinline__ int sys_sum_i(int v) {
  for (int o = 32 / PK; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int PK>
__device__ __forceinline__ unsigned sys_or(unsigned v) {
  for (int o = 32 / PK; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Lanes of the half that holds lane l (PK = 2) or the whole wave.
template <int PK>
__device__ __forceinline__ unsigned long long sys_lanes(int l) {
  return PK == 1 ? ~0ull : (0xffffffffull << (l & 32));
}

// LDS slot of lane j in the per-lane tables (the kick's partner tables with
// two systems per wave, the Hermite test's states): the second half is
// offset by one entry so that the two halves' broadcast reads of partner jj
// fall in different banks.
__device__ __forceinline__ int kick_slot(int j) { return j + (j >> 5); }
constexpr int kKickSlots = 66;

// Partner jj of the lane's system: wave-uniform lane reads (PK = 1) or the
// LDS tables (PK = 2).
template <int PK>
__device__ __forceinline__ void kick_partner(int jj, int hb, double x, double y, double z,
                                             double m, double rc, const double4* kp,
                                             const double* krc, double& xj, double& yj,
                                             double& zj, double& mj, double& rcj) {
  if (PK == 1) {
    xj = readlane_d(x, jj);
    yj = readlane_d(y, jj);
    zj = readlane_d(z, jj);
    mj = readlane_d(m, jj);
    rcj = readlane_d(rc, jj);
  } else {
    // kick_slot(hb + jj) = kick_slot(hb) + jj for jj < 32
    const int t = kick_slot(hb) + jj;
    const double4 pj = kp[t];
    xj = pj.x;
    yj = pj.y;
    zj = pj.z;
    mj = pj.w;
    rcj = krc[t];
  }
}

// U consecutive partners jj0 .. jj0 + U - 1 (all below nloop), accumulated
// in index order.  The U pair terms are independent until the accumulation,
// so their latency chains overlap.  The common case K = 1 (dK = 0) is taken
// for every pair first, and the rare pairs inside r_crit,ij are redone with
// the changeover (Eqs. 4-5); mj (K ir^3 - dK ir^2) with K = 1, dK = 0 is
// mj ir^3 exactly, so both paths round as the single formula does.  The
// fused operations are spelled out, so that the roundings do not depend on
// how the partner data arrive (lane reads or LDS).
template <int PK, int U>
__device__ __forceinline__ void kick_chunk(int jj0, int nh, int lane, int hb, double x, double y,
                                           double z, double m, double rc, double pf2,
                                           bool want_cand, const double4* kp, const double* krc,
                                           double& ax, double& ay, double& az,
                                           unsigned long long& cand) {
  double dx[U], dy[U], dz[U], r2[U], ir[U], rcij[U], mj[U], s[U];
  bool ok[U];
  bool near = false;
  // stage by stage over the U pairs, so that the independent chains
  // interleave; the reciprocal square root is the hardware estimate refined
  // by two Newton steps on the halved residual (not the single third-order
  // step of rsqrt_nr, so the last bit can differ from the main-mode kick's)
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const int jj = jj0 + k;
    double xj, yj, zj, rcj;
    kick_partner<PK>(jj, hb, x, y, z, m, rc, kp, krc, xj, yj, zj, mj[k], rcj);
    ok[k] = hb + jj != lane && (PK == 1 || jj < nh);
    dx[k] = xj - x;
    dy[k] = yj - y;
    dz[k] = zj - z;
    rcij[k] = fmax(rc, rcj);
  }
  double hx[U], e[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    r2[k] = fma(dz[k], dz[k], fma(dy[k], dy[k], dx[k] * dx[k]));
    hx[k] = 0.5 * r2[k];
    ir[k] = __builtin_amdgcn_rsq(r2[k]);
  }
#pragma unroll
  for (int k = 0; k < U; ++k) e[k] = fma(-hx[k] * ir[k], ir[k], 0.5);
#pragma unroll
  for (int k = 0; k < U; ++k) ir[k] = fma(ir[k], e[k], ir[k]);
#pragma unroll
  for (int k = 0; k < U; ++k) e[k] = fma(-hx[k] * ir[k], ir[k], 0.5);
#pragma unroll
  for (int k = 0; k < U; ++k) ir[k] = fma(ir[k], e[k], ir[k]);
#pragma unroll
  for (int k = 0; k < U; ++k) {
    s[k] = mj[k] * ((ir[k] * ir[k]) * ir[k]);
    near = near || (ok[k] && r2[k] * ir[k] < rcij[k]);
  }
  if (near) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const double r = r2[k] * ir[k];
      if (ok[k] && r < rcij[k]) {
        double K, dK;
        changeover(r, rcij[k], K, dK);
        const double ir2 = ir[k] * ir[k];
        s[k] = mj[k] * fma(K * ir2, ir[k], -(dK * ir2));
      }
    }
  }
  // accumulated without branches: a pair that does not count adds 0 * dx
  // (its own lane: dx = 0; a partner slot past the system: finite dx); the
  // chunk's candidate bits gather in a small mask placed once
  unsigned cb = 0u;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const double sk = ok[k] ? s[k] : 0.0;
    ax = fma(sk, dx[k], ax);
    ay = fma(sk, dy[k], ay);
    az = fma(sk, dz[k], az);
    if (want_cand) cb |= (ok[k] && r2[k] < pf2 * rcij[k] * rcij[k]) ? (1u << k) : 0u;
  }
  if (want_cand) cand |= (unsigned long long)cb << (hb + jj0);
}

// Pair acceleration of H_B (Eq. 2 gradient) on the lane's body from every
// other body of the system; with want_cand, also the partners inside the
// prechecker radius pf r_crit,ij (Sec. 2.2), as bits of lane indices.
// rc = 0 everywhere gives the Newtonian pair sum (K = 1, the encounter-free
// map).  The system occupies lanes hb .. hb + nh - 1; partners are visited
// in index order jj = 0 .. nh - 1 whatever PK, so both layouts give the same
// sums.  One system per wave reads the partner by wave-uniform lane reads;
// two systems per wave (nloop = the larger size, kp / krc: LDS tables of
// kKickSlots entries) read it from LDS, where each half's lanes all read one
// address.
template <int PK>
__device__ __forceinline__ void sys_kick(int nloop, int nh, int lane, int hb, double x, double y,
                                         double z, double m, double rc, double G, double pf2,
                                         bool want_cand, double& ax, double& ay, double& az,
                                         unsigned long long& cand, double4* kp, double* krc) {
  ax = ay = az = 0.0;
  cand = 0ull;
  if (PK == 2) {
    __syncthreads();  // earlier reads of the tables are done
    kp[kick_slot(lane)] = make_double4(x, y, z, m);
    krc[kick_slot(lane)] = rc;
    __syncthreads();
  }
  int jj = 0;
  for (; jj + 8 <= nloop; jj += 8)
    kick_chunk<PK, 8>(jj, nh, lane, hb, x, y, z, m, rc, pf2, want_cand, kp, krc, ax, ay, az,
                      cand);
  if (jj + 4 <= nloop) {
    kick_chunk<PK, 4>(jj, nh, lane, hb, x, y, z, m, rc, pf2, want_cand, kp, krc, ax, ay, az,
                      cand);
    jj += 4;
  }
  for (; jj < nloop; ++jj)
    kick_chunk<PK, 1>(jj, nh, lane, hb, x, y, z, m, rc, pf2, want_cand, kp, krc, ax, ay, az,
                      cand);
  ax *= G;
  ay *= G;
  az *= G;
}

// The b-th lowest set bit of M (b < popc(M)).
__device__ __forceinline__ int nth_bit(unsigned long long M, int b) {
  for (int t = 0; t < b; ++t) M &= M - 1ull;
  return __ffsll((long long)M) - 1;
}

// One group of sz <= 8 members (mask M) with the column-parallel BS; mm and
// mrc are this wave's LDS arrays.  Returns the BS status; on return every
// member lane's pre-drift state pre[] has been replaced by its result.
template <int P>
__device__ __forceinline__ int group_par(const BatchArgs& a, int sz, unsigned long long M,
                                         double pre[6], double m, double rc, double Gm0,
                                         double* mm, double* mrc, long long* nsub, double H,
                                         double R, double* mR, int* ckey, long long* cpos) {
  const int lane = threadIdx.x & 63;
  const int b = par_memb<P>(lane);
  const int body = b < sz ? nth_bit(M, b) : 0;
  double y[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) y[c] = __shfl(pre[c], body, 64);
  if (b >= sz) {
    y[0] = 1.0;
    y[1] = y[2] = y[3] = y[4] = y[5] = 0.0;
  }
  // member tables indexed by member: lane t < sz fetches member t's data
  const int bt = lane < sz ? nth_bit(M, lane) : 0;
  const double mb = __shfl(m, bt, 64), rcb = __shfl(rc, bt, 64), Rbt = __shfl(R, bt, 64);
  __syncthreads();
  if (lane < sz) {
    mm[lane] = mb;
    mrc[lane] = rcb;
    if (mR) mR[lane] = Rbt;
  }
  __syncthreads();
  const int r = bs_group<P, false>(sz, y, mm, mrc, H, a.G, Gm0, a.tol, a.max_depth, nsub, -1.0,
                                   ckey, cpos, mR);
  const int rank = __popcll(M & ((1ull << lane) - 1ull));
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double t = __shfl(y[c], par_lane<P>(0, 0, min(rank, P - 1)), 64);
    if ((M >> lane) & 1ull) pre[c] = t;
  }
  return r;
}

// Groups of 9..64 members: lane = member, the sequential BS with its
// extrapolation tableau in this system's slice R of the workspace.
__device__ __forceinline__ int group_seq(const BatchArgs& a, int sz, unsigned long long M,
                                         double pre[6], double m, double rc, double Gm0,
                                         double (*R)[6][64], long long* nsub, double H,
                                         double Rad, bool coll, int* ckey, long long* cpos) {
  const int lane = threadIdx.x & 63;
  const int body = lane < sz ? nth_bit(M, lane) : 0;
  double y[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) y[c] = __shfl(pre[c], body, 64);
  double mb = __shfl(m, body, 64), rcb = __shfl(rc, body, 64), Rb = __shfl(Rad, body, 64);
  if (lane >= sz) {
    y[0] = 1.0;
    y[1] = y[2] = y[3] = y[4] = y[5] = 0.0;
    mb = 0.0;
    rcb = 0.0;
    Rb = 0.0;
  }
  const int r = bs_integrate(sz, lane, y, H, mb, rcb, a.G, Gm0, a.tol, a.max_depth, R, nsub, Rb,
                             coll ? ckey : nullptr, cpos);
  const int rank = __popcll(M & ((1ull << lane) - 1ull));
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const double t = __shfl(y[c], rank, 64);
    if ((M >> lane) & 1ull) pre[c] = t;
  }
  return r;
}

// Event record of a merger or an ejection, written by one lane.
__device__ __forceinline__ void put_event(const BatchArgs& a, int kind, int sys, int idi, int idj,
                                          long long step, double frac, double mi, double mj,
                                          double Ri, double Rj, const double* yi,
                                          const double* si, const double* yj, const double* sj,
                                          double U) {
  if (!a.record) return;
  const unsigned long long k = atomicAdd(a.ev_cnt, 1ull);
  if ((long long)k >= a.ev_cap) return;
  genga_event e;
  e.kind = kind;
  e.sys = sys;
  e.id_i = idi;
  e.id_j = idj;
  e.step = step;
  e.frac = frac;
  e.m_i = mi;
  e.m_j = mj;
  e.R_i = Ri;
  e.R_j = Rj;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    e.x_i[q] = yi[q];
    e.v_i[q] = yi[3 + q];
    e.s_i[q] = si[q];
    e.x_j[q] = yj ? yj[q] : 0.0;
    e.v_j[q] = yj ? yj[3 + q] : 0.0;
    e.s_j[q] = sj ? sj[q] : 0.0;
  }
  e.U = U;
  a.ev[k] = e;
}

// PK systems per wave: one (lanes 0..63 for up to 64 bodies) or two (lanes
// 0-31 and 32-63, systems of up to 32 bodies, so that small systems fill the
// wave).  Every per-system quantity is a per-lane value uniform over the
// system's lanes; the wave runs the step while either of its systems is
// live, a stopped system's lanes keeping their state.  Both layouts do the
// same arithmetic in the same order on each system.
// With radii, limits or nmin (a.phys), bodies leave as in the paper's
// multi-simulation mode (Sec. 3.2.7, 3.2.8, 3.4.6): a group's BS stops at
// the substep in which two members touch, they merge, and the group goes on
// over the rest of the step; after the groups, bodies beyond rcut or inside
// rcut_sun leave; every freed lane takes the system's last body (freed lanes
// in descending order) and the system's count drops; below nmin bodies the
// system stops.  The step's encounter bits stay with the lanes they were
// found on (the rows before the removal).
template <int LB, int PK, bool PH>
__global__ __launch_bounds__(64, LB) void k_batch(BatchArgs a) {
  __shared__ double mm[kBsPar], mrc[kBsPar], mR[kBsPar];
  __shared__ double4 kp[PK == 2 ? kKickSlots : 1];
  __shared__ double krc[PK == 2 ? kKickSlots : 1];
  __shared__ double hs[13][kKickSlots];  // pre-drift state, drifted state, radius
  __shared__ unsigned kh[PK][kKepBins];  // each system's drifts by iteration count
  const int lane = threadIdx.x;
  if (lane < PK * kKepBins) kh[lane / kKepBins][lane % kKepBins] = 0u;
  __syncthreads();
  const int hb = PK == 1 ? 0 : (lane & 32);  // first lane of the lane's system
  const int hl = lane - hb;                  // the body's index in its system
  const int si = PK * blockIdx.x + (PK == 1 ? 0 : (lane >> 5));
  const bool has = si < a.nsys;
  const int s = has ? a.order[si] : 0;
  const int o = has ? a.off[s] : 0;
  const int ncap = has ? a.off[s + 1] - o : 0;  // the system's rows
  int n = has ? a.ss[s].nlive : 0;              // bodies still in it
  auto loop_n = [&](int nn) {
    return PK == 1 ? nn : max(__builtin_amdgcn_readlane(nn, 0), __builtin_amdgcn_readlane(nn, 32));
  };
  int nloop = loop_n(n);
  bool act = hl < n;
  const double m0 = has ? a.m0[s] : 1.0;
  const double Gm0 = a.G * m0;
  // inactive lanes hold a massless dummy body far from the others
  double4 p = make_double4(1.0e3 + lane, 0.0, 0.0, 0.0);
  double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
  unsigned long long cand = 0ull, enc = 0ull, enc_last = 0ull;
  double R = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0;
  int id = 0;
  if (act) {
    p = a.xm[o + hl];
    q = a.vv[o + hl];
    cand = a.cand[o + hl] << hb;  // stored as bits of indices in the system
    if (PH) {
      R = a.rad[o + hl];
      const double4 t = a.sp[o + hl];
      S0 = t.x;
      S1 = t.y;
      S2 = t.z;
      id = a.ids[o + hl];
    }
  }
  double x = p.x, y = p.y, z = p.z, vx = q.x, vy = q.y, vz = q.z;
  double m = p.w;
  long long nsub = 0;
  unsigned long long enc_total = 0;
  int kit = 0, nenc = 0, ngrp = 0, maxg = 0;
  unsigned fl = 0u;
  double Usys = 0.0;
  const long long step0 = has ? a.ss[s].steps : 0;
  // a system stopped by an earlier failure takes no more steps
  const bool stopped = !has || (a.ss[s].flags & (F_KEPLER | F_BS | F_NMIN)) != 0u;
  bool live = !stopped;
  int done = 0;
  for (int step = 0; step < a.nsteps; ++step) {
    if (__ballot(live) == 0ull) break;
    const bool live0 = live;
    const bool actv = act && live0;
    // the step-start state is restored if the step fails (with the bodies a
    // merger or an ejection removed in it)
    const double sx = x, sy = y, sz0 = z, svx = vx, svy = vy, svz = vz;
    const unsigned long long scand = cand;
    const double sm = m, sR = R, sS0 = S0, sS1 = S1, sS2 = S2, sU = Usys;
    const int sid = id, sn = n;
    (void)sm, (void)sR, (void)sS0, (void)sS1, (void)sS2, (void)sU, (void)sid, (void)sn;
    const double rc =
        actv && !a.enc_free ? rcrit(x, y, z, vx, vy, vz, m, Gm0, m0, a.n1, a.n2, a.absdt) : 0.0;
    double ax, ay, az;
    unsigned long long dummy;
    sys_kick<PK>(nloop, n, lane, hb, x, y, z, m, rc, a.G, a.pf2, false, ax, ay, az, dummy, kp,
                 krc);
    vx += a.h * ax;
    vy += a.h * ay;
    vz += a.h * az;
    const double P1x = sys_sum<PK>(m * vx), P1y = sys_sum<PK>(m * vy),
                 P1z = sys_sum<PK>(m * vz);
    x += a.h * P1x / m0;
    y += a.h * P1y / m0;
    z += a.h * P1z / m0;
    double pre[6] = {x, y, z, vx, vy, vz};
    if (actv) {
      const int it = kepler_drift(Gm0, a.dt, x, y, z, vx, vy, vz, a.max_iter);
      if (it < 0) fl |= F_KEPLER;
      kit = max(kit, abs(it));
      atomicAdd(&kh[PK == 1 ? 0 : (lane >> 5)][min(abs(it), kKepBins - 1)], 1u);
    }
    // Hermite test of the candidate pairs i < j (Eqs. 10-12)
    enc = 0ull;
    const unsigned long long above = lane < 63 ? ~((2ull << lane) - 1ull) : 0ull;
    const unsigned long long mine = actv && !a.enc_free ? (cand & above) : 0ull;
    // Each lane walks its own candidates, reading the partner's states from
    // LDS, so a pass serves one candidate of every lane (not one partner of
    // the whole wave)
    if (__ballot(mine != 0ull) != 0ull) {
      __syncthreads();  // earlier reads of the table are done
      const int t = kick_slot(lane);
#pragma unroll
      for (int c = 0; c < 6; ++c) hs[c][t] = pre[c];
      hs[6][t] = x;
      hs[7][t] = y;
      hs[8][t] = z;
      hs[9][t] = vx;
      hs[10][t] = vy;
      hs[11][t] = vz;
      hs[12][t] = rc;
      __syncthreads();
      unsigned long long mc = mine;
      while (__ballot(mc != 0ull) != 0ull) {
        if (mc) {
          const int j = __ffsll((long long)mc) - 1;
          mc &= mc - 1ull;
          const int tj = kick_slot(j);
          const double d2 = hermite_dmin2(
              a.dt, hs[0][tj] - pre[0], hs[1][tj] - pre[1], hs[2][tj] - pre[2],
              hs[3][tj] - pre[3], hs[4][tj] - pre[4], hs[5][tj] - pre[5], hs[6][tj] - x,
              hs[7][tj] - y, hs[8][tj] - z, hs[9][tj] - vx, hs[10][tj] - vy, hs[11][tj] - vz);
          const double rcij = fmax(rc, hs[12][tj]);
          if (d2 < rcij * rcij) enc |= 1ull << j;
        }
      }
    }
    const int ne = sys_sum_i<PK>(__popcll(enc));
    const int ne_w =
        PK == 1 ? ne : __builtin_amdgcn_readlane(ne, 0) + __builtin_amdgcn_readlane(ne, 32);
    int sgrp = 0, smaxg = 0;
    bool dead = false;
    double rcl = rc;  // a merged body keeps the larger radius for the step
    if (ne_w > 0) {
      // symmetric adjacency, then minimum-label components (App. A)
      unsigned long long adj = enc;
      unsigned long long rows = __ballot(enc != 0ull);
      while (rows) {
        const int i2 = __ffsll((long long)rows) - 1;
        rows &= rows - 1ull;
        const unsigned long long ei = readlane_u64(enc, i2);
        if ((ei >> lane) & 1ull) adj |= 1ull << i2;
      }
      const unsigned long long U = __ballot(adj != 0ull);  // lanes in some pair
      int lab = lane;
      bool changed = true;
      while (changed) {
        int nl = lab;
        if (PK == 1) {
          for (int j = 0; j < n; ++j) {
            const int lj = __builtin_amdgcn_readlane(lab, j);
            if (((adj >> j) & 1ull) && lj < nl) nl = lj;
          }
        } else {
          for (unsigned long long u = U; u; u &= u - 1ull) {
            const int j = __ffsll((long long)u) - 1;
            const int lj = __builtin_amdgcn_readlane(lab, j);
            if (((adj >> j) & 1ull) && lj < nl) nl = lj;
          }
        }
        changed = __ballot(nl != lab) != 0ull;
        lab = nl;
      }
      const bool ing = actv && adj != 0ull;
      unsigned long long roots = __ballot(ing && lab == lane);
      while (roots) {
        const int r = __ffsll((long long)roots) - 1;
        roots &= roots - 1ull;
        unsigned long long M = __ballot(ing && lab == r);
        int sz = __popcll(M);
        // the group belongs to the system of lane r
        const bool own = PK == 1 || ((lane ^ r) & 32) == 0;
        const double Gm0g = PK == 1 ? Gm0 : readlane_d(Gm0, r);
        const int sg = PK == 1 ? s : __builtin_amdgcn_readlane(s, r);
        if (own) {
          ++sgrp;
          smaxg = max(smaxg, sz);
        }
        double H = a.dt, f0 = 0.0;
        for (;;) {
          long long gsub = 0, cpos = 0;
          int key = -1, st;
          double* mRp = PH && a.coll ? mR : nullptr;
          if (sz <= 2)
            st = group_par<2>(a, sz, M, pre, m, rcl, Gm0g, mm, mrc, &gsub, H, R, mRp, &key, &cpos);
          else if (sz <= 4)
            st = group_par<4>(a, sz, M, pre, m, rcl, Gm0g, mm, mrc, &gsub, H, R, mRp, &key, &cpos);
          else if (sz <= kBsPar)
            st = group_par<8>(a, sz, M, pre, m, rcl, Gm0g, mm, mrc, &gsub, H, R, mRp, &key, &cpos);
          else
            st = group_seq(a, sz, M, pre, m, rcl, Gm0g,
                           reinterpret_cast<double(*)[6][64]>(a.rbuf + (size_t)a.rslot[sg] * kBsRDoubles),
                           &gsub, H, R, PH && a.coll != 0, &key, &cpos);
          if (own) nsub += gsub;
          if (!PH || st != 1) {
            if (st != 0 && own) fl |= F_BS;
            break;
          }
          // two members touch: merge them at the start of that substep and
          // integrate the group, one member fewer, over the rest of the step
          const double fc = ldexp((double)cpos, -a.max_depth);
          const int la = nth_bit(M, key >> 6), lb = nth_bit(M, key & 63);
          const double mla = readlane_d(m, la), mlb = readlane_d(m, lb);
          const int ls = mlb > mla ? lb : la, lg = ls == la ? lb : la;
          double ys[6], yg[6], ss[3], sgv[3], ym[6], sm[3], Mm, Rm;
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            ys[c] = readlane_d(pre[c], ls);
            yg[c] = readlane_d(pre[c], lg);
          }
          ss[0] = readlane_d(S0, ls);
          ss[1] = readlane_d(S1, ls);
          ss[2] = readlane_d(S2, ls);
          sgv[0] = readlane_d(S0, lg);
          sgv[1] = readlane_d(S1, lg);
          sgv[2] = readlane_d(S2, lg);
          const double ms = readlane_d(m, ls), mg = readlane_d(m, lg);
          const double Rs = readlane_d(R, ls), Rg = readlane_d(R, lg);
          const double Uc = merge_bodies(a.G, ms, mg, ys, yg, Rs, Rg, ss, sgv, Mm, ym, Rm, sm);
          const double frac = f0 + (1.0 - f0) * fc;
          // read in converged control flow: inside the branch below lane lg
          // is inactive, and a register's value in an inactive lane need not
          // survive register allocation there
          const int idg = __builtin_amdgcn_readlane(id, lg);
          if (lane == ls)
            put_event(a, GENGA_EV_MERGE, sg, id, idg, step0 + step, frac, ms, mg, Rs, Rg, ys, ss,
                      yg, sgv, Uc);
          if (own) Usys += Uc;
          const double rcm = fmax(readlane_d(rcl, ls), readlane_d(rcl, lg));
          if (lane == ls) {
#pragma unroll
            for (int c = 0; c < 6; ++c) pre[c] = ym[c];
            m = Mm;
            R = Rm;
            S0 = sm[0];
            S1 = sm[1];
            S2 = sm[2];
            rcl = rcm;
          }
          if (lane == lg) dead = true;
          M &= ~(1ull << lg);
          --sz;
          H = H * (1.0 - fc);
          f0 = frac;
        }
      }
      if (ing) {
        x = pre[0];
        y = pre[1];
        z = pre[2];
        vx = pre[3];
        vy = pre[4];
        vz = pre[5];
      }
    }
    if (PH) {
      // ejections (Sec. 3.2.8) of the bodies still present
      if (actv && !dead && (a.rcut > 0.0 || a.rcut_sun > 0.0)) {
        const double r = sqrt(x * x + y * y + z * z);
        int kind = 0;
        if (a.rcut > 0.0 && r > a.rcut) kind = GENGA_EV_EJECT_FAR;
        if (a.rcut_sun > 0.0 && r < a.rcut_sun) kind = GENGA_EV_EJECT_SUN;
        if (kind) {
          const double yv[6] = {x, y, z, vx, vy, vz}, sv[3] = {S0, S1, S2};
          put_event(a, kind, s, id, -1, step0 + step, 1.0, m, 0.0, R, 0.0, yv, sv, nullptr,
                    nullptr, 0.0);
          dead = true;
        }
      }
      // the freed lanes take the last bodies (highest freed lane first)
      while (true) {
        const unsigned long long dm = __ballot(dead && act) & sys_lanes<PK>(lane);
        if (__ballot(dm != 0ull) == 0ull) break;
        int src = lane;
        if (dm != 0ull) {
          const int hgh = 63 - __builtin_clzll(dm);
          const int last = hb + n - 1;
          if (lane == hgh) src = last;
          --n;  // uniform over the half
        }
        x = __shfl(x, src, 64);
        y = __shfl(y, src, 64);
        z = __shfl(z, src, 64);
        vx = __shfl(vx, src, 64);
        vy = __shfl(vy, src, 64);
        vz = __shfl(vz, src, 64);
        m = __shfl(m, src, 64);
        R = __shfl(R, src, 64);
        S0 = __shfl(S0, src, 64);
        S1 = __shfl(S1, src, 64);
        S2 = __shfl(S2, src, 64);
        rcl = __shfl(rcl, src, 64);
        id = __shfl(id, src, 64);
        dead = __shfl((int)dead, src, 64) != 0;
        act = hl < n;
        if (!act) dead = false;
      }
      nloop = loop_n(n);
      if (!act) {
        // a lane past the system's count holds a massless dummy body
        x = 1.0e3 + lane;
        y = z = vx = vy = vz = 0.0;
        m = 0.0;
        R = 0.0;
        rcl = 0.0;
      }
    }
    const double P2x = sys_sum<PK>(m * vx), P2y = sys_sum<PK>(m * vy),
                 P2z = sys_sum<PK>(m * vz);
    x += a.h * P2x / m0;
    y += a.h * P2y / m0;
    z += a.h * P2z / m0;
    sys_kick<PK>(nloop, n, lane, hb, x, y, z, m, rcl, a.G, a.pf2, !a.enc_free, ax, ay, az, cand,
                 kp, krc);
    vx += a.h * ax;
    vy += a.h * ay;
    vz += a.h * az;
    // a failing system stops here (the paper's multi-simulation mode stops
    // systems individually), keeping its last good state; a system stopped
    // earlier keeps its state through the steps its partner half still takes
    const bool fail = (__ballot(fl != 0u) & sys_lanes<PK>(lane)) != 0ull;
    if (!live0 || fail) {
      x = sx;
      y = sy;
      z = sz0;
      vx = svx;
      vy = svy;
      vz = svz;
      cand = scand;
      if (PH) {
        m = sm;
        R = sR;
        S0 = sS0;
        S1 = sS1;
        S2 = sS2;
        id = sid;
        n = sn;
        Usys = sU;
        act = hl < n;
        nloop = loop_n(n);
      }
    }
    if (live0) {
      enc_last = enc;
      enc_total += (unsigned long long)ne;
      nenc = ne;
      ngrp = sgrp;
      maxg = smaxg;
      if (fail) {
        live = false;
      } else {
        ++done;
        if (PH && a.nmin > 0 && n < a.nmin) {
          fl |= F_NMIN;  // fewer than nmin bodies: the system stops (Sec. 3.4.6)
          live = false;
        }
      }
    }
  }
  if (act && !stopped) {
    a.xm[o + hl] = make_double4(x, y, z, m);
    a.vv[o + hl] = make_double4(vx, vy, vz, 0.0);
    a.cand[o + hl] = cand >> hb;
    if (PH) {
      a.sp[o + hl] = make_double4(S0, S1, S2, 0.0);
      a.ids[o + hl] = id;
      a.rad[o + hl] = R;
    }
  }
  // every row of the system: in a step that removed bodies the encounter
  // bits stay on the rows they were found on
  if (hl < ncap && !stopped && a.nsteps > 0) a.encm[o + hl] = enc_last >> hb;
  const unsigned fall = sys_or<PK>(fl);
  const int kitw = sys_max_i<PK>(kit);
  __syncthreads();  // the histogram's LDS atomics are complete
  if (hl < kKepBins && a.nsteps > 0 && !stopped)
    a.ss[s].khist[hl] += kh[PK == 1 ? 0 : (lane >> 5)][hl];
  if (hl == 0 && a.nsteps > 0 && !stopped) {
    BatchSysStat& t = a.ss[s];
    t.steps += done;
    t.sub += (unsigned long long)nsub;
    t.enc_total += enc_total;
    t.nenc = nenc;
    t.ngroups = ngrp;
    t.maxg = maxg;
    t.kit = max(t.kit, kitw);
    t.nlive = n;
    t.U += Usys;
    if (fall) {
      t.flags |= fall;
      atomicOr(a.flags, F_SYS_STOP);
    }
  }
}

// ---- state conversion, first candidates, energy: one wave per system ------
__global__ __launch_bounds__(64) void k_batch_pack(const double* __restrict__ m,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ v,
                                                   const int* __restrict__ off,
                                                   const double* __restrict__ m0s,
                                                   double4* __restrict__ xm,
                                                   double4* __restrict__ vv, int helio,
                                                   int keep_mass) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int o = off[s], n = off[s + 1] - o;
  const bool act = lane < n;
  double mi = 0.0, ux = 0.0, uy = 0.0, uz = 0.0;
  if (act) {
    mi = keep_mass ? xm[o + lane].w : m[o + lane];
    ux = v[3 * (o + lane)];
    uy = v[3 * (o + lane) + 1];
    uz = v[3 * (o + lane) + 2];
  }
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    // heliocentric u -> barycentric v = u - sum m u / (m0 + sum m)
    const double M = wave_sum(mi);
    const double den = m0s[s] + M;
    sx = wave_sum(mi * ux) / den;
    sy = wave_sum(mi * uy) / den;
    sz = wave_sum(mi * uz) / den;
  }
  if (act) {
    xm[o + lane] = make_double4(x[3 * (o + lane)], x[3 * (o + lane) + 1], x[3 * (o + lane) + 2], mi);
    vv[o + lane] = make_double4(ux - sx, uy - sy, uz - sz, 0.0);
  }
}

// Rows past a system's live count (bodies that merged or left) are NaN.
__global__ __launch_bounds__(64) void k_batch_unpack(const double4* __restrict__ xm,
                                                     const double4* __restrict__ vv,
                                                     const int* __restrict__ off,
                                                     const double* __restrict__ m0s,
                                                     const BatchSysStat* __restrict__ ss,
                                                     double* __restrict__ x,
                                                     double* __restrict__ v, int helio) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int o = off[s], ncap = off[s + 1] - o, n = ss[s].nlive;
  const bool act = lane < n;
  if (lane >= n && lane < ncap) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int q = 0; q < 3; ++q) x[3 * (o + lane) + q] = v[3 * (o + lane) + q] = nan;
  }
  double4 p = make_double4(0.0, 0.0, 0.0, 0.0), q = p;
  if (act) {
    p = xm[o + lane];
    q = vv[o + lane];
  }
  double sx = 0.0, sy = 0.0, sz = 0.0;
  if (helio) {
    // barycentric v -> heliocentric u = v + sum m v / m0
    sx = wave_sum(p.w * q.x) / m0s[s];
    sy = wave_sum(p.w * q.y) / m0s[s];
    sz = wave_sum(p.w * q.z) / m0s[s];
  }
  if (act) {
    x[3 * (o + lane)] = p.x;
    x[3 * (o + lane) + 1] = p.y;
    x[3 * (o + lane) + 2] = p.z;
    v[3 * (o + lane)] = q.x + sx;
    v[3 * (o + lane) + 1] = q.y + sy;
    v[3 * (o + lane) + 2] = q.z + sz;
  }
}

// Candidates entering the first step: radii of the initial state and the
// prechecker on the initial positions (Sec. 2.2).
__global__ __launch_bounds__(64) void k_batch_prime(BatchArgs a) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int o = a.off[s], n = a.ss[s].nlive;
  const bool act = lane < n;
  const double m0 = a.m0[s];
  double4 p = make_double4(1.0e3 + lane, 0.0, 0.0, 0.0), q = make_double4(0.0, 0.0, 0.0, 0.0);
  if (act) {
    p = a.xm[o + lane];
    q = a.vv[o + lane];
  }
  const double rc = act && !a.enc_free
                        ? rcrit(p.x, p.y, p.z, q.x, q.y, q.z, p.w, a.G * m0, m0, a.n1, a.n2, a.absdt)
                        : 0.0;
  double ax, ay, az;
  unsigned long long cand;
  sys_kick<1>(n, n, lane, 0, p.x, p.y, p.z, p.w, rc, a.G, a.pf2, !a.enc_free, ax, ay, az, cand,
              nullptr, nullptr);
  if (act) {
    a.cand[o + lane] = cand;
    a.encm[o + lane] = 0ull;
  }
}

// E = sum m v^2/2 + |P|^2/2m0 - sum G m0 m/r - sum_{i<j} G m_i m_j/r_ij and
// L = sum m x x v of each system (Eqs. 1-3).
__global__ __launch_bounds__(64) void k_batch_energy(const double4* __restrict__ xm,
                                                     const double4* __restrict__ vv,
                                                     const int* __restrict__ off,
                                                     const double* __restrict__ m0s,
                                                     const BatchSysStat* __restrict__ ss, double G,
                                                     double* __restrict__ E,
                                                     double* __restrict__ L) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int o = off[s], n = ss[s].nlive;
  const bool act = lane < n;
  double4 p = make_double4(1.0e3 + lane, 0.0, 0.0, 0.0), q = make_double4(0.0, 0.0, 0.0, 0.0);
  if (act) {
    p = xm[o + lane];
    q = vv[o + lane];
  }
  const double m0 = m0s[s];
  double kin = 0.0, pot = 0.0;
  if (act) {
    kin = 0.5 * p.w * (q.x * q.x + q.y * q.y + q.z * q.z);
    pot = -G * m0 * p.w / sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  }
  for (int j = 0; j < n; ++j) {
    const double xj = readlane_d(p.x, j), yj = readlane_d(p.y, j), zj = readlane_d(p.z, j);
    const double mj = readlane_d(p.w, j);
    if (act && j > lane) {
      const double dx = xj - p.x, dy = yj - p.y, dz = zj - p.z;
      pot -= G * p.w * mj / sqrt(dx * dx + dy * dy + dz * dz);
    }
  }
  const double Px = wave_sum(p.w * q.x), Py = wave_sum(p.w * q.y), Pz = wave_sum(p.w * q.z);
  const double e = wave_sum(kin + pot) + (Px * Px + Py * Py + Pz * Pz) / (2.0 * m0);
  const double lx = wave_sum(p.w * (p.y * q.z - p.z * q.y));
  const double ly = wave_sum(p.w * (p.z * q.x - p.x * q.z));
  const double lz = wave_sum(p.w * (p.x * q.y - p.y * q.x));
  if (lane == 0) {
    E[s] = e;
    L[3 * s] = lx;
    L[3 * s + 1] = ly;
    L[3 * s + 2] = lz;
  }
}

// Every system's bodies present, rows as given (init).
__global__ __launch_bounds__(64) void k_batch_reset(const int* __restrict__ off,
                                                    BatchSysStat* __restrict__ ss,
                                                    int* __restrict__ ids, double4* __restrict__ sp,
                                                    double* __restrict__ rad) {
  const int s = blockIdx.x, lane = threadIdx.x;
  const int o = off[s], n = off[s + 1] - o;
  if (lane < n) {
    ids[o + lane] = o + lane;
    sp[o + lane] = make_double4(0.0, 0.0, 0.0, 0.0);
    rad[o + lane] = 0.0;
  }
  if (lane == 0) ss[s].nlive = n;
}

BatchArgs batch_args(const BatchWs& b, const StepConsts& c, bool scratch, int variant_order) {
  BatchArgs a;
  a.xm = scratch ? b.xm2 : b.xm;
  a.vv = scratch ? b.vv2 : b.vv;
  a.cand = scratch ? b.cand2 : b.cand;
  a.encm = scratch ? b.encm2 : b.encm;
  a.off = b.off;
  a.m0 = b.m0;
  a.order = variant_order ? b.order_desc : b.order_nat;
  a.ss = scratch ? b.ss2 : b.ss;
  a.rbuf = b.rbuf;
  a.rslot = b.rslot;
  a.rad = scratch ? b.rad2 : b.rad;
  a.sp = scratch ? b.sp2 : b.sp;
  a.ids = scratch ? b.ids2 : b.ids;
  a.ev = b.ev;
  a.ev_cnt = b.ev_cnt;
  a.ev_cap = b.nb;
  a.record = scratch ? 0 : 1;
  a.coll = b.coll;
  a.rcut = b.rcut;
  a.rcut_sun = b.rcut_sun;
  a.nmin = b.nmin;
  a.phys = b.coll || b.rcut > 0.0 || b.rcut_sun > 0.0 || b.nmin > 0;
  a.flags = scratch ? b.flags2 : &b.st->flags;
  a.nsys = b.nsys;
  a.nsteps = 0;
  a.G = c.G;
  a.dt = c.dt;
  a.h = c.h;
  a.absdt = fabs(c.dt);
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.pf2 = c.pf2;
  a.tol = c.bs_tol;
  a.max_depth = c.bs_max_depth;
  a.max_iter = c.kepler_max_iter;
  a.enc_free = c.encounter_free;
  return a;
}

}  // namespace

const char* batch_variant_name(int v) {
  static const char* names[kBatchVariants] = {
      "1 wave/SIMD, natural order",  "1 wave/SIMD, largest first",
      "2 waves/SIMD, natural order", "2 waves/SIMD, largest first",
      "4 waves/SIMD, natural order", "4 waves/SIMD, largest first",
      "2 systems/wave, 1 wave/SIMD, largest first",
      "2 systems/wave, 2 waves/SIMD, largest first",
      "2 systems/wave, 4 waves/SIMD, largest first"};
  return v >= 0 && v < kBatchVariants ? names[v] : "?";
}

bool batch_variant_ok(const BatchWs& b, int v) {
  return v >= 0 && v < kBatchVariants && (v < kBatchPackedVariant0 || b.maxn <= 32);
}

size_t batch_carve(BatchWs& b, int nsys, int64_t nb, int nbig, void* base) {
  b.nsys = nsys;
  b.nb = nb;
  b.nbig = nbig;
  size_t off = 0;
  auto take = [&](size_t sz) -> void* {
    const size_t o = off;
    off += (sz + 255) & ~size_t(255);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const size_t n = (size_t)std::max<int64_t>(nb, 1), ns = (size_t)nsys;
  b.xm = (double4*)take(n * sizeof(double4));
  b.vv = (double4*)take(n * sizeof(double4));
  b.cand = (unsigned long long*)take(n * sizeof(unsigned long long));
  b.encm = (unsigned long long*)take(n * sizeof(unsigned long long));
  b.xm2 = (double4*)take(n * sizeof(double4));
  b.vv2 = (double4*)take(n * sizeof(double4));
  b.cand2 = (unsigned long long*)take(n * sizeof(unsigned long long));
  b.encm2 = (unsigned long long*)take(n * sizeof(unsigned long long));
  b.off = (int*)take((ns + 1) * sizeof(int));
  b.m0 = (double*)take(ns * sizeof(double));
  b.order_nat = (int*)take(ns * sizeof(int));
  b.order_desc = (int*)take(ns * sizeof(int));
  b.ss = (BatchSysStat*)take(ns * sizeof(BatchSysStat));
  b.rslot = (int*)take(ns * sizeof(int));
  b.rbuf = (double*)take((size_t)std::max(nbig, 1) * kBsRDoubles * sizeof(double));
  b.ss2 = (BatchSysStat*)take(ns * sizeof(BatchSysStat));
  b.rad = (double*)take(n * sizeof(double));
  b.rad2 = (double*)take(n * sizeof(double));
  b.sp = (double4*)take(n * sizeof(double4));
  b.sp2 = (double4*)take(n * sizeof(double4));
  b.ids = (int*)take(n * sizeof(int));
  b.ids2 = (int*)take(n * sizeof(int));
  b.ev = (genga_event*)take(n * sizeof(genga_event));
  b.ev_cnt = (unsigned long long*)take(sizeof(unsigned long long));
  b.flags2 = (unsigned*)take(sizeof(unsigned));
  b.flag_in = (int*)take(sizeof(int));
  b.st = (DevStat*)take(sizeof(DevStat));
  return off;
}

hipError_t batch_pack(const BatchWs& b, const double* m, const double* x, const double* v,
                      int coords_in, bool keep_mass, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_pack, dim3(b.nsys), dim3(64), 0, s, m, x, v, b.off, b.m0, b.xm, b.vv,
                     coords_in == GENGA_HELIO, keep_mass ? 1 : 0);
  return hipGetLastError();
}

hipError_t batch_unpack(const BatchWs& b, double* x, double* v, int coords_out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_unpack, dim3(b.nsys), dim3(64), 0, s, b.xm, b.vv, b.off, b.m0, b.ss,
                     x, v, coords_out == GENGA_HELIO);
  return hipGetLastError();
}

hipError_t batch_prime(const BatchWs& b, const StepConsts& c, hipStream_t s) {
  BatchArgs a = batch_args(b, c, false, 0);
  hipLaunchKernelGGL(k_batch_prime, dim3(b.nsys), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t batch_energy(const BatchWs& b, const StepConsts& c, double* E, double* L,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_batch_energy, dim3(b.nsys), dim3(64), 0, s, b.xm, b.vv, b.off, b.m0, b.ss,
                     c.G, E, L);
  return hipGetLastError();
}

hipError_t batch_run(const BatchWs& b, const StepConsts& c, int variant, int nsteps, bool scratch,
                     hipStream_t s) {
  if (!batch_variant_ok(b, variant)) return hipErrorInvalidValue;
  const bool packed = variant >= kBatchPackedVariant0;
  BatchArgs a = batch_args(b, c, scratch, packed ? 1 : (variant & 1));
  a.nsteps = nsteps;
  const dim3 blk(64);
  // contexts whose bodies can leave run the kernel with that logic compiled
  // in; the others run it without
  if (!packed) {
    const dim3 g(b.nsys);
    switch ((variant >> 1) + (a.phys ? 3 : 0)) {
      case 0: hipLaunchKernelGGL((k_batch<1, 1, false>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_batch<2, 1, false>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_batch<4, 1, false>), g, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_batch<1, 1, true>), g, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_batch<2, 1, true>), g, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((k_batch<4, 1, true>), g, blk, 0, s, a); break;
    }
  } else {
    // two systems per wave: consecutive systems of the largest-first order
    const dim3 g((b.nsys + 1) / 2);
    switch ((variant - kBatchPackedVariant0) + (a.phys ? 3 : 0)) {
      case 0: hipLaunchKernelGGL((k_batch<1, 2, false>), g, blk, 0, s, a); break;
      case 1: hipLaunchKernelGGL((k_batch<2, 2, false>), g, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_batch<4, 2, false>), g, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((k_batch<1, 2, true>), g, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_batch<2, 2, true>), g, blk, 0, s, a); break;
      default: hipLaunchKernelGGL((k_batch<4, 2, true>), g, blk, 0, s, a); break;
    }
  }
  return hipGetLastError();
}

hipError_t batch_copy_to_scratch(const BatchWs& b, hipStream_t s) {
  const size_t n = (size_t)std::max<int64_t>(b.nb, 1);
  hipError_t e = hipMemcpyAsync(b.xm2, b.xm, n * sizeof(double4), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.vv2, b.vv, n * sizeof(double4), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.cand2, b.cand, n * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s);
  // the systems' counters go along (the live counts are needed)
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.ss2, b.ss, (size_t)b.nsys * sizeof(BatchSysStat), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.rad2, b.rad, n * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.sp2, b.sp, n * sizeof(double4), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b.ids2, b.ids, n * sizeof(int), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(b.flags2, 0, sizeof(unsigned), s);
  return e;
}

// New masses for every row; positions and velocities stay.
__global__ __launch_bounds__(256) void k_batch_masses(const double* __restrict__ m,
                                                      double4* __restrict__ xm, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) xm[i].w = m[i];
}

hipError_t batch_set_masses(const BatchWs& b, const double* m, hipStream_t s) {
  if (b.nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_masses, dim3((unsigned)((b.nb + 255) / 256)), dim3(256), 0, s, m,
                     b.xm, b.nb);
  return hipGetLastError();
}

hipError_t batch_reset_bodies(const BatchWs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(b.nsys), dim3(64), 0, s, b.off, b.ss, b.ids, b.sp, b.rad);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemsetAsync(b.ev_cnt, 0, sizeof(unsigned long long), s);
  return e;
}

}  // namespace genga
