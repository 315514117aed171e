// Main-mode kernels of the hybrid symplectic step (Grimm & Stadel,
// arXiv:1404.2324, Sec. 2.2 step recipe and Sec. 3.2 kernels), for gfx950.
//
// One step is six launches on one stream (captured once into a HIP graph):
//   k_open_drift   opening kick: cached non-candidate acceleration + candidate
//                  pairs recomputed with the new radii (KickA/KickB, Sec 3.2.3);
//                  Sun kick tau/2 (Eq. 3) + pre-drift copy + Kepler drift
//                  (Eq. 9) + momentum partials for the second Sun kick
//   k_encounter    Hermite test of every candidate (Eqs. 10-12), ballot
//                  compaction of the confirmed pairs
//   k_group        equivalence classes of the pairs in LDS (App. A)
//   k_bs           Bulirsch-Stoer integration of H_A per group, one wave each
//   k_kick         closing kick: all pairs and the prechecker, per j-block
//   k_kick_finish  fixed-order sum of the partials, second Sun kick tau/2,
//                  v += tau/2 a, next radii
#include <hip/hip_ext.h>

#include <climits>
#include <cstddef>

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
struct KickArgs {
  const double4* __restrict__ xm;     // read by the pair kernel
  double4* __restrict__ xm_rw;        // same array, updated by the finish
  double4* __restrict__ xs;           // start positions of the next step
  const double* __restrict__ thr;
  const double* __restrict__ rc;
  double4* __restrict__ part;
  int* __restrict__ ccnt;
  int* __restrict__ ctab;
  double4* __restrict__ vv;
  double4* __restrict__ afar;
  double* __restrict__ rc_next;
  double* __restrict__ acc_out;
  const double* __restrict__ partP2;  // momentum partials after the drift
  const double* __restrict__ dP;      // momentum change of each BS group
  DevStat* __restrict__ st;
  int n, np, jb_len, cpb, nblk;
  int encounter_free;
  double G, h, m0, mu, n1, n2, absdt, pf;
};

enum { KICK_CLOSE = 0, KICK_INIT = 1, KICK_ACC = 2 };

// All-pairs kick of H_B (Eq. 2 gradient) with the prechecker.
// Grid (ceil(n/64), njb); a workgroup holds 64 i-bodies (one per lane) and a
// j-range split over its waves.  j-data is wave-uniform and read through the
// scalar cache into SGPRs; the FP64 pair loop runs on the VALU.  Pairs with
// r^2 < max((pf rc_i)^2, (pf rc_j)^2) are candidates: their K-weighted term is
// summed apart ("near") and appended to the per-body candidate table; all
// other pairs have K = 1 and form the reusable "far" sum.  Each workgroup
// writes its j-block partials; k_kick_finish combines them in a fixed order
// (a kernel boundary instead of a device-scope fence per workgroup, which
// costs an L2 write-back on this multi-XCD part).
// xm and thr come as kernel arguments of their own: as noalias parameters the
// compiler can prove the wave-uniform j loads invariant and issue them as
// scalar loads (struct members do not carry that guarantee).
template <int MODE>
__global__ __launch_bounds__(kKickWaves * 64) void k_kick(KickArgs a,
                                                          const double4* __restrict__ xmj,
                                                          const double* __restrict__ thrj) {
  constexpr int W = kKickWaves;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.x * 64 + lane;
  const bool iv = i < a.n;
  double xi = 0.0, yi = 0.0, zi = 0.0, ti = kTiny;
  if (iv) {
    const double4 p = a.xm[i];
    xi = p.x;
    yi = p.y;
    zi = p.z;
    ti = a.thr[i];
  }
  const int jb = blockIdx.y;
  const int j0 = jb * a.jb_len;
  const int j1 = min(a.n, j0 + a.jb_len);
  const int wl = (max(0, j1 - j0) + W - 1) / W;
  const int js = j0 + wave * wl;
  const int je = min(j1, js + wl);

  double fx = 0.0, fy = 0.0, fz = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  auto pair = [&](const double4& pj, double tj, int j) {
    const double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt_nr(r2);
    const double ir2 = ir * ir;
    const double s = pj.w * (ir2 * ir);
    const bool cand = r2 < fmax(ti, tj);
    const double sf = cand ? 0.0 : s;
    fx += sf * dx;
    fy += sf * dy;
    fz += sf * dz;
    if (__builtin_expect(cand, 0)) {
      if (iv && j != i) {
        double K = 1.0, dK = 0.0;
        if (!a.encounter_free) changeover(r2 * ir, fmax(a.rc[i], a.rc[j]), K, dK);
        const double sn = pj.w * (K * ir2 * ir - dK * ir2);
        nx += sn * dx;
        ny += sn * dy;
        nz += sn * dz;
        if (MODE != KICK_ACC && !a.encounter_free) {
          const int slot = atomicAdd(&a.ccnt[i], 1);
          if (slot < a.cpb)
            a.ctab[(size_t)i * a.cpb + slot] = j;
          else
            atomicOr(&a.st->flags, F_CAND_OVF);
        }
      }
    }
  };
  // four partners per round trip of the scalar loads (the scalar cache
  // returns out of order, so every use waits for all loads in flight)
  int j = js;
  for (; j + 3 < je; j += 4) {
    const double4 p0 = xmj[j], p1 = xmj[j + 1], p2 = xmj[j + 2], p3 = xmj[j + 3];
    const double t0 = thrj[j], t1 = thrj[j + 1], t2 = thrj[j + 2], t3 = thrj[j + 3];
    pair(p0, t0, j);
    pair(p1, t1, j + 1);
    pair(p2, t2, j + 2);
    pair(p3, t3, j + 3);
  }
  for (; j < je; ++j) pair(xmj[j], thrj[j], j);

  if (MODE == KICK_CLOSE && blockIdx.x == 0 && blockIdx.y == 0 && wave == 0) {
    // momentum after the drift and BS for the second Sun kick: drift partials
    // plus each group's change, strided over the lanes, then a butterfly
    double px = 0.0, py = 0.0, pz = 0.0;
    for (int b = lane; b < a.nblk; b += 64) {
      px += a.partP2[4 * b + 0];
      py += a.partP2[4 * b + 1];
      pz += a.partP2[4 * b + 2];
    }
    const int ng = a.encounter_free ? 0 : a.st->ngroups;
    for (int g = lane; g < ng; g += 64) {
      px += a.dP[4 * g + 0];
      py += a.dP[4 * g + 1];
      pz += a.dP[4 * g + 2];
    }
    px = wave_sum(px);
    py = wave_sum(py);
    pz = wave_sum(pz);
    if (lane == 0) {
      a.st->P2[0] = px;
      a.st->P2[1] = py;
      a.st->P2[2] = pz;
      a.st->ctl = 0u;  // the finish sets the bits for the next opening kick
    }
  }
  if (MODE == KICK_INIT && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    a.st->ctl = 0u;
  __shared__ double sh[W][6][64];
  sh[wave][0][lane] = fx;
  sh[wave][1][lane] = fy;
  sh[wave][2][lane] = fz;
  sh[wave][3][lane] = nx;
  sh[wave][4][lane] = ny;
  sh[wave][5][lane] = nz;
  __syncthreads();
  for (int c = threadIdx.x >> 6; c < 6; c += W) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += sh[w][c][lane];
    sh[0][c][lane] = t;
  }
  __syncthreads();
  if (threadIdx.x < 64 && iv) {
    double4* q = &a.part[((size_t)jb * a.np + i) * 2];
    q[0] = make_double4(sh[0][0][lane], sh[0][1][lane], sh[0][2][lane], 0.0);
    q[1] = make_double4(sh[0][3][lane], sh[0][4][lane], sh[0][5][lane], 0.0);
  }
}

// Closing-kick epilogue, four lanes per body: the j-block partials are summed
// in a fixed order (strided per lane, then a butterfly over the four lanes);
// the far part is kept for the next opening kick.
//   CLOSE: second Sun kick of the step (x += tau/2 P/m0 with P assembled by
//          the pair kernel from the drift's momentum partials and each BS
//          group's momentum change; the pair kernel only needs relative
//          positions, so the shift can follow it), v += tau/2 a, next radii
//          (Eq. 6) and the reuse check
//   INIT:  far part only (first step's opening kick)
//   ACC:   acceleration out
template <int MODE>
__global__ __launch_bounds__(kVecBlock) void k_kick_finish(KickArgs a, int njb) {
  const int t = blockIdx.x * kVecBlock + threadIdx.x;
  const int i = t >> 2, sub = t & 3;
  const bool iv = i < a.n;
  double S0 = 0, S1 = 0, S2 = 0, S3 = 0, S4 = 0, S5 = 0;
  if (iv) {
    for (int b = sub; b < njb; b += 4) {
      const double4* q = &a.part[((size_t)b * a.np + i) * 2];
      const double4 f = q[0];
      const double4 g = q[1];
      S0 += f.x;
      S1 += f.y;
      S2 += f.z;
      S3 += g.x;
      S4 += g.y;
      S5 += g.z;
    }
  }
#pragma unroll
  for (int o = 1; o < 4; o <<= 1) {
    S0 += __shfl_xor(S0, o, 64);
    S1 += __shfl_xor(S1, o, 64);
    S2 += __shfl_xor(S2, o, 64);
    S3 += __shfl_xor(S3, o, 64);
    S4 += __shfl_xor(S4, o, 64);
    S5 += __shfl_xor(S5, o, 64);
  }
  if (!iv || sub != 0) return;
  const double G = a.G;
  if (MODE == KICK_ACC) {
    a.acc_out[3 * (size_t)i + 0] = G * (S0 + S3);
    a.acc_out[3 * (size_t)i + 1] = G * (S1 + S4);
    a.acc_out[3 * (size_t)i + 2] = G * (S2 + S5);
    return;
  }
  a.afar[i] = make_double4(G * S0, G * S1, G * S2, 0.0);
  if (MODE == KICK_INIT) {
    a.rc_next[i] = a.rc[i];
    a.xs[i] = a.xm_rw[i];
    return;
  }
  const double Px = a.st->P2[0], Py = a.st->P2[1], Pz = a.st->P2[2];
  double4 p = a.xm_rw[i];
  p.x += a.h * Px / a.m0;
  p.y += a.h * Py / a.m0;
  p.z += a.h * Pz / a.m0;
  a.xm_rw[i] = p;
  a.xs[i] = p;
  double4 v = a.vv[i];
  v.x += a.h * (G * (S0 + S3));
  v.y += a.h * (G * (S1 + S4));
  v.z += a.h * (G * (S2 + S5));
  a.vv[i] = v;
  const double rcn =
      rcrit(p.x, p.y, p.z, v.x, v.y, v.z, p.w, a.mu, a.m0, a.n1, a.n2, a.absdt);
  a.rc_next[i] = rcn;
  if (!a.encounter_free && rcn > a.pf * a.rc[i]) atomicOr(&a.st->ctl, C_FULLKICK);
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
  const int* __restrict__ ccnt;
  const int* __restrict__ ctab;
  double* __restrict__ partP;
  double* __restrict__ partP2;
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
__global__ __launch_bounds__(kVecBlock) void k_open_drift(OpenArgs a) {
  __shared__ double sh[3 * (kVecBlock / 64)];
  const int i = blockIdx.x * kVecBlock + threadIdx.x;
  const bool iv = i < a.n;
  const bool full = (__builtin_amdgcn_readfirstlane(a.st->ctl) & C_FULLKICK) != 0;
  const double Ps = a.h / a.m0;
  const double sx = Ps * a.st->P2[0], sy = Ps * a.st->P2[1], sz = Ps * a.st->P2[2];
  double m = 0.0, kx = 0.0, ky = 0.0, kz = 0.0, dx = 0.0, dy = 0.0, dz = 0.0;
  int it = 0;
  if (iv) {
    const double4 p = a.xs[i];
    const double rci = a.rc_next[i];
    if (a.xstart) a.xstart[i] = p;
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (full) {
      for (int j = 0; j < a.n; ++j)
        if (j != i) pair_hb(p.x, p.y, p.z, rci, a.xs[j], a.rc_next[j], a.encounter_free, ax, ay, az);
      ax *= a.G;
      ay *= a.G;
      az *= a.G;
    } else {
      const double4 af = a.afar[i];
      const int cnt = min(a.ccnt[i], a.cpb);
      const int* row = a.ctab + (size_t)i * a.cpb;
      double cx = 0.0, cy = 0.0, cz = 0.0;
      // Partners are summed in ascending order (deterministic).  Rows of up
      // to 8 (nearly all), 16 or kRowSort partners are sorted by a bitonic
      // network of that width in registers; partner data is then fetched 8
      // at a time with independent loads.  Longer rows fall back to an
      // ordered scan.
      if (cnt <= kPre) {
        int jj[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) jj[u] = u < cnt ? row[u] : INT_MAX;
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
    double4 v = a.vv[i];
    v.x += a.h * ax;
    v.y += a.h * ay;
    v.z += a.h * az;
    a.rc_cur[i] = rci;
    a.thr[i] = a.encounter_free ? kTiny : fmax(a.pf2 * rci * rci, kTiny);
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
  if ((threadIdx.x & 63) == 0 && itm > a.st->kep_itmax) atomicMax(&a.st->kep_itmax, itm);
  double Px = m * kx, Py = m * ky, Pz = m * kz;
  block_sum3<kVecBlock>(Px, Py, Pz, sh);
  double Qx = m * dx, Qy = m * dy, Qz = m * dz;
  block_sum3<kVecBlock>(Qx, Qy, Qz, sh);
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

// Exclusive scan over a block of 1024 threads; returns the prefix and puts the
// total in *total.
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
  for (int k = 0; k < kEncThreads / 64; ++k) {
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

// Equivalence classes of the encounter pairs (App. A), one workgroup: LINK
// starts as the identity, every pair lowers both ends to the smaller link
// (LDS atomic min), links are shortened by LINK[i] = LINK[LINK[i]], and both
// sweeps repeat until nothing changes.  Groups are numbered by their smallest
// member; offsets and members go to global memory for the BS kernel.  Also
// clears the candidate table for the closing kick and counts its pairs.
__global__ __launch_bounds__(kEncThreads) void k_group(EncArgs a) {
  __shared__ int link[kGroupMaxN];
  __shared__ int gid[kGroupMaxN];
  __shared__ int2 pr[kEncLds];
  __shared__ int gsz[kGroupMaxN / 2 + 1];
  __shared__ int gof[kGroupMaxN / 2 + 1];
  __shared__ unsigned char inp[kGroupMaxN];
  __shared__ int shw[kEncThreads / 64];
  __shared__ int s_changed;
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = a.n;
  const int ne_all = a.st->nenc;
  const int ne = min(min(ne_all, kEncLds), a.enc_cap);
  for (int i = tid; i < n; i += kEncThreads) {
    link[i] = i;
    inp[i] = 0;
  }
  for (int e = tid; e < ne; e += kEncThreads) pr[e] = a.encij[e];
  __syncthreads();
  // candidate pairs i < j: every pair sits in both rows (the test is
  // symmetric), so half the sum of the row lengths
  int rows = 0;
  for (int i = tid; i < n; i += kEncThreads) {
    rows += min(a.ccnt[i], a.cpb);
    a.ccnt[i] = 0;
  }
  for (int e = tid; e < ne; e += kEncThreads) {
    inp[pr[e].x] = 1;
    inp[pr[e].y] = 1;
  }
  // equivalence classes
  while (true) {
    if (tid == 0) s_changed = 0;
    __syncthreads();
    bool ch = false;
    for (int e = tid; e < ne; e += kEncThreads) {
      const int p1 = pr[e].x, p2 = pr[e].y;
      const int l1 = link[p1], l2 = link[p2];
      if (l1 != l2) {
        atomicMin(&link[p1], l2);
        atomicMin(&link[p2], l1);
        ch = true;
      }
    }
    __syncthreads();
    for (int i = tid; i < n; i += kEncThreads) {
      const int l = link[i];
      const int ll = link[l];
      if (ll < l) {
        atomicMin(&link[i], ll);
        ch = true;
      }
    }
    if (ch) s_changed = 1;
    __syncthreads();
    if (!s_changed) break;
    __syncthreads();
  }
  // consecutive group ids in order of the smallest member
  constexpr int PER = kGroupMaxN / kEncThreads;
  int cntr = 0;
  for (int k = 0; k < PER; ++k) {
    const int i = tid * PER + k;
    if (i < n && inp[i] && link[i] == i) ++cntr;
  }
  int ng = 0;
  int off = block_excl_scan(cntr, shw, &ng);
  for (int k = 0; k < PER; ++k) {
    const int i = tid * PER + k;
    if (i < n && inp[i] && link[i] == i) gid[i] = off++;
  }
  for (int g = tid; g <= ng; g += kEncThreads) gsz[g] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += kEncThreads)
    if (inp[i]) atomicAdd(&gsz[gid[link[i]]], 1);
  __syncthreads();
  // offsets: exclusive scan of the sizes
  constexpr int GPER = (kGroupMaxN / 2 + kEncThreads - 1) / kEncThreads;
  int loc = 0, mx = 0;
  for (int k = 0; k < GPER; ++k) {
    const int g = tid * GPER + k;
    if (g < ng) {
      loc += gsz[g];
      mx = max(mx, gsz[g]);
    }
  }
  int tot = 0;
  int o2 = block_excl_scan(loc, shw, &tot);
  for (int k = 0; k < GPER; ++k) {
    const int g = tid * GPER + k;
    if (g < ng) {
      gof[g] = o2;
      a.goff[g] = o2;
      o2 += gsz[g];
    }
  }
  if (tid == 0) a.goff[ng] = tot;
  int nrow = 0;
  (void)block_excl_scan(rows, shw, &nrow);
  mx = wave_max_i(mx);
  __syncthreads();
  if (lane == 0) shw[tid >> 6] = mx;
  for (int g = tid; g < ng; g += kEncThreads) gsz[g] = 0;
  __syncthreads();
  if (tid == 0) {
    int m2 = 0;
    for (int k = 0; k < kEncThreads / 64; ++k) m2 = max(m2, shw[k]);
    a.st->maxg = m2;
    a.st->ngroups = ng;
    a.st->ncand = nrow / 2;
    a.st->enc_total += (unsigned long long)ne_all;
    if (ne_all > kEncLds || ne_all > a.enc_cap) atomicOr(&a.st->flags, F_ENC_OVF);
  }
  for (int i = tid; i < n; i += kEncThreads) {
    if (inp[i]) {
      const int g = gid[link[i]];
      const int pos = gof[g] + atomicAdd(&gsz[g], 1);
      a.gmem[pos] = i;
    }
  }
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
  DevStat* __restrict__ st;
  double G, Gm0, dt, tol;
  int max_depth;
};

// Main-mode group of sz <= P members (sorted indices in mem, masses and radii
// in mm, mrc): start from the pre-drift copy, integrate, write back; returns
// the BS status and, per member lane, its momentum change m (v_BS - v_drift).
template <int P>
__device__ __forceinline__ int bs_member_group(const BsArgs& a, int sz, const int* mem,
                                               double* mm, double* mrc, long long* nsub,
                                               double& dpx, double& dpy, double& dpz) {
  const int lane = threadIdx.x & 63;
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
  if (ml >= 0) {
    mm[lane] = mw;
    mrc[lane] = rcw;
  }
  __syncthreads();
  const int r = bs_group<P, false>(sz, y, mm, mrc, a.dt, a.G, a.Gm0, a.tol, a.max_depth, nsub);
  dpx = dpy = dpz = 0.0;
  if (lane == par_lane<P>(0, 0, b) && id >= 0) {  // one lane per member writes
    const double m = mm[b];
    dpx = m * (y[3] - vo.x);
    dpy = m * (y[4] - vo.y);
    dpz = m * (y[5] - vo.z);
    a.xm[id] = make_double4(y[0], y[1], y[2], m);
    a.vv[id] = make_double4(y[3], y[4], y[5], 0.0);
  }
  return r;
}

// One wave per encounter group (grid-stride over the device-side count):
// members sorted ascending, state reset to the pre-drift copy, H_A integrated
// over tau by BS, result written back.  Groups of up to 8 members take the
// all-columns path with speculative depths, larger ones (up to 64) one lane
// per member with the columns in sequence.
__global__ __launch_bounds__(64) void k_bs(BsArgs a) {
  __shared__ double R[kBsCols][6][64];
  __shared__ int mem[64];
  __shared__ double mm[kBsPar], mrc[kBsPar];
  const int lane = threadIdx.x;
  const int ng = __builtin_amdgcn_readfirstlane(a.st->ngroups);
  long long nsub = 0;
  for (int g = blockIdx.x; g < ng; g += gridDim.x) {
    const int o = a.goff[g];
    const int sz = a.goff[g + 1] - o;
    if (sz > kBsMaxGroup) {
      if (lane == 0) atomicOr(&a.st->flags, F_GROUP);
      continue;
    }
    const int my = lane < sz ? a.gmem[o + lane] : INT_MAX;
    int rank = 0;
    for (int q = 0; q < sz; ++q) rank += (__builtin_amdgcn_readlane(my, q) < my) ? 1 : 0;
    __syncthreads();
    if (lane < sz) mem[rank] = my;
    __syncthreads();
    double dpx = 0.0, dpy = 0.0, dpz = 0.0;
    if (sz <= kBsPar) {
      int r;
      if (sz <= 2)
        r = bs_member_group<2>(a, sz, mem, mm, mrc, &nsub, dpx, dpy, dpz);
      else if (sz <= 4)
        r = bs_member_group<4>(a, sz, mem, mm, mrc, &nsub, dpx, dpy, dpz);
      else
        r = bs_member_group<8>(a, sz, mem, mm, mrc, &nsub, dpx, dpy, dpz);
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
                                 a.max_depth, R, &nsub);
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
    // the group's momentum change for the second Sun kick (fixed lane order)
    dpx = wave_sum(dpx);
    dpy = wave_sum(dpy);
    dpz = wave_sum(dpz);
    if (lane == 0) {
      a.dP[4 * g + 0] = dpx;
      a.dP[4 * g + 1] = dpy;
      a.dP[4 * g + 2] = dpz;
    }
    __syncthreads();
  }
  if (lane == 0 && nsub > 0) atomicAdd(&a.st->bs_sub, (unsigned long long)nsub);
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
__global__ void k_pack(const double* __restrict__ m, const double* __restrict__ x,
                       const double* __restrict__ v, const double* __restrict__ mom,
                       double4* __restrict__ xm, double4* __restrict__ vv, int n,
                       int np, int helio, double m0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  if (i >= n) {
    xm[i] = make_double4(0.0, 0.0, 0.0, 0.0);
    vv[i] = make_double4(0.0, 0.0, 0.0, 0.0);
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
                         double* __restrict__ v, int n, int helio, double m0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
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
__global__ void k_rcrit_init(const double4* __restrict__ xm, const double4* __restrict__ vv,
                             double* __restrict__ rc, double* __restrict__ thr,
                             int* __restrict__ ccnt, int n, double mu, double m0,
                             double n1, double n2, double absdt, double pf2,
                             int enc_free) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 p = xm[i], q = vv[i];
  const double r = rcrit(p.x, p.y, p.z, q.x, q.y, q.z, p.w, mu, m0, n1, n2, absdt);
  rc[i] = r;
  thr[i] = enc_free ? kTiny : fmax(pf2 * r * r, kTiny);
  ccnt[i] = 0;
}

// Per-body energy terms and angular momentum; rows[8 i + k]:
// kinetic, -G m0 m/r, -1/2 G m sum_j m_j/r_ij, m v (3), m x x v (3) -> 9 terms
__global__ void k_energy_rows(const double4* __restrict__ xm, const double4* __restrict__ vv,
                              int n, double G, double m0, double* __restrict__ rows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
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
__global__ void k_thresholds(const double* __restrict__ rc, double* __restrict__ thr,
                             int* __restrict__ ccnt, int n, double pf2, int enc_free) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  thr[i] = enc_free ? kTiny : fmax(pf2 * rc[i] * rc[i], kTiny);
  ccnt[i] = 0;
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

KickArgs kick_args(const MassiveWs& w, const StepConsts& c) {
  KickArgs a;
  a.xm = w.xm;
  a.xm_rw = w.xm;
  a.xs = w.xs;
  a.thr = w.thr;
  a.rc = w.rc_cur;
  a.part = w.part;
  a.ccnt = w.ccnt;
  a.ctab = w.ctab;
  a.vv = w.vv;
  a.afar = w.afar;
  a.rc_next = w.rc_next;
  a.acc_out = nullptr;
  a.partP2 = w.partP2;
  a.dP = w.dP;
  a.st = w.st;
  a.n = w.n;
  a.np = w.np;
  a.jb_len = w.jb_len;
  a.cpb = w.cpb;
  a.nblk = w.nblk;
  a.encounter_free = c.encounter_free;
  a.G = c.G;
  a.h = c.h;
  a.m0 = c.m0;
  a.mu = c.mu;
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.absdt = fabs(c.dt);
  a.pf = c.pf;
  return a;
}

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
  return c;
}

static void kick_shape(int n, int& nitile, int& njb, int& jb_len) {
  nitile = ceil_div(n, 64);
  const int by_target = ceil_div(kKickTarget, nitile);
  const int by_len = ceil_div(n, kKickWaves * 16);
  njb = std::max(1, std::min(by_target, by_len));
  jb_len = ceil_div(n, njb);
  njb = ceil_div(n, jb_len);
}

size_t massive_ws_bytes(int n, const genga_params& p, bool snap) {
  if (n < 1) return 0;
  MassiveWs w;
  return massive_carve(w, n, p, nullptr, snap);
}

// Lay the main-mode arrays out in the workspace starting at base (nullptr:
// only size the layout).  Returns the bytes used.
size_t massive_carve(MassiveWs& w, int n, const genga_params& p, void* base, bool snap) {
  w.n = n;
  w.np = ceil_div(n, 256) * 256;
  kick_shape(n, w.nitile, w.njb, w.jb_len);
  w.nblk = ceil_div(n, kVecBlock);
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
  w.part = (double4*)take((size_t)w.njb * np * 2 * sizeof(double4));
  w.rc_cur = (double*)take(np * sizeof(double));
  w.rc_next = (double*)take(np * sizeof(double));
  w.thr = (double*)take(np * sizeof(double));
  w.partP = (double*)take((size_t)w.nblk * 4 * sizeof(double));
  w.partP2 = (double*)take((size_t)w.nblk * 4 * sizeof(double));
  w.dP = (double*)take((np / 2 + 1) * 4 * sizeof(double));
  w.red = (double*)take(std::max<size_t>(np * 9, 64) * sizeof(double));
  w.ccnt = (int*)take(np * sizeof(int));
  w.ctab = (int*)take(np * (size_t)std::max(1, w.cpb) * sizeof(int));
  w.encij = (int2*)take((size_t)std::max(1, w.enc_cap) * sizeof(int2));
  w.encd2 = (double*)take((size_t)std::max(1, w.enc_cap) * sizeof(double));
  w.encrc2 = (double*)take((size_t)std::max(1, w.enc_cap) * sizeof(double));
  w.goff = (int*)take((np + 1) * sizeof(int));
  w.gmem = (int*)take(np * sizeof(int));
  w.flag_in = (int*)take(sizeof(int));
  w.xstart = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.xpost = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.vpost = snap ? (double4*)take(np * sizeof(double4)) : nullptr;
  w.st = (DevStat*)take(sizeof(DevStat));
  return off;
}

hipError_t massive_pack(const MassiveWs& w, const StepConsts& c, const double* m,
                        const double* x, const double* v, int coords_in,
                        hipStream_t s) {
  const int helio = coords_in == GENGA_HELIO;
  if (helio) hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, m, v, nullptr, nullptr, w.n, w.red);
  hipLaunchKernelGGL(k_pack, dim3(ceil_div(w.np, 256)), dim3(256), 0, s, m, x, v, w.red,
                     w.xm, w.vv, w.n, w.np, helio, c.m0);
  return hipGetLastError();
}

hipError_t massive_unpack(const MassiveWs& w, const StepConsts& c, double* x,
                          double* v, int coords_out, hipStream_t s) {
  const int helio = coords_out == GENGA_HELIO;
  if (helio)
    hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, nullptr, nullptr, w.xm, w.vv, w.n, w.red);
  hipLaunchKernelGGL(k_unpack, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xm, w.vv, w.red,
                     x, v, w.n, helio, c.m0);
  return hipGetLastError();
}

hipError_t massive_prime(const MassiveWs& w, const StepConsts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_rcrit_init, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xm, w.vv,
                     w.rc_cur, w.thr, w.ccnt, w.n, c.mu, c.m0, c.n1, c.n2, fabs(c.dt),
                     c.pf2, c.encounter_free);
  KickArgs a = kick_args(w, c);
  hipLaunchKernelGGL(k_kick<KICK_INIT>, dim3(w.nitile, w.njb), dim3(kKickWaves * 64), 0, s, a,
                     a.xm, a.thr);
  hipLaunchKernelGGL(k_kick_finish<KICK_INIT>, dim3(ceil_div(4 * w.n, kVecBlock)), dim3(kVecBlock), 0, s, a, w.njb);
  // the momentum for the first step's first Sun kick
  double* P2 = reinterpret_cast<double*>(reinterpret_cast<char*>(w.st) + offsetof(DevStat, P2));
  hipLaunchKernelGGL(k_momentum, dim3(1), dim3(1024), 0, s, nullptr, nullptr, w.xm, w.vv, w.n, P2);
  return hipGetLastError();
}

hipError_t massive_accel(const MassiveWs& w, const StepConsts& c, double* acc,
                         hipStream_t s) {
  KickArgs a = kick_args(w, c);
  a.acc_out = acc;
  hipLaunchKernelGGL(k_kick<KICK_ACC>, dim3(w.nitile, w.njb), dim3(kKickWaves * 64), 0, s, a,
                     a.xm, a.thr);
  hipLaunchKernelGGL(k_kick_finish<KICK_ACC>, dim3(ceil_div(4 * w.n, kVecBlock)), dim3(kVecBlock), 0, s, a, w.njb);
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
  o.ccnt = w.ccnt;
  o.ctab = w.ctab;
  o.partP = w.partP;
  o.partP2 = w.partP2;
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
  STEP_LAUNCH(0, k_open_drift, dim3(w.nblk), dim3(kVecBlock), o);

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
    STEP_LAUNCH(1, k_encounter, dim3(ceil_div(w.n * w.cpb, kVecBlock)), dim3(kVecBlock), e);
    STEP_LAUNCH(2, k_group, dim3(1), dim3(kEncThreads), e);

    BsArgs b;
    b.xm = w.xm;
    b.vv = w.vv;
    b.dP = w.dP;
    b.xpre = w.xpre;
    b.vpre = w.vpre;
    b.rc = w.rc_cur;
    b.goff = w.goff;
    b.gmem = w.gmem;
    b.st = w.st;
    b.G = c.G;
    b.Gm0 = c.mu;
    b.dt = c.dt;
    b.tol = c.bs_tol;
    b.max_depth = c.bs_max_depth;
    STEP_LAUNCH(3, k_bs, dim3(std::max(1, std::min(256, w.n / 2))), dim3(64), b);
  }

  KickArgs a = kick_args(w, c);
  STEP_LAUNCH(4, k_kick<KICK_CLOSE>, dim3(w.nitile, w.njb), dim3(kKickWaves * 64), a,
              (const double4*)a.xm, (const double*)a.thr);
  STEP_LAUNCH(5, k_kick_finish<KICK_CLOSE>, dim3(ceil_div(4 * w.n, kVecBlock)), dim3(kVecBlock),
              a, w.njb);
  return hipGetLastError();
}

hipError_t massive_energy(const MassiveWs& w, const StepConsts& c, double* dE,
                          double* dL, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_rows, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xm, w.vv,
                     w.n, c.G, c.m0, w.red);
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
                     w.ccnt, w.n, c.pf2, c.encounter_free);
  return hipGetLastError();
}

hipError_t massive_masses(const MassiveWs& w, double* m, hipStream_t s) {
  hipLaunchKernelGGL(k_masses, dim3(ceil_div(w.n, 256)), dim3(256), 0, s, w.xm, m, w.n);
  return hipGetLastError();
}

}  // namespace genga
