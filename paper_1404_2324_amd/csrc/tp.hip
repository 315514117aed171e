// Test-particle mode (Sec. 3.3): massless particles feel at most 32 massive
// bodies and nothing else.  The massive bodies take the main-mode step; then
// one lane per particle runs the particle's whole step in one pass:
//   k_tp_main  opening kick (planets at the start of the step), Sun kick with
//              the planets' momentum, Kepler drift, Hermite test against the
//              particle's candidate planets; particles without an encounter
//              finish the step here (second Sun kick, closing kick, new
//              candidate mask); the others are compacted into a list
//   k_tp_bs    one wave per listed particle: BS of the particle with the
//              planets it encounters (planets feel only the star there), then
//              the rest of its step; a particle that comes closer to a planet
//              than the sum of their physical radii during a BS substep is
//              removed there and reported (Sec. 3.3)
// Particle state is stored as SoA (x[3][ntp], v[3][ntp]) plus a 32-bit
// candidate mask: 52 bytes read and written per particle and step.  A removed
// particle's x and v are NaN; every kernel skips it.
#include <algorithm>
#include <climits>

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
  double* __restrict__ bs_rct;        // their radii
  double* __restrict__ bs_y;          // their pre-drift state [6][cap]
  const double* __restrict__ rad;     // radii: planets [32], particles [ntp]
  CollRec* __restrict__ coll;         // removal reports
  int64_t ntp, cap;
  int nm, nblk, enc_free, max_iter;
  double G, h, m0, mu, dt, absdt, n2, pf2, tol;
  int max_depth;
};

// Kick of H_B on a particle from the planets (Eq. 2 gradient, K from the pair
// radius max(rct, rc_j)); positions from p (w = mass).
__device__ __forceinline__ void tp_kick_acc(const TpArgs& a, const double4* __restrict__ p,
                                            double x, double y, double z, double rct,
                                            double& ax, double& ay, double& az) {
  ax = ay = az = 0.0;
  for (int j = 0; j < a.nm; ++j) {
    const double4 pj = p[j];
    const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ir = rsqrt_nr(r2);
    const double ir2 = ir * ir;
    double K = 1.0, dK = 0.0;
    if (!a.enc_free) {
      const double rcij = fmax(rct, a.rc[j]);
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
__device__ __forceinline__ void tp_finish(const TpArgs& a, int64_t k, double x, double y,
                                          double z, double vx, double vy, double vz,
                                          double rct, double P2x, double P2y, double P2z) {
  x += a.h * P2x / a.m0;
  y += a.h * P2y / a.m0;
  z += a.h * P2z / a.m0;
  double ax, ay, az;
  tp_kick_acc(a, a.pfin, x, y, z, rct, ax, ay, az);
  vx += a.h * ax;
  vy += a.h * ay;
  vz += a.h * az;
  unsigned msk = 0u;
  if (!a.enc_free) {
    for (int j = 0; j < a.nm; ++j) {
      const double4 pj = a.pfin[j];
      const double dx = pj.x - x, dy = pj.y - y, dz = pj.z - z;
      const double rcij = fmax(rct, a.rc[j]);
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

__global__ __launch_bounds__(256) void k_tp_main(TpArgs a) {
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
    tp_kick_acc(a, a.px0, x, y, z, rct, ax, ay, az);
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
    if (!a.enc_free && cmask) {
      for (int j = 0; j < a.nm; ++j) {
        if (!(cmask & (1u << j))) continue;
        const double4 p0 = a.ppre[j], q0 = a.vpre[j], p1 = a.ppost[j], q1 = a.vpost[j];
        const double d2 = hermite_dmin2(a.dt, p0.x - xm0, p0.y - ym0, p0.z - zm0,
                                        q0.x - vxm, q0.y - vym, q0.z - vzm,
                                        p1.x - x, p1.y - y, p1.z - z,
                                        q1.x - vx, q1.y - vy, q1.z - vz);
        const double rcij = fmax(rct, a.rc[j]);
        if (d2 < rcij * rcij) emask |= 1u << j;
      }
    }
    if (emask) {
      listed = true;
    } else {
      tp_finish(a, k, x, y, z, vx, vy, vz, rct, P2x, P2y, P2z);
    }
  }
  const int itm = wave_max_i(abs(it));
  if (lane == 0 && itm > 0) atomicMax(&a.st->kep_itmax, itm);
  // ballot compaction of the particles with an encounter
  const unsigned long long lm = __ballot(listed);
  int base = 0;
  if (lane == 0 && lm) base = (int)atomicAdd(&a.st->tp_nbs, (unsigned)__popcll(lm));
  base = __shfl(base, 0, 64);
  const int ne = listed ? __popc(emask) : 0;
  int nen = ne;
  for (int o = 32; o > 0; o >>= 1) nen += __shfl_xor(nen, o, 64);
  if (lane == 0 && nen) {
    atomicAdd(&a.st->tp_enc, nen);
    atomicAdd(&a.st->tp_enc_total, (unsigned long long)nen);
  }
  if (listed) {
    const int64_t pos = base + (int)lanemask_count_tp(lm);
    if (pos < a.cap) {
      a.bs_idx[pos] = (int)k;
      a.bs_mask[pos] = emask;
      a.bs_rct[pos] = rct;
      a.bs_y[pos] = xm0;
      a.bs_y[a.cap + pos] = ym0;
      a.bs_y[2 * a.cap + pos] = zm0;
      a.bs_y[3 * a.cap + pos] = vxm;
      a.bs_y[4 * a.cap + pos] = vym;
      a.bs_y[5 * a.cap + pos] = vzm;
    }
  }
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
  const int b = lane % P;
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

__global__ __launch_bounds__(64) void k_tp_bs(TpArgs a) {
  __shared__ double mm[kBsPar], mrc[kBsPar];
  const int lane = threadIdx.x;
  const int64_t nl = __builtin_amdgcn_readfirstlane((int)min((int64_t)a.st->tp_nbs, a.cap));
  long long nsub = 0;
  const double P2x = a.st->P2[0], P2y = a.st->P2[1], P2z = a.st->P2[2];
  for (int64_t e = blockIdx.x; e < nl; e += gridDim.x) {
    const unsigned em = a.bs_mask[e];
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
      tp_finish(a, a.bs_idx[e], y[0], y[1], y[2], y[3], y[4], y[5], rct, P2x, P2y, P2z);
    }
  }
  if (lane == 0 && nsub > 0) atomicAdd(&a.st->bs_sub, (unsigned long long)nsub);
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
  a.pfin = w.xm;
  a.rc = w.rc_cur;
  a.partP = w.partP;
  a.st = w.st;
  a.bs_idx = t.bs_idx;
  a.bs_mask = t.bs_mask;
  a.bs_rct = t.bs_rct;
  a.bs_y = t.bs_y;
  a.rad = t.rad;
  a.coll = t.coll;
  a.ntp = t.ntp;
  a.cap = t.ntp;
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

size_t tp_carve(TpWs& t, int64_t ntp, void* base) {
  t.ntp = ntp;
  const size_t n = (size_t)std::max<int64_t>(ntp, 1);
  size_t off = 0;
  auto take = [&](size_t sz) -> void* {
    const size_t o = off;
    off += (sz + 255) & ~size_t(255);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  t.x = (double*)take(3 * n * sizeof(double));
  t.v = (double*)take(3 * n * sizeof(double));
  t.mask = (unsigned*)take(n * sizeof(unsigned));
  t.bs_idx = (int*)take(n * sizeof(int));
  t.bs_mask = (unsigned*)take(n * sizeof(unsigned));
  t.bs_rct = (double*)take(n * sizeof(double));
  t.bs_y = (double*)take(6 * n * sizeof(double));
  t.rad = (double*)take((kTpMaxPlanets + n) * sizeof(double));
  t.coll = (CollRec*)take(n * sizeof(CollRec));
  return off;
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
  hipLaunchKernelGGL(k_tp_main, dim3(ceil_div64(t.ntp, 256)), dim3(256), 0, s, a);
  if (!c.encounter_free)
    hipLaunchKernelGGL(k_tp_bs, dim3(2048), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace genga
