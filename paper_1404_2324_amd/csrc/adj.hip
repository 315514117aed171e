// Reverse-mode gradient of the encounter-free map (K = 1: the MVS map in
// democratic coordinates, Sec. 2.1; the paper itself has no adjoint):
//   one step = kick tau/2, Sun kick tau/2, Kepler drift tau, Sun kick tau/2,
//   kick tau/2.
// Given dL/dx_T and dL/dv_T the backward pass returns dL/dx_0, dL/dv_0 and
// dL/dm.  Memory: the forward pass keeps the state every k steps
// (checkpoints); the backward pass walks the segments from the last,
// recomputes each segment forward keeping its step-start states (the tape),
// then applies the vector-Jacobian product of every sub-flow in reverse:
//   kick:  v' = v + h a(x):      x^ += h J_a(x)^T v^',  m^ += h (da/dm)^T v^'
//   Sun:   x' = x + h P/m0:      v_j^ += h m_j/m0 S,    m_j^ += h v_j.S/m0,
//                                S = sum_i x_i^'
//   drift: (x', v') = f x + g v, fdot x + gdot v, with f, g, fdot, gdot
//          functions of r0 = |x|, eta0 = x.v, beta = 2 mu/r0 - v^2 and the
//          universal anomaly s, which solves r0 G1 + eta0 G2 + mu G3 = tau
//          (implicit function: ds/dq = -(dF/dq)/r).
// Systems are packed SB (a power of two >= the largest system) lanes each,
// 64/SB systems per wave; pair terms move by lane shuffles inside a segment.
#include <algorithm>

#include "adj_device.h"
#include "device_math.h"
#include "genga_impl.h"

namespace genga {
namespace {

struct AdjArgs {
  double4* __restrict__ xm;       // batched state
  double4* __restrict__ vv;
  const int* __restrict__ off;
  const double* __restrict__ m0;
  double* __restrict__ ckpt;      // [C][6][nb]
  double* __restrict__ tape;      // [k][6][nlanes]
  const double* __restrict__ gxT;  // [nb][3]
  const double* __restrict__ gvT;
  double* __restrict__ gx0;
  double* __restrict__ gv0;
  double* __restrict__ gm;        // [nb]
  unsigned* __restrict__ flags;
  int nsys, T, K, C, nlanes;
  int64_t nb;
  double G, dt, h, n1, n2, absdt;
  int max_iter;
};

template <int SB>
struct Lane {
  int seg, b, s, row, n;
  bool act;
};

template <int SB>
__device__ __forceinline__ Lane<SB> lane_of(const AdjArgs& a) {
  Lane<SB> L;
  const int lane = threadIdx.x & 63;
  L.seg = lane / SB;
  L.b = lane % SB;
  L.s = blockIdx.x * (64 / SB) + L.seg;
  L.n = 0;
  L.row = 0;
  if (L.s < a.nsys) {
    L.n = a.off[L.s + 1] - a.off[L.s];
    L.row = a.off[L.s] + L.b;
  }
  L.act = L.b < L.n;
  return L;
}

template <int SB>
__device__ __forceinline__ double seg_sum(double v) {
#pragma unroll
  for (int o = SB / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// a_i = sum_j G m_j (x_j - x_i)/r^3 inside the lane's segment.
template <int SB>
__device__ __forceinline__ void seg_acc(double G, double x, double y, double z, double m,
                                        double& ax, double& ay, double& az) {
  const int lane = threadIdx.x & 63, base = lane & ~(SB - 1);
  ax = ay = az = 0.0;
#pragma unroll 4
  for (int j = 0; j < SB; ++j) {
    const double xj = __shfl(x, base + j, 64), yj = __shfl(y, base + j, 64),
                 zj = __shfl(z, base + j, 64), mj = __shfl(m, base + j, 64);
    if (base + j != lane) {
      const double dx = xj - x, dy = yj - y, dz = zj - z;
      const double ir = rsqrt_nr(dx * dx + dy * dy + dz * dz);
      const double s = mj * ir * ir * ir;
      ax += s * dx;
      ay += s * dy;
      az += s * dz;
    }
  }
  ax *= G;
  ay *= G;
  az *= G;
}

// One step of the encounter-free map.
template <int SB>
__device__ __forceinline__ void free_step(const AdjArgs& a, bool act, double Gm0, double m0,
                                          double m, double& x, double& y, double& z, double& vx,
                                          double& vy, double& vz, unsigned& fl) {
  double ax, ay, az;
  seg_acc<SB>(a.G, x, y, z, m, ax, ay, az);
  vx += a.h * ax;
  vy += a.h * ay;
  vz += a.h * az;
  const double hm0 = a.h / m0;  // the Sun kick's factor (the replay uses the same)
  double Px = seg_sum<SB>(m * vx), Py = seg_sum<SB>(m * vy), Pz = seg_sum<SB>(m * vz);
  x += hm0 * Px;
  y += hm0 * Py;
  z += hm0 * Pz;
  if (act && kepler_drift(Gm0, a.dt, x, y, z, vx, vy, vz, a.max_iter) < 0) fl |= F_KEPLER;
  Px = seg_sum<SB>(m * vx);
  Py = seg_sum<SB>(m * vy);
  Pz = seg_sum<SB>(m * vz);
  x += hm0 * Px;
  y += hm0 * Py;
  z += hm0 * Pz;
  seg_acc<SB>(a.G, x, y, z, m, ax, ay, az);
  vx += a.h * ax;
  vy += a.h * ay;
  vz += a.h * az;
}

// A pair inside r_crit (Eq. 6) means the hybrid method would switch the pair
// to K < 1 there, so the K = 1 map is no longer the method's step.
template <int SB>
__device__ __forceinline__ bool seg_close(const AdjArgs& a, bool act, double Gm0, double m0,
                                          double m, double x, double y, double z, double vx,
                                          double vy, double vz) {
  const int lane = threadIdx.x & 63, base = lane & ~(SB - 1);
  const double rc = act ? rcrit(x, y, z, vx, vy, vz, m, Gm0, m0, a.n1, a.n2, a.absdt) : 0.0;
  bool close = false;
  for (int j = 0; j < SB; ++j) {
    const double xj = __shfl(x, base + j, 64), yj = __shfl(y, base + j, 64),
                 zj = __shfl(z, base + j, 64), rcj = __shfl(rc, base + j, 64);
    const double mj = __shfl(m, base + j, 64);
    if (act && mj > 0.0 && base + j != lane) {
      const double dx = xj - x, dy = yj - y, dz = zj - z;
      const double rcij = fmax(rc, rcj);
      if (dx * dx + dy * dy + dz * dz < rcij * rcij) close = true;
    }
  }
  return close;
}

template <int SB>
__device__ __forceinline__ void load_state(const AdjArgs& a, const Lane<SB>& L, double& x,
                                           double& y, double& z, double& vx, double& vy,
                                           double& vz, double& m) {
  const int lane = threadIdx.x & 63;
  x = 1.0e3 + lane;  // inactive lanes: massless, far away
  y = z = vx = vy = vz = m = 0.0;
  if (L.act) {
    const double4 p = a.xm[L.row], q = a.vv[L.row];
    x = p.x;
    y = p.y;
    z = p.z;
    m = p.w;
    vx = q.x;
    vy = q.y;
    vz = q.z;
  }
}

template <int SB>
__global__ __launch_bounds__(64) void k_adj_fwd(AdjArgs a) {
  const Lane<SB> L = lane_of<SB>(a);
  double x, y, z, vx, vy, vz, m;
  load_state<SB>(a, L, x, y, z, vx, vy, vz, m);
  const double m0 = L.s < a.nsys ? a.m0[L.s] : 1.0, Gm0 = a.G * m0;
  unsigned fl = 0u;
  for (int t = 0; t < a.T; ++t) {
    if (t % a.K == 0 && L.act) {
      double* c = a.ckpt + (size_t)(t / a.K) * 6 * a.nb;
      c[L.row] = x;
      c[a.nb + L.row] = y;
      c[2 * a.nb + L.row] = z;
      c[3 * a.nb + L.row] = vx;
      c[4 * a.nb + L.row] = vy;
      c[5 * a.nb + L.row] = vz;
    }
    if (seg_close<SB>(a, L.act, Gm0, m0, m, x, y, z, vx, vy, vz)) fl |= F_ADJ_ENC;
    free_step<SB>(a, L.act, Gm0, m0, m, x, y, z, vx, vy, vz, fl);
  }
  if (L.act) {
    a.xm[L.row] = make_double4(x, y, z, m);
    a.vv[L.row] = make_double4(vx, vy, vz, 0.0);
  }
  if (fl) atomicOr(a.flags, fl);
}

// ---- vector-Jacobian products ----------------------------------------------
// (J_a^T w)_k = sum_j T_kj (m_k w_j - m_j w_k), T = G (I/r^3 - 3 d d^T/r^5),
// and (da/dm)^T w for m_k = sum_i G (x_k - x_i).w_i / r_ik^3.
template <int SB>
__device__ __forceinline__ void kick_vjp(double G, double h, double x, double y, double z,
                                         double m, double wx, double wy, double wz,
                                         double& gx, double& gy, double& gz, double& gmass) {
  const int lane = threadIdx.x & 63, base = lane & ~(SB - 1);
  double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0;
#pragma unroll 2
  for (int j = 0; j < SB; ++j) {
    const int l = base + j;
    const double xj = __shfl(x, l, 64), yj = __shfl(y, l, 64), zj = __shfl(z, l, 64);
    const double mj = __shfl(m, l, 64);
    const double wxj = __shfl(wx, l, 64), wyj = __shfl(wy, l, 64), wzj = __shfl(wz, l, 64);
    if (l != lane) {
      const double dx = xj - x, dy = yj - y, dz = zj - z;
      const double ir = rsqrt_nr(dx * dx + dy * dy + dz * dz);
      const double ir2 = ir * ir, ir3 = ir2 * ir;
      // u = m_k w_j - m_j w_k;  T u = u/r^3 - 3 d (d.u)/r^5
      const double ux = m * wxj - mj * wx, uy = m * wyj - mj * wy, uz = m * wzj - mj * wz;
      const double du = 3.0 * (dx * ux + dy * uy + dz * uz) * ir3 * ir2;
      sx += ux * ir3 - dx * du;
      sy += uy * ir3 - dy * du;
      sz += uz * ir3 - dz * du;
      // d = x_j - x_k, so (x_k - x_j).w_j = -d.w_j
      sm -= (dx * wxj + dy * wyj + dz * wzj) * ir3;
    }
  }
  gx += h * G * sx;
  gy += h * G * sy;
  gz += h * G * sz;
  gmass += h * G * sm;
}

template <int SB>
__global__ __launch_bounds__(64) void k_adj_bwd(AdjArgs a) {
  const Lane<SB> L = lane_of<SB>(a);
  const int gl = blockIdx.x * 64 + (threadIdx.x & 63);
  double x, y, z, vx, vy, vz, m;
  load_state<SB>(a, L, x, y, z, vx, vy, vz, m);  // for the masses
  const double m0 = L.s < a.nsys ? a.m0[L.s] : 1.0, Gm0 = a.G * m0;
  double lx = 0.0, ly = 0.0, lz = 0.0, lvx = 0.0, lvy = 0.0, lvz = 0.0, lm = 0.0;
  if (L.act) {
    lx = a.gxT[3 * L.row];
    ly = a.gxT[3 * L.row + 1];
    lz = a.gxT[3 * L.row + 2];
    lvx = a.gvT[3 * L.row];
    lvy = a.gvT[3 * L.row + 1];
    lvz = a.gvT[3 * L.row + 2];
  }
  unsigned fl = 0u;
  const int lane = threadIdx.x & 63;
  for (int c = a.C - 1; c >= 0; --c) {
    const int t0 = c * a.K, t1 = min(a.T, t0 + a.K);
    x = 1.0e3 + lane;
    y = z = vx = vy = vz = 0.0;
    if (L.act) {
      const double* cp = a.ckpt + (size_t)c * 6 * a.nb;
      x = cp[L.row];
      y = cp[a.nb + L.row];
      z = cp[2 * a.nb + L.row];
      vx = cp[3 * a.nb + L.row];
      vy = cp[4 * a.nb + L.row];
      vz = cp[5 * a.nb + L.row];
    }
    for (int t = t0; t < t1; ++t) {
      double* tp = a.tape + (size_t)(t - t0) * 6 * a.nlanes;
      tp[gl] = x;
      tp[a.nlanes + gl] = y;
      tp[2 * a.nlanes + gl] = z;
      tp[3 * a.nlanes + gl] = vx;
      tp[4 * a.nlanes + gl] = vy;
      tp[5 * a.nlanes + gl] = vz;
      free_step<SB>(a, L.act, Gm0, m0, m, x, y, z, vx, vy, vz, fl);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const double* tp = a.tape + (size_t)(t - t0) * 6 * a.nlanes;
      // recompute the step's intermediate states
      double px = tp[gl], py = tp[a.nlanes + gl], pz = tp[2 * a.nlanes + gl];
      double qx = tp[3 * a.nlanes + gl], qy = tp[4 * a.nlanes + gl], qz = tp[5 * a.nlanes + gl];
      const double xa[3] = {px, py, pz};  // positions of the first kick
      double ax, ay, az;
      seg_acc<SB>(a.G, px, py, pz, m, ax, ay, az);
      qx += a.h * ax;
      qy += a.h * ay;
      qz += a.h * az;
      const double v1[3] = {qx, qy, qz};  // velocities of the first Sun kick
      double Px = seg_sum<SB>(m * qx), Py = seg_sum<SB>(m * qy), Pz = seg_sum<SB>(m * qz);
      px += (a.h / m0) * Px;
      py += (a.h / m0) * Py;
      pz += (a.h / m0) * Pz;
      const double x2[3] = {px, py, pz};  // pre-drift state (x2, v1)
      double sK = 0.0;
      if (L.act) kepler_drift(Gm0, a.dt, px, py, pz, qx, qy, qz, a.max_iter, &sK);
      const double v3[3] = {qx, qy, qz};  // velocities of the second Sun kick
      Px = seg_sum<SB>(m * qx);
      Py = seg_sum<SB>(m * qy);
      Pz = seg_sum<SB>(m * qz);
      px += (a.h / m0) * Px;
      py += (a.h / m0) * Py;
      pz += (a.h / m0) * Pz;  // (px, py, pz): positions of the second kick
      // second kick: x4 -> v5 = v3 + h a(x4)
      double gx = lx, gy = ly, gz = lz;
      kick_vjp<SB>(a.G, a.h, px, py, pz, m, lvx, lvy, lvz, gx, gy, gz, lm);
      // second Sun kick: x4 = x3 + h P(v3)/m0
      double S0 = seg_sum<SB>(gx), S1 = seg_sum<SB>(gy), S2 = seg_sum<SB>(gz);
      double w3x = lvx + a.h * m / m0 * S0, w3y = lvy + a.h * m / m0 * S1,
             w3z = lvz + a.h * m / m0 * S2;
      lm += a.h / m0 * (v3[0] * S0 + v3[1] * S1 + v3[2] * S2);
      // drift
      double l2[3] = {gx, gy, gz}, lv1[3] = {w3x, w3y, w3z};
      if (L.act) {
        const double lx3[3] = {gx, gy, gz}, lv3[3] = {w3x, w3y, w3z};
        const double vpre[3] = {v1[0], v1[1], v1[2]};
        kepler_vjp(Gm0, a.dt, x2, vpre, sK, lx3, lv3, l2, lv1);
      }
      // first Sun kick: x2 = x + h P(v1)/m0
      S0 = seg_sum<SB>(l2[0]);
      S1 = seg_sum<SB>(l2[1]);
      S2 = seg_sum<SB>(l2[2]);
      double w1x = lv1[0] + a.h * m / m0 * S0, w1y = lv1[1] + a.h * m / m0 * S1,
             w1z = lv1[2] + a.h * m / m0 * S2;
      lm += a.h / m0 * (v1[0] * S0 + v1[1] * S1 + v1[2] * S2);
      // first kick: v1 = v + h a(x)
      gx = l2[0];
      gy = l2[1];
      gz = l2[2];
      kick_vjp<SB>(a.G, a.h, xa[0], xa[1], xa[2], m, w1x, w1y, w1z, gx, gy, gz, lm);
      lx = gx;
      ly = gy;
      lz = gz;
      lvx = w1x;
      lvy = w1y;
      lvz = w1z;
      if (!L.act) lx = ly = lz = lvx = lvy = lvz = lm = 0.0;
    }
  }
  if (L.act) {
    a.gx0[3 * L.row] = lx;
    a.gx0[3 * L.row + 1] = ly;
    a.gx0[3 * L.row + 2] = lz;
    a.gv0[3 * L.row] = lvx;
    a.gv0[3 * L.row + 1] = lvy;
    a.gv0[3 * L.row + 2] = lvz;
    a.gm[L.row] = lm;
  }
  if (fl) atomicOr(a.flags, fl);
}

}  // namespace

int adj_segment_lanes(int max_n) {
  int sb = 1;
  while (sb < max_n) sb <<= 1;
  return sb;
}

hipError_t adj_forward(const BatchWs& b, const StepConsts& c, int sb, int T, int K, double* ckpt,
                       hipStream_t s) {
  AdjArgs a{};
  a.xm = b.xm;
  a.vv = b.vv;
  a.off = b.off;
  a.m0 = b.m0;
  a.ckpt = ckpt;
  a.flags = &b.st->flags;
  a.nsys = b.nsys;
  a.T = T;
  a.K = K;
  a.C = (T + K - 1) / K;
  a.nb = b.nb;
  a.G = c.G;
  a.dt = c.dt;
  a.h = c.h;
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.absdt = fabs(c.dt);
  a.max_iter = c.kepler_max_iter;
  const int W = 64 / sb;
  const dim3 g((b.nsys + W - 1) / W), blk(64);
  switch (sb) {
    case 1: hipLaunchKernelGGL(k_adj_fwd<1>, g, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_adj_fwd<2>, g, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_adj_fwd<4>, g, blk, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_adj_fwd<8>, g, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL(k_adj_fwd<16>, g, blk, 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_adj_fwd<32>, g, blk, 0, s, a); break;
    default: hipLaunchKernelGGL(k_adj_fwd<64>, g, blk, 0, s, a); break;
  }
  return hipGetLastError();
}

size_t adj_tape_bytes(int nsys, int sb, int K) {
  const int W = 64 / sb;
  const size_t nl = (size_t)((nsys + W - 1) / W) * 64;
  return nl * 6 * (size_t)K * sizeof(double);
}

hipError_t adj_backward(const BatchWs& b, const StepConsts& c, int sb, int T, int K,
                        double* ckpt, double* tape, const double* gxT, const double* gvT,
                        double* gx0, double* gv0, double* gm, hipStream_t s) {
  AdjArgs a{};
  a.xm = b.xm;
  a.vv = b.vv;
  a.off = b.off;
  a.m0 = b.m0;
  a.ckpt = ckpt;
  a.tape = tape;
  a.gxT = gxT;
  a.gvT = gvT;
  a.gx0 = gx0;
  a.gv0 = gv0;
  a.gm = gm;
  a.flags = &b.st->flags;
  a.nsys = b.nsys;
  a.T = T;
  a.K = K;
  a.C = (T + K - 1) / K;
  a.nb = b.nb;
  a.G = c.G;
  a.dt = c.dt;
  a.h = c.h;
  a.n1 = c.n1;
  a.n2 = c.n2;
  a.absdt = fabs(c.dt);
  a.max_iter = c.kepler_max_iter;
  const int W = 64 / sb;
  a.nlanes = ((b.nsys + W - 1) / W) * 64;
  const dim3 g((b.nsys + W - 1) / W), blk(64);
  switch (sb) {
    case 1: hipLaunchKernelGGL(k_adj_bwd<1>, g, blk, 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_adj_bwd<2>, g, blk, 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_adj_bwd<4>, g, blk, 0, s, a); break;
    case 8: hipLaunchKernelGGL(k_adj_bwd<8>, g, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL(k_adj_bwd<16>, g, blk, 0, s, a); break;
    case 32: hipLaunchKernelGGL(k_adj_bwd<32>, g, blk, 0, s, a); break;
    default: hipLaunchKernelGGL(k_adj_bwd<64>, g, blk, 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace genga
