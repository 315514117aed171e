/*
 * Plain FP64 CPU oracle for the hybrid symplectic N-body step of
 * Grimm & Stadel, "The GENGA Code" (arXiv:1404.2324).
 *
 * TEST INFRASTRUCTURE ONLY: it is the reference the GPU library is checked
 * against, never a fallback of it.  Every routine is the plain definition of
 * what the paper computes, in the paper's order, without the two
 * optimisations that reach the same result faster:
 *   - the kick-reuse of KickA/KickB (Sec. 3.2.3) is replaced by recomputing
 *     every pair in every half kick;
 *   - the prechecker (Sec. 2.2) is replaced by the Hermite test on every
 *     pair; the prechecker's candidate set C is still formed so that the
 *     method's encounter set (E intersected with C) and the count of
 *     precheck misses (E minus C) can both be reported.
 *
 * Readings of passages that are silent or garbled are marked "Reading:".
 * Parity status of each routine is listed in the header comment of the
 * routine; "parity unpinned" marks a choice the paper does not fix.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared
 */
#include "genga_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define V3(a, i) (&(a)[3 * (size_t)(i)])

static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Threads of the OpenMP loops over independent rows (the timing of the
 * oracle on all host cores and on one core).                               */
void go_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}
int go_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* Changeover function, Eq. (4) with y of Eq. (5).
 * K = 0 for y <= 0, y^2/(2y^2-2y+1) for 0<y<1, 1 for y >= 1.
 * Reading: K is continuous at y = 0 and y = 1, so the closed ends are
 * assigned to the constant branches.  dK/dy = 2y(1-y)/(2y^2-2y+1)^2 is the
 * derivative of the middle branch.                                          */
void go_changeover(double y, double *K, double *dKdy) {
    if (y <= 0.0) {
        *K = 0.0;
        *dKdy = 0.0;
    } else if (y >= 1.0) {
        *K = 1.0;
        *dKdy = 0.0;
    } else {
        double D = 2.0 * y * y - 2.0 * y + 1.0;
        *K = y * y / D;
        *dKdy = 2.0 * y * (1.0 - y) / (D * D);
    }
}

/* K and dK/dr for a pair at separation r with pair critical radius rcij,
 * y = (r - 0.1 rcij) / (0.9 rcij)  (Eq. 5; the "r_rcrit" of the printed
 * equation is read as r_crit).  A non-positive rcij means no changeover.  */
static void pair_K(double r, double rcij, double *K, double *dKdr) {
    if (!(rcij > 0.0)) {
        *K = 1.0;
        *dKdr = 0.0;
        return;
    }
    double y = (r - 0.1 * rcij) / (0.9 * rcij);
    double dKdy;
    go_changeover(y, K, &dKdy);
    *dKdr = dKdy / (0.9 * rcij);
}

/* ------------------------------------------------------------------------ */
/* Critical radius, Eq. (6): rc_i = max(n1 R_H,i, n2 |tau| |v_i|).
 * Reading: R_H,i = a_i (m_i / (3 m0))^(1/3) with the osculating semi-major
 * axis a_i from 1/a = 2/r - v^2/mu, mu = G m0, using the democratic (x_i,
 * v_i); when 1/a <= 0 the heliocentric distance r_i replaces a_i.  |tau| so
 * that a backward step uses the same radius.  (parity unpinned: the paper
 * leaves R_H undefined.)                                                   */
void go_rcrit(const go_params *p, int n, const double *m, const double *x,
              const double *v, double *rc) {
    double mu = p->G * p->m0;
    for (int i = 0; i < n; ++i) {
        double r = sqrt(dot3(V3(x, i), V3(x, i)));
        double vv = dot3(V3(v, i), V3(v, i));
        double inva = 2.0 / r - vv / mu;
        double a = inva > 0.0 ? 1.0 / inva : r;
        double rh = a * cbrt(m[i] / (3.0 * p->m0));
        double rv = p->n2 * fabs(p->dt) * sqrt(vv);
        double r1 = p->n1 * rh;
        rc[i] = r1 > rv ? r1 : rv;
    }
}

/* ------------------------------------------------------------------------ */
/* Acceleration of the perturbing part H_B (Eq. 2).  Reading: the kick is the
 * exact negative gradient of Eq. (2) divided by m_i,
 *   a_i = sum_{j != i} G m_j [ K/r^3 - K'(r)/r^2 ] (x_j - x_i),
 * so that the sub-flow is Hamiltonian.  With encounter_free set, K = 1 and
 * K' = 0: the plain Newtonian sum of the MVS map.
 * Pinned by: brute-force sum in extended precision, the central-difference
 * gradient of H_B, sum_i m_i a_i = 0, the Newtonian special case.           */
void go_accel(const go_params *p, int n, const double *m, const double *x,
              const double *rc, double *acc) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d0 = x[3 * j + 0] - x[3 * i + 0];
            double d1 = x[3 * j + 1] - x[3 * i + 1];
            double d2 = x[3 * j + 2] - x[3 * i + 2];
            double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            double r = sqrt(r2);
            double f;
            if (p->encounter_free) {
                f = 1.0 / (r2 * r);
            } else {
                double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
                double K, dK;
                pair_K(r, rcij, &K, &dK);
                f = K / (r2 * r) - dK / r2;
            }
            double s = p->G * m[j] * f;
            a0 += s * d0;
            a1 += s * d1;
            a2 += s * d2;
        }
        acc[3 * i + 0] = a0;
        acc[3 * i + 1] = a1;
        acc[3 * i + 2] = a2;
    }
}

/* Sun part H_C (Eq. 3): its flow moves every heliocentric position by
 * h P / m0 with P = sum_j m_j v_j, velocities unchanged.                    */
void go_sun_drift(const go_params *p, int n, const double *m, double *x,
                  const double *v, double h) {
    double P[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < 3; ++k) P[k] += m[j] * v[3 * j + k];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) x[3 * i + k] += h * P[k] / p->m0;
}

/* ------------------------------------------------------------------------ */
/* Stumpff functions c0..c3 of z (textbook universal-variable formulation,
 * Danby 1988, to which Sec. 2.2 refers for the f and g functions).
 * c_k(z) = sum_n (-z)^n / (k+2n)!.  The argument is quartered until
 * |z| < 0.1, c2 and c3 are summed as series, c0 = 1 - z c2, c1 = 1 - z c3,
 * and the results are rebuilt with the quadruple-argument identities
 *   c0(4z) = 2 c0^2 - 1, c1(4z) = c0 c1, c2(4z) = c1^2/2,
 *   c3(4z) = (c2 + c0 c3)/4.                                               */
void go_stumpff(double z, double c[4]) {
    int nq = 0;
    while (fabs(z) >= 0.1 && nq < 64) { /* bounded for non-finite z */
        z *= 0.25;
        ++nq;
    }
    /* series to n = 8: the first neglected term is below 1e-20 */
    double c2 = 0.0, c3 = 0.0;
    {
        double t2 = 1.0 / 2.0, t3 = 1.0 / 6.0;
        for (int k = 0; k <= 8; ++k) {
            c2 += t2;
            c3 += t3;
            t2 *= -z / ((double)(2 * k + 3) * (double)(2 * k + 4));
            t3 *= -z / ((double)(2 * k + 4) * (double)(2 * k + 5));
        }
    }
    double c0 = 1.0 - z * c2;
    double c1 = 1.0 - z * c3;
    for (int q = 0; q < nq; ++q) {
        double n0 = 2.0 * c0 * c0 - 1.0;
        double n1 = c0 * c1;
        double n2 = 0.5 * c1 * c1;
        double n3 = 0.25 * (c2 + c0 * c3);
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    c[0] = c0;
    c[1] = c1;
    c[2] = c2;
    c[3] = c3;
}

/* c4 and c5, used only by the tangent-linear model of the drift. */
static void stumpff45(double z, const double c[4], double *c4, double *c5) {
    if (fabs(z) < 1.0) {
        double s4 = 0.0, s5 = 0.0, t4 = 1.0 / 24.0, t5 = 1.0 / 120.0;
        for (int k = 0; k <= 14; ++k) {
            s4 += t4;
            s5 += t5;
            t4 *= -z / ((double)(2 * k + 5) * (double)(2 * k + 6));
            t5 *= -z / ((double)(2 * k + 6) * (double)(2 * k + 7));
        }
        *c4 = s4;
        *c5 = s5;
    } else {
        /* c_k = 1/k! - z c_{k+2} */
        *c4 = (0.5 - c[2]) / z;
        *c5 = (1.0 / 6.0 - c[3]) / z;
    }
}

/* Keplerian drift of one body for time dt with mu = G m0 (Sec. 2.2, Eq. 9:
 * x = f x0 + g v0, v = fdot x0 + gdot v0), written in universal variables.
 * With r0 = |x0|, eta0 = x0.v0, beta = 2 mu / r0 - v0^2, zeta0 = mu - beta r0
 * and G_k = s^k c_k(beta s^2), the universal Kepler equation
 *   F(s) = r0 G1 + eta0 G2 + mu G3 - dt = 0,  F' = r = r0 + eta0 G1 + zeta0 G2,
 *   F'' = eta0 G0 + zeta0 G1
 * is solved by the Laguerre-Conway iteration (order 5) from s = dt / r0 until
 * |ds| <= 2^-50 |s|, or until |F| is within 2^-48 of the sum of the magnitudes
 * of its terms (the residual is rounding noise; strongly hyperbolic orbits
 * over long steps end there).  Reading: the paper gives no stopping rule.  Then f = 1 - mu G2/r0, g = dt - mu G3,
 * fdot = -mu G1/(r r0), gdot = 1 - mu G2/r.
 * Reading: universal variables replace the paper's fallback to BS for
 * unbound or non-converging orbits; non-convergence is an error.
 * Pinned by: the closed-form Kepler orbit, f gdot - fdot g = 1, conserved
 * energy and angular momentum, drift(dt) then drift(-dt) = identity.        */
static void gk_at(double s, double beta, double G[4]) {
    double c[4];
    go_stumpff(beta * s * s, c);
    G[0] = c[0];
    G[1] = s * c[1];
    G[2] = s * s * c[2];
    G[3] = s * s * s * c[3];
}

static int kepler_solve(double mu, double r0, double eta0, double beta,
                        double dt, int max_iter, double *s_out, int *iters) {
    double zeta0 = mu - beta * r0;
    double s = dt / r0;
    int it = 0;
    int ok = 0;
    for (it = 1; it <= max_iter; ++it) {
        double G[4];
        gk_at(s, beta, G);
        double F = r0 * G[1] + eta0 * G[2] + mu * G[3] - dt;
        /* residual at the rounding level of its own terms: s cannot improve */
        double Fscale = fabs(r0 * G[1]) + fabs(eta0 * G[2]) + fabs(mu * G[3]) + fabs(dt);
        if (fabs(F) <= ldexp(Fscale, -48)) {
            ok = 1;
            break;
        }
        double Fp = r0 + eta0 * G[1] + zeta0 * G[2];
        double Fpp = eta0 * G[0] + zeta0 * G[1];
        const double nl = 5.0;
        double disc = (nl - 1.0) * (nl - 1.0) * Fp * Fp - nl * (nl - 1.0) * F * Fpp;
        double sq = sqrt(fabs(disc));
        double den = Fp + (Fp >= 0.0 ? sq : -sq);
        double ds = -nl * F / den;
        s += ds;
        if (fabs(ds) <= ldexp(fabs(s), -50)) {
            ok = 1;
            break;
        }
    }
    if (iters) *iters = ok ? it : max_iter;
    *s_out = s;
    return ok ? GO_OK : GO_EKEPLER;
}

int go_kepler(double mu, const double *x0, const double *v0, double dt,
              double *x, double *v, int max_iter, int *iters) {
    double r0 = sqrt(dot3(x0, x0));
    double eta0 = dot3(x0, v0);
    double beta = 2.0 * mu / r0 - dot3(v0, v0);
    double zeta0 = mu - beta * r0;
    double s;
    int rcode = kepler_solve(mu, r0, eta0, beta, dt, max_iter, &s, iters);
    double G[4];
    gk_at(s, beta, G);
    double r = r0 + eta0 * G[1] + zeta0 * G[2];
    double f = 1.0 - mu * G[2] / r0;
    double g = dt - mu * G[3];
    double fd = -mu * G[1] / (r * r0);
    double gd = 1.0 - mu * G[2] / r;
    double xn[3], vn[3];
    for (int k = 0; k < 3; ++k) {
        xn[k] = f * x0[k] + g * v0[k];
        vn[k] = fd * x0[k] + gd * v0[k];
    }
    for (int k = 0; k < 3; ++k) {
        x[k] = xn[k];
        v[k] = vn[k];
    }
    return rcode;
}

/* The root s of the universal Kepler equation that go_kepler takes (its own
 * iteration), for the complex-step derivative of the drift. */
int go_kepler_root(double mu, const double *x0, const double *v0, double dt, int max_iter,
                   double *s, int *iters) {
    double r0 = sqrt(dot3(x0, x0));
    double eta0 = dot3(x0, v0);
    double beta = 2.0 * mu / r0 - dot3(v0, v0);
    return kepler_solve(mu, r0, eta0, beta, dt, max_iter, s, iters);
}

/* ------------------------------------------------------------------------ */
/* Close-encounter test, Eqs. (10)-(12).  P(t) is the cubic Hermite
 * interpolant of the squared separation over t in [0,1] (physical time
 * t*dt) from P0 = |dx0|^2, P1 = |dx1|^2 and the physical-time derivatives
 * Pd0 = 2 dx0.dv0, Pd1 = 2 dx1.dv1.
 * Reading: the coefficient a of dP/dt = a t^2 + b t + c printed in the paper
 * has a sign error; differentiating Eq. (10) gives
 *   a = 6 (P0 - P1) + 3 dt (Pd0 + Pd1), b = 6 (P1 - P0) - 2 dt (2 Pd0 + Pd1),
 *   c = dt Pd0.
 * Reading: the returned minimum is taken over t = 0, t = 1 and the real
 * roots of the quadratic inside (0, 1); a = 0 reduces to the linear case.
 * Pinned by: straight-line relative motion (P exactly quadratic) and dense
 * sampling of Eq. (10).                                                     */
static double hermite_P(double t, double dt, double P0, double P1, double Pd0,
                        double Pd1) {
    double u = 1.0 - t;
    return P0 * (1.0 + 2.0 * t) * u * u + P1 * t * t * (3.0 - 2.0 * t) +
           Pd0 * dt * t * u * u - Pd1 * dt * t * t * u;
}

double go_hermite_dmin2(double dt, const double *dx0, const double *dv0,
                        const double *dx1, const double *dv1) {
    double P0 = dot3(dx0, dx0), P1 = dot3(dx1, dx1);
    double Pd0 = 2.0 * dot3(dx0, dv0), Pd1 = 2.0 * dot3(dx1, dv1);
    double a = 6.0 * (P0 - P1) + 3.0 * dt * (Pd0 + Pd1);
    double b = 6.0 * (P1 - P0) - 2.0 * dt * (2.0 * Pd0 + Pd1);
    double c = dt * Pd0;
    double best = P0 < P1 ? P0 : P1;
    double roots[2];
    int nr = 0;
    if (a != 0.0) {
        double disc = b * b - 4.0 * a * c;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -0.5 * (b + (b >= 0.0 ? sq : -sq));
            roots[nr++] = q / a;
            if (q != 0.0) roots[nr++] = c / q;
        }
    } else if (b != 0.0) {
        roots[nr++] = -c / b;
    }
    for (int k = 0; k < nr; ++k) {
        double t = roots[k];
        if (t > 0.0 && t < 1.0) {
            double Pt = hermite_P(t, dt, P0, P1, Pd0, Pd1);
            if (Pt < best) best = Pt;
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Close-encounter groups (Sec. 3.2.5, App. A): the equivalence classes of
 * the encounter relation, i.e. the connected components of the encounter
 * graph, labelled by their smallest member index.  Plain definition: every
 * body in a pair starts with its own index and repeatedly takes the minimum
 * label over its pairs until nothing changes.  label[i] = -1 for bodies in
 * no pair.  Returns the number of groups.
 * Pinned by: breadth-first components on small graphs.                     */
int go_groups(int n, int npairs, const int32_t *ij, int32_t *label) {
    for (int i = 0; i < n; ++i) label[i] = -1;
    for (int e = 0; e < npairs; ++e) {
        label[ij[2 * e]] = ij[2 * e];
        label[ij[2 * e + 1]] = ij[2 * e + 1];
    }
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int e = 0; e < npairs; ++e) {
            int a = ij[2 * e], b = ij[2 * e + 1];
            int l = label[a] < label[b] ? label[a] : label[b];
            if (label[a] != l) { label[a] = l; changed = 1; }
            if (label[b] != l) { label[b] = l; changed = 1; }
        }
    }
    int ng = 0;
    for (int i = 0; i < n; ++i)
        if (label[i] == i) ++ng;
    return ng;
}

/* ------------------------------------------------------------------------ */
/* Direct integration of H_A (Eq. 1) for one close-encounter group
 * (Sec. 2.2 and 3.2.6): the star is fixed at the origin during the step,
 *   dx_i/dt = v_i,
 *   dv_i/dt = -G m0 x_i/|x_i|^3
 *             + sum_{j in group} G m_j [(1-K)/r^3 + K'(r)/r^2] (x_j - x_i),
 * with the critical radii of the step frozen.  The method is
 * Bulirsch-Stoer: Gragg's modified midpoint rule with n_k = 2k substeps
 * (k = 1..8), Aitken-Neville extrapolation in h^2, and per-body relative
 * errors of position and velocity.  A substep is accepted at the first
 * column k >= 2 whose error is <= bs_tol; if all 8 columns fail the substep
 * is halved (binary refinement that covers H exactly), up to bs_max_depth
 * halvings.  Reading: the paper names the method only; the sequence, the
 * error norm, the tolerance and the halving rule are this oracle's (parity
 * unpinned against the paper; pinned by Kepler agreement and the group's
 * conserved H_A).
 * tp_mode: body 0 is a massless test particle; only it feels the pair
 * terms, the other members (planets) feel only the star (Sec. 3.3).
 * rad (tp_mode only, may be NULL): physical radii of the members.  After each
 * accepted substep the particle's separation from every planet member is
 * tested over the substep with the Hermite rule of Eqs. (10)-(12) applied to
 * that substep; below the sum of the radii the integration stops at the
 * start of the substep (a collision, Sec. 3.2.7 and Sec. 3.3).              */
#define BS_KMAX 8
#define BS_COLLIDED 1

typedef struct {
    const go_params *p;
    int ng;
    const double *m;
    const double *rc;
    int tp_mode;
    const double *rad;
} ha_sys;

static void ha_deriv(const ha_sys *s, const double *y, double *dy) {
    int ng = s->ng;
    double Gm0 = s->p->G * s->p->m0;
    for (int i = 0; i < ng; ++i) {
        const double *xi = &y[6 * i];
        double r2 = dot3(xi, xi);
        double r = sqrt(r2);
        double fs = -Gm0 / (r2 * r);
        double a0 = fs * xi[0], a1 = fs * xi[1], a2 = fs * xi[2];
        if (!s->tp_mode || i == 0) {
            for (int j = 0; j < ng; ++j) {
                if (j == i) continue;
                const double *xj = &y[6 * j];
                double d0 = xj[0] - xi[0], d1 = xj[1] - xi[1], d2 = xj[2] - xi[2];
                double q2 = d0 * d0 + d1 * d1 + d2 * d2;
                double q = sqrt(q2);
                double rcij = s->rc[i] > s->rc[j] ? s->rc[i] : s->rc[j];
                double K, dK;
                pair_K(q, rcij, &K, &dK);
                double f = (1.0 - K) / (q2 * q) + dK / q2;
                double sj = s->p->G * s->m[j] * f;
                a0 += sj * d0;
                a1 += sj * d1;
                a2 += sj * d2;
            }
        }
        dy[6 * i + 0] = y[6 * i + 3];
        dy[6 * i + 1] = y[6 * i + 4];
        dy[6 * i + 2] = y[6 * i + 5];
        dy[6 * i + 3] = a0;
        dy[6 * i + 4] = a1;
        dy[6 * i + 5] = a2;
    }
}

/* Gragg's modified midpoint rule over H with nsub substeps. */
static void mmid(const ha_sys *s, const double *y0, double H, int nsub,
                 double *yout, double *ym, double *yn, double *d, double *tmp) {
    int dim = 6 * s->ng;
    double hs = H / nsub;
    ha_deriv(s, y0, d);
    for (int k = 0; k < dim; ++k) {
        ym[k] = y0[k];
        yn[k] = y0[k] + hs * d[k];
    }
    for (int m = 1; m < nsub; ++m) {
        ha_deriv(s, yn, d);
        for (int k = 0; k < dim; ++k) {
            tmp[k] = ym[k] + 2.0 * hs * d[k];
            ym[k] = yn[k];
            yn[k] = tmp[k];
        }
    }
    ha_deriv(s, yn, d);
    for (int k = 0; k < dim; ++k) yout[k] = 0.5 * (ym[k] + yn[k] + hs * d[k]);
}

static double vrel(const double *a, const double *b) {
    double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
    double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double den = sqrt(dot3(a, a));
    return den > 0.0 ? num / den : num;
}

/* One BS attempt over H from y0.  Returns 1 and fills yout on success. */
static int bs_attempt(const ha_sys *s, const double *y0, double H, double *yout,
                      double *T, double *w) {
    int dim = 6 * s->ng;
    double *ym = w, *yn = w + dim, *d = w + 2 * dim, *tmp = w + 3 * dim;
#define TT(k, j) (&T[((size_t)(k) * BS_KMAX + (j)) * dim])
    for (int k = 0; k < BS_KMAX; ++k) {
        int nk = 2 * (k + 1);
        mmid(s, y0, H, nk, TT(k, 0), ym, yn, d, tmp);
        for (int j = 1; j <= k; ++j) {
            int nkj = 2 * (k - j + 1);
            double ratio = (double)nk / (double)nkj;
            double den = ratio * ratio - 1.0;
            double *cur = TT(k, j), *prev = TT(k, j - 1), *up = TT(k - 1, j - 1);
            for (int q = 0; q < dim; ++q) cur[q] = prev[q] + (prev[q] - up[q]) / den;
        }
        if (k >= 1) {
            double err = 0.0;
            const double *A = TT(k, k), *B = TT(k, k - 1);
            for (int i = 0; i < s->ng; ++i) {
                double ex = vrel(&A[6 * i], &B[6 * i]);
                double ev = vrel(&A[6 * i + 3], &B[6 * i + 3]);
                if (ex > err) err = ex;
                if (ev > err) err = ev;
            }
            if (err <= s->p->bs_tol) {
                memcpy(yout, A, sizeof(double) * dim);
                return 1;
            }
        }
    }
#undef TT
    return 0;
}

/* Lowest planet member the particle (member 0) comes closer to than the sum
 * of their radii during the substep y0 -> y1 of length h, or 0 for none.  */
static int tp_collision(const ha_sys *s, const double *y0, const double *y1, double h) {
    for (int j = 1; j < s->ng; ++j) {
        double dx0[3], dv0[3], dx1[3], dv1[3];
        for (int k = 0; k < 3; ++k) {
            dx0[k] = y0[6 * j + k] - y0[k];
            dv0[k] = y0[6 * j + 3 + k] - y0[3 + k];
            dx1[k] = y1[6 * j + k] - y1[k];
            dv1[k] = y1[6 * j + 3 + k] - y1[3 + k];
        }
        double R = s->rad[0] + s->rad[j];
        if (go_hermite_dmin2(h, dx0, dv0, dx1, dv1) < R * R) return j;
    }
    return 0;
}

/* Massive groups with radii (Sec. 3.2.7): the first member pair (a, b),
 * a < b in member order, whose separation falls below R_a + R_b during the
 * substep y0 -> y1 of length h (the Hermite rule of Eqs. (10)-(12) applied
 * to the substep, as the paper reuses the encounter test between BS steps);
 * returns 1 and sets *ca, *cb, or 0.                                       */
static int group_collision(const ha_sys *s, const double *y0, const double *y1, double h,
                           int *ca, int *cb) {
    for (int a = 0; a < s->ng; ++a)
        for (int b = a + 1; b < s->ng; ++b) {
            double R = s->rad[a] + s->rad[b];
            if (!(R > 0.0)) continue;
            double dx0[3], dv0[3], dx1[3], dv1[3];
            for (int k = 0; k < 3; ++k) {
                dx0[k] = y0[6 * b + k] - y0[6 * a + k];
                dv0[k] = y0[6 * b + 3 + k] - y0[6 * a + 3 + k];
                dx1[k] = y1[6 * b + k] - y1[6 * a + k];
                dv1[k] = y1[6 * b + 3 + k] - y1[6 * a + 3 + k];
            }
            if (go_hermite_dmin2(h, dx0, dv0, dx1, dv1) < R * R) {
                *ca = a;
                *cb = b;
                return 1;
            }
        }
    return 0;
}

/* Returns GO_OK, GO_EBS, GO_EINVAL, or BS_COLLIDED with *coll_member (the
 * planet member; for a massive group the first member of the pair and
 * *coll_b the second) and *coll_frac (the fraction of H covered before the
 * substep in which the collision happens; y is the state there), and the
 * length of that substep in *coll_h.                                       */
static int bs_integrate2(const ha_sys *s, double *y, double H, int64_t *substeps,
                         int *coll_member, int *coll_b, double *coll_frac, double *coll_h);
static int bs_integrate(const ha_sys *s, double *y, double H, int64_t *substeps,
                        int *coll_member, double *coll_frac) {
    int cb = 0;
    double ch = 0.0;
    return bs_integrate2(s, y, H, substeps, coll_member, &cb, coll_frac, &ch);
}

static int bs_integrate2(const ha_sys *s, double *y, double H, int64_t *substeps,
                         int *coll_member, int *coll_b, double *coll_frac, double *coll_h) {
    int dim = 6 * s->ng;
    int D = s->p->bs_max_depth;
    if (D < 0 || D > 40) return GO_EINVAL;
    double *T = (double *)malloc(sizeof(double) * dim * BS_KMAX * BS_KMAX);
    double *w = (double *)malloc(sizeof(double) * dim * 5);
    if (!T || !w) {
        free(T);
        free(w);
        return GO_EINVAL;
    }
    double *ynew = w + 4 * dim;
    int64_t pos = 0, total = (int64_t)1 << D;
    int d = 0;
    int rcode = GO_OK;
    while (pos < total) {
        double h = ldexp(H, -d);
        if (bs_attempt(s, y, h, ynew, T, w)) {
            if (s->tp_mode && s->rad) {
                int j = tp_collision(s, y, ynew, h);
                if (j > 0) {
                    *coll_member = j;
                    *coll_frac = ldexp((double)pos, -D);
                    *coll_h = h;
                    rcode = BS_COLLIDED;
                    break;
                }
            } else if (s->rad) {
                int ca, cb;
                if (group_collision(s, y, ynew, h, &ca, &cb)) {
                    *coll_member = ca;
                    *coll_b = cb;
                    *coll_frac = ldexp((double)pos, -D);
                    *coll_h = h;
                    rcode = BS_COLLIDED;
                    break;
                }
            }
            memcpy(y, ynew, sizeof(double) * dim);
            if (substeps) ++*substeps;
            pos += (int64_t)1 << (D - d);
            while (d > 0 && (pos % ((int64_t)1 << (D - d + 1))) == 0) --d;
        } else {
            ++d;
            if (d > D) {
                rcode = GO_EBS;
                break;
            }
        }
    }
    free(T);
    free(w);
    return rcode;
}

int go_bs_group(const go_params *p, int ng, const double *m, const double *rc,
                double *x, double *v, double H, int64_t *substeps) {
    double *y = (double *)malloc(sizeof(double) * 6 * ng);
    if (!y) return GO_EINVAL;
    for (int i = 0; i < ng; ++i)
        for (int k = 0; k < 3; ++k) {
            y[6 * i + k] = x[3 * i + k];
            y[6 * i + 3 + k] = v[3 * i + k];
        }
    ha_sys s = {p, ng, m, rc, 0, NULL};
    int cm = 0;
    double cf = 0.0;
    int rcode = bs_integrate(&s, y, H, substeps, &cm, &cf);
    for (int i = 0; i < ng; ++i)
        for (int k = 0; k < 3; ++k) {
            x[3 * i + k] = y[6 * i + k];
            v[3 * i + k] = y[6 * i + 3 + k];
        }
    free(y);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Total energy in democratic coordinates, H_A + H_B + H_C (Eqs. 1-3):
 *   E = sum m v^2/2 + |P|^2/(2 m0) - sum G m0 m_i/r_i - sum_{i<j} G m_i m_j/r_ij
 * and angular momentum L = sum m_i x_i x v_i (conserved by every sub-flow).
 * E_rel = |(E_t - E_0)/E_0| (Sec. 4.1) is formed by the caller.             */
void go_energy(const go_params *p, int n, const double *m, const double *x,
               const double *v, double *E, double *L) {
    double kin = 0.0, pot = 0.0, P[3] = {0, 0, 0}, Lv[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        const double *xi = V3(x, i), *vi = V3(v, i);
        kin += 0.5 * m[i] * dot3(vi, vi);
        pot -= p->G * p->m0 * m[i] / sqrt(dot3(xi, xi));
        for (int k = 0; k < 3; ++k) P[k] += m[i] * vi[k];
        Lv[0] += m[i] * (xi[1] * vi[2] - xi[2] * vi[1]);
        Lv[1] += m[i] * (xi[2] * vi[0] - xi[0] * vi[2]);
        Lv[2] += m[i] * (xi[0] * vi[1] - xi[1] * vi[0]);
        for (int j = i + 1; j < n; ++j) {
            const double *xj = V3(x, j);
            double d0 = xj[0] - xi[0], d1 = xj[1] - xi[1], d2 = xj[2] - xi[2];
            pot -= p->G * m[i] * m[j] / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        }
    }
    *E = kin + dot3(P, P) / (2.0 * p->m0) + pot;
    if (L) {
        L[0] = Lv[0];
        L[1] = Lv[1];
        L[2] = Lv[2];
    }
}

/* Heliocentric velocities u -> barycentric v (democratic coordinates,
 * Sec. 2.1): v_i = u_i - sum_j m_j u_j / (m0 + sum_j m_j).  In place.      */
void go_helio_to_dem(const go_params *p, int n, const double *m, double *v) {
    double S[3] = {0, 0, 0}, M = 0.0;
    for (int j = 0; j < n; ++j) {
        M += m[j];
        for (int k = 0; k < 3; ++k) S[k] += m[j] * v[3 * j + k];
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) v[3 * i + k] -= S[k] / (p->m0 + M);
}

/* Inverse: u_i = v_i + sum_j m_j v_j / m0.  In place. */
void go_dem_to_helio(const go_params *p, int n, const double *m, double *v) {
    double P[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < 3; ++k) P[k] += m[j] * v[3 * j + k];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) v[3 * i + k] += P[k] / p->m0;
}

/* ------------------------------------------------------------------------ */
/* Precheck (Sec. 2.2): candidate pairs are those closer than
 * pf * r_crit,ij at the end of a closing kick, i.e. at the start of the
 * next step.  cand is an n x n matrix; only i < j entries are used.        */
static void precheck(const go_params *p, int n, const double *x,
                     const double *rc, uint8_t *cand) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) cand[(size_t)i * n + j] = 0;
        for (int j = i + 1; j < n; ++j) {
            double d0 = x[3 * j] - x[3 * i], d1 = x[3 * j + 1] - x[3 * i + 1],
                   d2 = x[3 * j + 2] - x[3 * i + 2];
            double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
            cand[(size_t)i * n + j] = r < p->pf * rcij;
        }
    }
}

/* Initialisation (Sec. 2.2: the very first opening kick is computed on its
 * own): critical radii and the candidate set for the first step.           */
int go_massive_init(const go_params *p, int n, const double *m,
                    const double *x, const double *v, double *rc,
                    uint8_t *cand) {
    if (n < 1) return GO_EINVAL;
    go_rcrit(p, n, m, x, v, rc);
    if (!p->encounter_free) precheck(p, n, x, rc, cand);
    return GO_OK;
}

static int kick_half(const go_params *p, int n, const double *m, const double *x,
                     double *v, const double *rc, double *acc) {
    go_accel(p, n, m, x, rc, acc);
    double h = 0.5 * p->dt;
    for (int i = 0; i < 3 * n; ++i) v[i] += h * acc[i];
    return GO_OK;
}

static int drift_all(const go_params *p, int64_t n, double *x, double *v,
                     int64_t *itmax) {
    double mu = p->G * p->m0;
    int bad = 0;
    int64_t mx = 0;
#pragma omp parallel for schedule(static) reduction(| : bad) reduction(max : mx)
    for (int64_t i = 0; i < n; ++i) {
        int it = 0;
        if (go_kepler(mu, V3(x, i), V3(v, i), p->dt, V3(x, i), V3(v, i),
                      p->kepler_max_iter, &it) != GO_OK)
            bad = 1;
        if (it > mx) mx = it;
    }
    if (mx > *itmax) *itmax = mx;
    return bad ? GO_EKEPLER : GO_OK;
}

typedef struct {
    int32_t i, j;
    double d2, rc2;
} enc_rec;

/* One step of the second-order scheme, Eq. (7), following the step recipe of
 * Sec. 2.2 (both cases; the opening kick here recomputes all pairs):
 *  1 critical radii, 2 opening kick tau/2, 3 Sun kick tau/2, 4 Kepler drift
 *  tau, 5 encounter search, 6 grouping, 7 direct integration of each group
 *  from the pre-drift state, 8 Sun kick tau/2, 9 closing kick tau/2 with the
 *  precheck.  Reading: the closing kick and its precheck use the radii of
 *  step 1; an encounter is a candidate pair whose Hermite minimum is below
 *  r_crit,ij^2 (strict).                                                   */
/* Collision / ejection state of a main-mode run (NULL: none).             */
typedef struct {
    double *R, *S;
    int32_t *id;
    double rcut, rcut_sun;
    int64_t step;
    go_event *ev;
    int ev_cap, n_ev;
    double U;
    uint8_t *dead;
    double *gR, *gS;
} phys_ctx;

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Perfect merger (Sec. 3.2.7): mass and momentum add up, the new body sits
 * at the centre of mass with its velocity, and its spin is the two spins
 * plus the pair's orbital angular momentum about that centre (angular
 * momentum conservation); U is the paper's internal energy of the collision.
 * Reading: the radius is that of the merged volume (equal densities).      */
double go_merge(double G, double mi, double mj, const double *yi, const double *yj,
                double Ri, double Rj, const double *si, const double *sj, double *m_out,
                double *y_out, double *R_out, double *s_out) {
    double M = mi + mj;
    for (int k = 0; k < 6; ++k) y_out[k] = (mi * yi[k] + mj * yj[k]) / M;
    double di[3], ui[3], dj[3], uj[3], li[3], lj[3];
    for (int k = 0; k < 3; ++k) {
        di[k] = yi[k] - y_out[k];
        ui[k] = yi[3 + k] - y_out[3 + k];
        dj[k] = yj[k] - y_out[k];
        uj[k] = yj[3 + k] - y_out[3 + k];
    }
    cross3(di, ui, li);
    cross3(dj, uj, lj);
    for (int k = 0; k < 3; ++k) s_out[k] = si[k] + sj[k] + mi * li[k] + mj * lj[k];
    *m_out = M;
    *R_out = cbrt(Ri * Ri * Ri + Rj * Rj * Rj);
    double dv[3], dx[3];
    for (int k = 0; k < 3; ++k) {
        dv[k] = yi[3 + k] - yj[3 + k];
        dx[k] = yi[k] - yj[k];
    }
    return 0.5 * mi * mj / M * dot3(dv, dv) - G * mi * mj / sqrt(dot3(dx, dx));
}

static void put_event(phys_ctx *ph, const go_event *e) {
    if (ph->n_ev < ph->ev_cap) ph->ev[ph->n_ev] = *e;
    ++ph->n_ev;
}

/* BS of one group with mergers (Sec. 3.2.6-3.2.7).  Members (ascending body
 * index gi) with masses m, radii rc, physical radii R and spins S; states
 * in y (6 per member).  When a member pair touches, the integration stops at
 * the start of that BS substep (the last state before the collision), the
 * pair merges (the more massive body survives, the lower index on equal
 * masses, Sec. 3.2.7) and the group, one member fewer, is integrated over
 * the rest of the step afresh.  Reading: the merged body keeps the larger
 * critical radius of the two for the rest of the step.  *png: members left. */
static int bs_group_phys(const go_params *p, int *png, int32_t *gi, double *m, double *rc,
                         double *R, double *S, double *y, int64_t *substeps, phys_ctx *ph) {
    int ng = *png;
    double H = p->dt, f0 = 0.0;
    int rcode = GO_OK;
    for (;;) {
        ha_sys hs = {p, ng, m, rc, 0, R};
        int ca = 0, cb = 0;
        double cf = 0.0, ch = 0.0;
        int r = bs_integrate2(&hs, y, H, substeps, &ca, &cb, &cf, &ch);
        if (r != BS_COLLIDED) {
            rcode = r;
            break;
        }
        double frac = f0 + (1.0 - f0) * cf;
        int sv = m[cb] > m[ca] ? cb : ca, gh = sv == ca ? cb : ca;
        go_event e;
        memset(&e, 0, sizeof(e));
        e.kind = GO_EV_MERGE;
        e.id_i = ph->id[gi[sv]];
        e.id_j = ph->id[gi[gh]];
        e.step = ph->step;
        e.frac = frac;
        e.m_i = m[sv];
        e.m_j = m[gh];
        e.R_i = R[sv];
        e.R_j = R[gh];
        for (int k = 0; k < 3; ++k) {
            e.x_i[k] = y[6 * sv + k];
            e.v_i[k] = y[6 * sv + 3 + k];
            e.s_i[k] = S[3 * sv + k];
            e.x_j[k] = y[6 * gh + k];
            e.v_j[k] = y[6 * gh + 3 + k];
            e.s_j[k] = S[3 * gh + k];
        }
        double ym[6], Mm, Rm, sm[3];
        e.U = go_merge(p->G, m[sv], m[gh], &y[6 * sv], &y[6 * gh], R[sv], R[gh], &S[3 * sv],
                       &S[3 * gh], &Mm, ym, &Rm, sm);
        put_event(ph, &e);
        ph->U += e.U;
        memcpy(&y[6 * sv], ym, sizeof(ym));
        m[sv] = Mm;
        R[sv] = Rm;
        memcpy(&S[3 * sv], sm, sizeof(sm));
        rc[sv] = rc[sv] > rc[gh] ? rc[sv] : rc[gh];
        ph->dead[gi[gh]] = 1;
        for (int q = gh; q + 1 < ng; ++q) {
            gi[q] = gi[q + 1];
            m[q] = m[q + 1];
            rc[q] = rc[q + 1];
            R[q] = R[q + 1];
            memcpy(&S[3 * q], &S[3 * (q + 1)], 3 * sizeof(double));
            memcpy(&y[6 * q], &y[6 * (q + 1)], 6 * sizeof(double));
        }
        --ng;
        H = H * (1.0 - cf);
        f0 = frac;
    }
    *png = ng;
    return rcode;
}

/* Ejections (Sec. 3.2.8) after the direct integration: a body farther from
 * the central mass than rcut, or closer than rcut_sun, is reported and
 * removed.  Then the freed rows are filled (Sec. 3.4.6: the last body moves
 * into a deleted position), in descending row order.  Returns the new n.   */
static int remove_dead(const go_params *p, int n, double *m, double *x, double *v, double *rc,
                       phys_ctx *ph) {
    (void)p;
    for (int i = 0; i < n; ++i) {
        if (ph->dead[i]) continue;
        double r = sqrt(dot3(V3(x, i), V3(x, i)));
        int kind = 0;
        if (ph->rcut > 0.0 && r > ph->rcut) kind = GO_EV_EJECT_FAR;
        if (ph->rcut_sun > 0.0 && r < ph->rcut_sun) kind = GO_EV_EJECT_SUN;
        if (!kind) continue;
        go_event e;
        memset(&e, 0, sizeof(e));
        e.kind = kind;
        e.id_i = ph->id[i];
        e.id_j = -1;
        e.step = ph->step;
        e.frac = 1.0;
        e.m_i = m[i];
        e.R_i = ph->R[i];
        for (int k = 0; k < 3; ++k) {
            e.x_i[k] = x[3 * i + k];
            e.v_i[k] = v[3 * i + k];
            e.s_i[k] = ph->S[3 * i + k];
        }
        put_event(ph, &e);
        ph->dead[i] = 1;
    }
    for (int h = n - 1; h >= 0; --h) {
        if (!ph->dead[h]) continue;
        int last = n - 1;
        if (h != last) {
            m[h] = m[last];
            rc[h] = rc[last];
            ph->R[h] = ph->R[last];
            ph->id[h] = ph->id[last];
            memcpy(V3(x, h), V3(x, last), 3 * sizeof(double));
            memcpy(V3(v, h), V3(v, last), 3 * sizeof(double));
            memcpy(V3(ph->S, h), V3(ph->S, last), 3 * sizeof(double));
        }
        ph->dead[h] = 0;
        --n;
    }
    return n;
}

static int massive_step1(const go_params *p, int *pn, double *m, double *x,
                         double *v, double *rc, uint8_t *cand, go_stats *st,
                         enc_rec *enc, double *acc, double *xm, double *vm,
                         int32_t *pairs, int32_t *label, int32_t *order,
                         double *gx, double *gv, double *gm, double *grc,
                         phys_ctx *ph, int all_pairs) {
    int n = *pn;
    double h = 0.5 * p->dt;
    int rcode = GO_OK;
    if (p->encounter_free) {
        if (ph) return GO_EINVAL;
        kick_half(p, n, m, x, v, rc, acc);
        go_sun_drift(p, n, m, x, v, h);
        rcode = drift_all(p, n, x, v, &st->kepler_iter_max);
        go_sun_drift(p, n, m, x, v, h);
        kick_half(p, n, m, x, v, rc, acc);
        st->n_cand = st->n_enc = st->n_miss = st->n_groups = st->max_group = 0;
        return rcode;
    }
    /* 1 */
    go_rcrit(p, n, m, x, v, rc);
    int64_t ncand = 0;
    for (size_t k = 0; k < (size_t)n * n; ++k) ncand += cand[k];
    /* 2, 3 */
    kick_half(p, n, m, x, v, rc, acc);
    go_sun_drift(p, n, m, x, v, h);
    /* 4 */
    memcpy(xm, x, sizeof(double) * 3 * n);
    memcpy(vm, v, sizeof(double) * 3 * n);
    rcode = drift_all(p, n, x, v, &st->kepler_iter_max);
    if (rcode != GO_OK) return rcode;
    /* 5: Hermite test on every pair; method set = E and C */
    int64_t nenc = 0, nmiss = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            double dx0[3], dv0[3], dx1[3], dv1[3];
            for (int k = 0; k < 3; ++k) {
                dx0[k] = xm[3 * j + k] - xm[3 * i + k];
                dv0[k] = vm[3 * j + k] - vm[3 * i + k];
                dx1[k] = x[3 * j + k] - x[3 * i + k];
                dv1[k] = v[3 * j + k] - v[3 * i + k];
            }
            double d2 = go_hermite_dmin2(p->dt, dx0, dv0, dx1, dv1);
            double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
            if (d2 < rcij * rcij) {
                if (all_pairs || cand[(size_t)i * n + j]) {
                    enc[nenc].i = i;
                    enc[nenc].j = j;
                    enc[nenc].d2 = d2;
                    enc[nenc].rc2 = rcij * rcij;
                    ++nenc;
                } else {
                    ++nmiss;
                }
            }
        }
    }
    st->n_cand = ncand;
    st->n_enc = nenc;
    st->n_miss = nmiss;
    st->enc_total += nenc;
    st->miss_total += nmiss;
    st->n_groups = 0;
    st->max_group = 0;
    if (nenc > 0) {
        /* 6 */
        for (int64_t e = 0; e < nenc; ++e) {
            pairs[2 * e] = enc[e].i;
            pairs[2 * e + 1] = enc[e].j;
        }
        int ngr = go_groups(n, (int)nenc, pairs, label);
        st->n_groups = ngr;
        /* 7: each group, in order of its label, members ascending */
        for (int g = 0; g < n; ++g) {
            if (label[g] != g) continue;
            int ng = 0;
            for (int i = g; i < n; ++i)
                if (label[i] == g) order[ng++] = i;
            if (ng > st->max_group) st->max_group = ng;
            for (int q = 0; q < ng; ++q) {
                int i = order[q];
                for (int k = 0; k < 3; ++k) {
                    gx[3 * q + k] = xm[3 * i + k];
                    gv[3 * q + k] = vm[3 * i + k];
                }
                gm[q] = m[i];
                grc[q] = rc[i];
            }
            if (!ph) {
                int rc2 = go_bs_group(p, ng, gm, grc, gx, gv, p->dt, &st->bs_substeps);
                if (rc2 != GO_OK) return rc2;
                for (int q = 0; q < ng; ++q) {
                    int i = order[q];
                    for (int k = 0; k < 3; ++k) {
                        x[3 * i + k] = gx[3 * q + k];
                        v[3 * i + k] = gv[3 * q + k];
                    }
                }
            } else {
                /* y holds x, v per member in gx (6 per member) */
                double *y = gx;
                for (int q = ng - 1; q >= 0; --q) {
                    int i = order[q];
                    for (int k = 0; k < 3; ++k) {
                        y[6 * q + k] = xm[3 * i + k];
                        y[6 * q + 3 + k] = vm[3 * i + k];
                    }
                    ph->gR[q] = ph->R[i];
                    for (int k = 0; k < 3; ++k) ph->gS[3 * q + k] = ph->S[3 * i + k];
                }
                int ngl = ng;
                int rc2 = bs_group_phys(p, &ngl, order, gm, grc, ph->gR, ph->gS, y,
                                        &st->bs_substeps, ph);
                if (rc2 != GO_OK) return rc2;
                for (int q = 0; q < ngl; ++q) {
                    int i = order[q];
                    for (int k = 0; k < 3; ++k) {
                        x[3 * i + k] = y[6 * q + k];
                        v[3 * i + k] = y[6 * q + 3 + k];
                        ph->S[3 * i + k] = ph->gS[3 * q + k];
                    }
                    m[i] = gm[q];
                    rc[i] = grc[q];
                    ph->R[i] = ph->gR[q];
                }
            }
        }
    }
    /* do collisions: absorbed bodies and ejections leave (Sec. 3.2.7-3.2.8) */
    if (ph) {
        n = remove_dead(p, n, m, x, v, rc, ph);
        *pn = n;
    }
    /* 8, 9 */
    go_sun_drift(p, n, m, x, v, h);
    kick_half(p, n, m, x, v, rc, acc);
    precheck(p, n, x, rc, cand);
    return GO_OK;
}

int go_massive_step(const go_params *p, int n, const double *m, double *x,
                    double *v, double *rc, uint8_t *cand, int64_t nsteps,
                    go_stats *st, int enc_cap, int32_t *enc_ij,
                    double *enc_d2, double *enc_rc2, int *n_enc) {
    if (n < 1 || nsteps < 0) return GO_EINVAL;
    go_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    size_t N = (size_t)n;
    enc_rec *enc = (enc_rec *)malloc(sizeof(enc_rec) * (N * (N - 1) / 2 + 1));
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    double *xm = (double *)malloc(sizeof(double) * 3 * N);
    double *vm = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (N * (N - 1) + 2));
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
    double *gx = (double *)malloc(sizeof(double) * 3 * N);
    double *gv = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = (double *)malloc(sizeof(double) * N);
    double *grc = (double *)malloc(sizeof(double) * N);
    int rcode = GO_OK;
    if (!enc || !acc || !xm || !vm || !pairs || !label || !order || !gx || !gv ||
        !gm || !grc) {
        rcode = GO_EINVAL;
    } else {
        for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
            int nn = n;
            rcode = massive_step1(p, &nn, (double *)m, x, v, rc, cand, st, enc, acc, xm, vm,
                                  pairs, label, order, gx, gv, gm, grc, NULL, 0);
            if (rcode == GO_OK) ++st->steps;
        }
        if (n_enc) {
            *n_enc = (int)(nsteps > 0 ? st->n_enc : 0);
            if (nsteps > 0 && enc_ij) {
                int64_t lim = st->n_enc < enc_cap ? st->n_enc : enc_cap;
                for (int64_t e = 0; e < lim; ++e) {
                    enc_ij[2 * e] = enc[e].i;
                    enc_ij[2 * e + 1] = enc[e].j;
                    if (enc_d2) enc_d2[e] = enc[e].d2;
                    if (enc_rc2) enc_rc2[e] = enc[e].rc2;
                }
                if (st->n_enc > enc_cap && rcode == GO_OK) rcode = GO_EOVERFLOW;
            }
        }
    }
    free(enc);
    free(acc);
    free(xm);
    free(vm);
    free(pairs);
    free(label);
    free(order);
    free(gx);
    free(gv);
    free(gm);
    free(grc);
    return rcode;
}

int go_massive_step_phys(const go_params *p, int *pn, double *m, double *x, double *v,
                         double *rc, uint8_t *cand, int64_t nsteps, go_stats *st,
                         double *R, double *S, int32_t *id, double rcut, double rcut_sun,
                         int nmin, int64_t step0, go_event *ev, int ev_cap, int *n_ev,
                         double *U) {
    if (!pn || *pn < 1 || nsteps < 0 || !R || !S || !id || !U || ev_cap < 0) return GO_EINVAL;
    if (p->encounter_free || (ev_cap > 0 && !ev)) return GO_EINVAL;
    go_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    size_t N = (size_t)*pn;
    enc_rec *enc = (enc_rec *)malloc(sizeof(enc_rec) * (N * (N - 1) / 2 + 1));
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    double *xm = (double *)malloc(sizeof(double) * 3 * N);
    double *vm = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (N * (N - 1) + 2));
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
    double *gx = (double *)malloc(sizeof(double) * 6 * N);
    double *gv = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = (double *)malloc(sizeof(double) * N);
    double *grc = (double *)malloc(sizeof(double) * N);
    double *gR = (double *)malloc(sizeof(double) * N);
    double *gS = (double *)malloc(sizeof(double) * 3 * N);
    uint8_t *dead = (uint8_t *)calloc(N, 1);
    phys_ctx ph = {R, S, id, rcut, rcut_sun, step0, ev, ev_cap, 0, *U, dead, gR, gS};
    int rcode = GO_OK;
    if (!enc || !acc || !xm || !vm || !pairs || !label || !order || !gx || !gv || !gm ||
        !grc || !gR || !gS || !dead) {
        rcode = GO_EINVAL;
    } else {
        for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
            ph.step = step0 + s;
            rcode = massive_step1(p, pn, m, x, v, rc, cand, st, enc, acc, xm, vm, pairs, label,
                                  order, gx, gv, gm, grc, &ph, 0);
            if (rcode == GO_OK) {
                ++st->steps;
                if (*pn < nmin) rcode = GO_STOPPED;
            }
        }
    }
    *U = ph.U;
    if (n_ev) *n_ev = ph.n_ev;
    if (rcode == GO_OK && ph.n_ev > ev_cap) rcode = GO_EOVERFLOW;
    free(enc);
    free(acc);
    free(xm);
    free(vm);
    free(pairs);
    free(label);
    free(order);
    free(gx);
    free(gv);
    free(gm);
    free(grc);
    free(gR);
    free(gS);
    free(dead);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Higher orders (Sec. 2.3): the step is a symmetric composition of the
 * second-order step with sub-steps w_k tau (Yoshida 1990; fourth order:
 * w1, w0, w1 with w1 = 1/(2 - 2^(1/3)), w0 = 1 - 2 w1; sixth order, his
 * solution A: w3, w2, w1, w0, w1, w2, w3 with w0 = 1 - 2 (w1 + w2 + w3)).
 * Some sub-steps run backward in time.  Each sub-step is the full hybrid
 * scheme -- critical radii with |w_k tau|, kicks, drift, encounter search,
 * grouping, BS -- except the prechecker: its candidates come from the
 * previous sub-step's closing kick, which is not synchronous with this
 * sub-step's drift, so every pair takes the Hermite test (Reading: "without
 * the prechecker" means the encounter set is E over all pairs, not E and C).
 * order 2 is the plain step.                                               */
int go_composition(int order, double *w) {
    if (order == 2) {
        w[0] = 1.0;
        return 1;
    }
    if (order == 4) {
        double c = cbrt(2.0);
        w[0] = w[2] = 1.0 / (2.0 - c);
        w[1] = 1.0 - 2.0 * w[0];
        return 3;
    }
    if (order == 6) {
        double w1 = -1.17767998417887, w2 = 0.235573213359357, w3 = 0.784513610477560;
        double w0 = 1.0 - 2.0 * (w1 + w2 + w3);
        double q[7] = {w3, w2, w1, w0, w1, w2, w3};
        memcpy(w, q, sizeof(q));
        return 7;
    }
    return 0;
}

int go_massive_step_order(const go_params *p, int order, int n, const double *m, double *x,
                          double *v, double *rc, int64_t nsteps, go_stats *st) {
    double w[7];
    int K = go_composition(order, w);
    if (K == 0 || n < 1 || nsteps < 0) return GO_EINVAL;
    go_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    size_t N = (size_t)n;
    enc_rec *enc = (enc_rec *)malloc(sizeof(enc_rec) * (N * (N - 1) / 2 + 1));
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    double *xm = (double *)malloc(sizeof(double) * 3 * N);
    double *vm = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (N * (N - 1) + 2));
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order_ = (int32_t *)malloc(sizeof(int32_t) * N);
    double *gx = (double *)malloc(sizeof(double) * 3 * N);
    double *gv = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = (double *)malloc(sizeof(double) * N);
    double *grc = (double *)malloc(sizeof(double) * N);
    uint8_t *cand = (uint8_t *)calloc(N * N, 1);
    int rcode = GO_OK;
    if (!enc || !acc || !xm || !vm || !pairs || !label || !order_ || !gx || !gv || !gm ||
        !grc || !cand) {
        rcode = GO_EINVAL;
    } else {
        go_stats sub;
        for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
            for (int k = 0; k < K && rcode == GO_OK; ++k) {
                go_params q = *p;
                q.dt = w[k] * p->dt;
                memset(&sub, 0, sizeof(sub));
                int nn = n;
                rcode = massive_step1(&q, &nn, (double *)m, x, v, rc, cand, &sub, enc, acc, xm,
                                      vm, pairs, label, order_, gx, gv, gm, grc, NULL, 1);
                st->enc_total += sub.enc_total;
                st->bs_substeps += sub.bs_substeps;
                if (sub.kepler_iter_max > st->kepler_iter_max)
                    st->kepler_iter_max = sub.kepler_iter_max;
                st->n_enc = sub.n_enc;
                st->n_groups = sub.n_groups;
                st->max_group = sub.max_group;
            }
            if (rcode == GO_OK) ++st->steps;
        }
    }
    free(enc);
    free(acc);
    free(xm);
    free(vm);
    free(pairs);
    free(label);
    free(order_);
    free(gx);
    free(gv);
    free(gm);
    free(grc);
    free(cand);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Test-particle mode (Sec. 3.3): massless particles feel the massive bodies
 * but not each other and exert nothing.  The Sun kick uses the momentum of
 * the massive bodies only and is applied to the test particles as well.
 * A test particle's critical radius has no Hill term (m = 0).  Each
 * test-particle encounter forms its own group: the particle together with
 * the massive bodies it encounters, integrated from the pre-drift state;
 * only the particle is written back (the massive bodies keep their own
 * result).  Reading: in that group the massive bodies feel only the star
 * (their mutual terms belong to their own groups).                         */
static void tp_accel(const go_params *p, int nm, const double *m,
                     const double *x, const double *rc, const double *xt,
                     double rct, double *a) {
    a[0] = a[1] = a[2] = 0.0;
    for (int j = 0; j < nm; ++j) {
        double d0 = x[3 * j] - xt[0], d1 = x[3 * j + 1] - xt[1],
               d2 = x[3 * j + 2] - xt[2];
        double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        double r = sqrt(r2);
        double f;
        if (p->encounter_free) {
            f = 1.0 / (r2 * r);
        } else {
            double rcij = rct > rc[j] ? rct : rc[j];
            double K, dK;
            pair_K(r, rcij, &K, &dK);
            f = K / (r2 * r) - dK / r2;
        }
        double s = p->G * m[j] * f;
        a[0] += s * d0;
        a[1] += s * d1;
        a[2] += s * d2;
    }
}

static double tp_rcrit(const go_params *p, const double *vt) {
    return p->n2 * fabs(p->dt) * sqrt(dot3(vt, vt));
}

static void tp_precheck(const go_params *p, int nm, const double *x,
                        const double *rc, const double *xt, double rct,
                        uint8_t *c) {
    for (int j = 0; j < nm; ++j) {
        double d0 = x[3 * j] - xt[0], d1 = x[3 * j + 1] - xt[1],
               d2 = x[3 * j + 2] - xt[2];
        double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        double rcij = rct > rc[j] ? rct : rc[j];
        c[j] = r < p->pf * rcij;
    }
}

int go_tp_init(const go_params *p, int nm, const double *m, const double *x,
               const double *v, double *rc, uint8_t *cand, int64_t ntp,
               const double *xt, const double *vt, uint8_t *cand_tp) {
    int r = go_massive_init(p, nm, m, x, v, rc, cand);
    if (r != GO_OK) return r;
    if (p->encounter_free) return GO_OK;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ntp; ++k)
        tp_precheck(p, nm, x, rc, V3(xt, k), tp_rcrit(p, V3(vt, k)),
                    &cand_tp[(size_t)k * nm]);
    return GO_OK;
}

int go_tp_step(const go_params *p, int nm, const double *m, double *x,
               double *v, double *rc, uint8_t *cand, int64_t ntp, double *xt,
               double *vt, uint8_t *cand_tp, int64_t nsteps, go_stats *st,
               const double *rad, int64_t step0, int32_t *coll_planet,
               int64_t *coll_step, double *coll_frac, double *coll_xv,
               double *tp_d2, double *tp_rc2) {
    if (nm < 1 || nm > 64 || ntp < 0 || nsteps < 0) return GO_EINVAL;
    if ((tp_d2 == NULL) != (tp_rc2 == NULL)) return GO_EINVAL;
    if (rad && (!coll_planet || !coll_step || !coll_frac || !coll_xv)) return GO_EINVAL;
    go_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    size_t N = (size_t)nm;
    double h = 0.5 * p->dt;
    double mu = p->G * p->m0;
    /* massive-body work buffers */
    enc_rec *enc = (enc_rec *)malloc(sizeof(enc_rec) * (N * (N - 1) / 2 + 1));
    double *acc = (double *)malloc(sizeof(double) * 3 * N);
    double *xm = (double *)malloc(sizeof(double) * 3 * N);
    double *vm = (double *)malloc(sizeof(double) * 3 * N);
    double *x0 = (double *)malloc(sizeof(double) * 3 * N);
    double *xe = (double *)malloc(sizeof(double) * 3 * N);
    double *ve = (double *)malloc(sizeof(double) * 3 * N);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * (N * (N - 1) + 2));
    int32_t *label = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * N);
    double *gx = (double *)malloc(sizeof(double) * 3 * N);
    double *gv = (double *)malloc(sizeof(double) * 3 * N);
    double *gm = (double *)malloc(sizeof(double) * N);
    double *grc = (double *)malloc(sizeof(double) * N);
    int rcode = GO_OK;
    if (!enc || !acc || !xm || !vm || !x0 || !xe || !ve || !pairs || !label ||
        !order || !gx || !gv || !gm || !grc)
        rcode = GO_EINVAL;
    for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
        /* the massive bodies' own step, keeping the states the particles
         * need: start positions x0, pre-drift (xm, vm), post-drift (xe, ve) */
        memcpy(x0, x, sizeof(double) * 3 * N);
        go_rcrit(p, nm, m, x, v, rc);
        kick_half(p, nm, m, x, v, rc, acc);
        double P1[3] = {0, 0, 0};
        for (int j = 0; j < nm; ++j)
            for (int k = 0; k < 3; ++k) P1[k] += m[j] * v[3 * j + k];
        go_sun_drift(p, nm, m, x, v, h);
        memcpy(xm, x, sizeof(double) * 3 * N);
        memcpy(vm, v, sizeof(double) * 3 * N);
        rcode = drift_all(p, nm, x, v, &st->kepler_iter_max);
        if (rcode != GO_OK) break;
        memcpy(xe, x, sizeof(double) * 3 * N);
        memcpy(ve, v, sizeof(double) * 3 * N);
        int64_t nenc = 0, nmiss = 0, ncand = 0;
        if (!p->encounter_free) {
            for (size_t k = 0; k < N * N; ++k) ncand += cand[k];
            for (int i = 0; i < nm; ++i)
                for (int j = i + 1; j < nm; ++j) {
                    double dx0[3], dv0[3], dx1[3], dv1[3];
                    for (int k = 0; k < 3; ++k) {
                        dx0[k] = xm[3 * j + k] - xm[3 * i + k];
                        dv0[k] = vm[3 * j + k] - vm[3 * i + k];
                        dx1[k] = x[3 * j + k] - x[3 * i + k];
                        dv1[k] = v[3 * j + k] - v[3 * i + k];
                    }
                    double d2 = go_hermite_dmin2(p->dt, dx0, dv0, dx1, dv1);
                    double rcij = rc[i] > rc[j] ? rc[i] : rc[j];
                    if (d2 < rcij * rcij) {
                        if (cand[(size_t)i * nm + j]) {
                            enc[nenc].i = i;
                            enc[nenc].j = j;
                            ++nenc;
                        } else {
                            ++nmiss;
                        }
                    }
                }
        }
        st->n_cand = ncand;
        st->n_enc = nenc;
        st->n_miss = nmiss;
        st->enc_total += nenc;
        st->miss_total += nmiss;
        st->n_groups = st->max_group = 0;
        if (nenc > 0) {
            for (int64_t e = 0; e < nenc; ++e) {
                pairs[2 * e] = enc[e].i;
                pairs[2 * e + 1] = enc[e].j;
            }
            st->n_groups = go_groups(nm, (int)nenc, pairs, label);
            for (int g = 0; g < nm && rcode == GO_OK; ++g) {
                if (label[g] != g) continue;
                int ng = 0;
                for (int i = g; i < nm; ++i)
                    if (label[i] == g) order[ng++] = i;
                if (ng > st->max_group) st->max_group = ng;
                for (int q = 0; q < ng; ++q) {
                    int i = order[q];
                    for (int k = 0; k < 3; ++k) {
                        gx[3 * q + k] = xm[3 * i + k];
                        gv[3 * q + k] = vm[3 * i + k];
                    }
                    gm[q] = m[i];
                    grc[q] = rc[i];
                }
                rcode = go_bs_group(p, ng, gm, grc, gx, gv, p->dt, &st->bs_substeps);
                for (int q = 0; q < ng; ++q) {
                    int i = order[q];
                    for (int k = 0; k < 3; ++k) {
                        x[3 * i + k] = gx[3 * q + k];
                        v[3 * i + k] = gv[3 * q + k];
                    }
                }
            }
            if (rcode != GO_OK) break;
        }
        double P2[3] = {0, 0, 0};
        for (int j = 0; j < nm; ++j)
            for (int k = 0; k < 3; ++k) P2[k] += m[j] * v[3 * j + k];
        go_sun_drift(p, nm, m, x, v, h);
        kick_half(p, nm, m, x, v, rc, acc);
        if (!p->encounter_free) precheck(p, nm, x, rc, cand);

        /* the test particles, each on its own (they do not interact) */
        int64_t tpenc = 0, bssub = 0, nrem = 0;
        int bad = 0;
        int64_t itmx = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : tpenc, bssub, nrem) \
    reduction(| : bad) reduction(max : itmx)
        for (int64_t k = 0; k < ntp; ++k) {
            double *xk = V3(xt, k), *vk = V3(vt, k);
            if (tp_d2)
                for (int j = 0; j < nm; ++j)
                    tp_d2[(size_t)k * nm + j] = tp_rc2[(size_t)k * nm + j] = NAN;
            if (isnan(xk[0])) continue; /* removed earlier */
            double rct = tp_rcrit(p, vk);
            double a[3];
            tp_accel(p, nm, m, x0, rc, xk, rct, a);
            for (int q = 0; q < 3; ++q) vk[q] += h * a[q];
            for (int q = 0; q < 3; ++q) xk[q] += h * P1[q] / p->m0;
            double xkm[3] = {xk[0], xk[1], xk[2]}, vkm[3] = {vk[0], vk[1], vk[2]};
            int it = 0;
            if (go_kepler(mu, xk, vk, p->dt, xk, vk, p->kepler_max_iter, &it) != GO_OK)
                bad = 1;
            if (it > itmx) itmx = it;
            if (!p->encounter_free) {
                int sel[64], ns = 0;
                uint8_t *ck = &cand_tp[(size_t)k * nm];
                for (int j = 0; j < nm; ++j) {
                    if (!ck[j]) continue;
                    double dx0[3], dv0[3], dx1[3], dv1[3];
                    for (int q = 0; q < 3; ++q) {
                        dx0[q] = xm[3 * j + q] - xkm[q];
                        dv0[q] = vm[3 * j + q] - vkm[q];
                        dx1[q] = xe[3 * j + q] - xk[q];
                        dv1[q] = ve[3 * j + q] - vk[q];
                    }
                    double d2 = go_hermite_dmin2(p->dt, dx0, dv0, dx1, dv1);
                    double rcij = rct > rc[j] ? rct : rc[j];
                    if (tp_d2) {
                        tp_d2[(size_t)k * nm + j] = d2;
                        tp_rc2[(size_t)k * nm + j] = rcij * rcij;
                    }
                    if (d2 < rcij * rcij) sel[ns++] = j;
                }
                if (ns > 0) {
                    tpenc += ns;
                    int ngp = ns + 1;
                    double ym[6 * 65];
                    double mg[65], rg[65];
                    for (int q = 0; q < 3; ++q) {
                        ym[q] = xkm[q];
                        ym[3 + q] = vkm[q];
                    }
                    double radg[65];
                    mg[0] = 0.0;
                    rg[0] = rct;
                    radg[0] = rad ? rad[nm + k] : 0.0;
                    for (int t = 0; t < ns; ++t) {
                        int j = sel[t];
                        for (int q = 0; q < 3; ++q) {
                            ym[6 * (t + 1) + q] = xm[3 * j + q];
                            ym[6 * (t + 1) + 3 + q] = vm[3 * j + q];
                        }
                        mg[t + 1] = m[j];
                        rg[t + 1] = rc[j];
                        radg[t + 1] = rad ? rad[j] : 0.0;
                    }
                    ha_sys hs = {p, ngp, mg, rg, 1, rad ? radg : NULL};
                    int64_t sub = 0;
                    int cm = 0;
                    double cf = 0.0;
                    int rb = bs_integrate(&hs, ym, p->dt, &sub, &cm, &cf);
                    bssub += sub;
                    if (rb == BS_COLLIDED) {
                        /* removed: report the state before the colliding substep */
                        coll_planet[k] = sel[cm - 1];
                        coll_step[k] = step0 + s;
                        coll_frac[k] = cf;
                        for (int q = 0; q < 6; ++q) coll_xv[6 * k + q] = ym[q];
                        for (int q = 0; q < 3; ++q) xk[q] = vk[q] = NAN;
                        memset(&cand_tp[(size_t)k * nm], 0, (size_t)nm);
                        ++nrem;
                        continue;
                    }
                    if (rb != GO_OK) bad = 2;
                    for (int q = 0; q < 3; ++q) {
                        xk[q] = ym[q];
                        vk[q] = ym[3 + q];
                    }
                }
            }
            for (int q = 0; q < 3; ++q) xk[q] += h * P2[q] / p->m0;
            tp_accel(p, nm, m, x, rc, xk, rct, a);
            for (int q = 0; q < 3; ++q) vk[q] += h * a[q];
            if (!p->encounter_free)
                tp_precheck(p, nm, x, rc, xk, rct, &cand_tp[(size_t)k * nm]);
        }
        st->tp_enc = tpenc;
        st->tp_enc_total += tpenc;
        st->tp_removed += nrem;
        st->bs_substeps += bssub;
        if (itmx > st->kepler_iter_max) st->kepler_iter_max = itmx;
        if (bad) {
            rcode = bad == 2 ? GO_EBS : GO_EKEPLER;
            break;
        }
        ++st->steps;
    }
    free(enc);
    free(acc);
    free(xm);
    free(vm);
    free(x0);
    free(xe);
    free(ve);
    free(pairs);
    free(label);
    free(order);
    free(gx);
    free(gv);
    free(gm);
    free(grc);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Encounter-free map (K = 1, the MVS map in democratic coordinates, Sec.
 * 2.1): kick tau/2, Sun kick tau/2, drift tau, Sun kick tau/2, kick tau/2.  */
int go_free_step(const go_params *p, int n, const double *m, double *x,
                 double *v, int64_t nsteps) {
    go_params q = *p;
    q.encounter_free = 1;
    double *acc = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!acc) return GO_EINVAL;
    int64_t itmax = 0;
    int rcode = GO_OK;
    double h = 0.5 * q.dt;
    for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
        kick_half(&q, n, m, x, v, NULL, acc);
        go_sun_drift(&q, n, m, x, v, h);
        rcode = drift_all(&q, n, x, v, &itmax);
        go_sun_drift(&q, n, m, x, v, h);
        kick_half(&q, n, m, x, v, NULL, acc);
    }
    free(acc);
    return rcode;
}

/* Tangent-linear model of one drift (forward-mode derivative of the
 * universal-variable map above).  The converged s satisfies F(s) = 0, so
 * by the implicit function theorem
 *   ds = -(G1 dr0 + G2 deta0 + F_beta dbeta) / r,
 * with dG_k/ds = G_{k-1} (dG_0/ds = -beta G1) and
 * dG_k/dbeta = (k G_{k+2} - s G_{k+1}) / 2.
 * Pinned by central finite differences.                                    */
static int kepler_tlm(double mu, const double *x0, const double *v0, double dt,
                      const double *dx0, const double *dv0, double *x,
                      double *v, double *dx, double *dv, int max_iter) {
    double r0 = sqrt(dot3(x0, x0));
    double eta0 = dot3(x0, v0);
    double vv = dot3(v0, v0);
    double beta = 2.0 * mu / r0 - vv;
    double s;
    int rcode = kepler_solve(mu, r0, eta0, beta, dt, max_iter, &s, NULL);
    double z = beta * s * s;
    double c[4], c4, c5;
    go_stumpff(z, c);
    stumpff45(z, c, &c4, &c5);
    double G0 = c[0], G1 = s * c[1], G2 = s * s * c[2], G3 = s * s * s * c[3];
    double G4 = s * s * s * s * c4, G5 = s * s * s * s * s * c5;
    double r = r0 * G0 + eta0 * G1 + mu * G2;
    double f = 1.0 - mu * G2 / r0, g = dt - mu * G3;
    double fd = -mu * G1 / (r * r0), gd = 1.0 - mu * G2 / r;
    /* input differentials */
    double dr0 = dot3(x0, dx0) / r0;
    double deta0 = dot3(dx0, v0) + dot3(x0, dv0);
    double dbeta = -2.0 * mu * dr0 / (r0 * r0) - 2.0 * dot3(v0, dv0);
    double dG1b = 0.5 * (1.0 * G3 - s * G2);
    double dG2b = 0.5 * (2.0 * G4 - s * G3);
    double dG3b = 0.5 * (3.0 * G5 - s * G4);
    double dG0b = 0.5 * (0.0 - s * G1);
    double Fb = r0 * dG1b + eta0 * dG2b + mu * dG3b;
    double ds = -(G1 * dr0 + G2 * deta0 + Fb * dbeta) / r;
    double dG0 = -beta * G1 * ds + dG0b * dbeta;
    double dG1 = G0 * ds + dG1b * dbeta;
    double dG2 = G1 * ds + dG2b * dbeta;
    double dG3 = G2 * ds + dG3b * dbeta;
    double dr = dr0 * G0 + r0 * dG0 + deta0 * G1 + eta0 * dG1 + mu * dG2;
    double df = -mu * dG2 / r0 + mu * G2 * dr0 / (r0 * r0);
    double dg = -mu * dG3;
    double dfd = -mu * (dG1 / (r * r0) - G1 * (dr * r0 + r * dr0) / ((r * r0) * (r * r0)));
    double dgd = -mu * (dG2 / r - G2 * dr / (r * r));
    double xn[3], vn[3], dxn[3], dvn[3];
    for (int k = 0; k < 3; ++k) {
        xn[k] = f * x0[k] + g * v0[k];
        vn[k] = fd * x0[k] + gd * v0[k];
        dxn[k] = df * x0[k] + f * dx0[k] + dg * v0[k] + g * dv0[k];
        dvn[k] = dfd * x0[k] + fd * dx0[k] + dgd * v0[k] + gd * dv0[k];
    }
    for (int k = 0; k < 3; ++k) {
        x[k] = xn[k];
        v[k] = vn[k];
        dx[k] = dxn[k];
        dv[k] = dvn[k];
    }
    return rcode;
}

/* Tangent-linear model of one encounter-free step, in place: the
 * derivatives (dx, dv) for input perturbations (dx, dv, dm) are carried
 * through kick, Sun kick, drift, Sun kick, kick. */
static void kick_tlm(const go_params *p, int n, const double *m,
                     const double *dm, const double *x, double *v,
                     const double *dx, double *dv, double *acc, double *dacc) {
    double h = 0.5 * p->dt;
    double G = p->G;
    for (int i = 0; i < n; ++i) {
        double a[3] = {0, 0, 0}, da[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3], dd[3];
            for (int k = 0; k < 3; ++k) {
                d[k] = x[3 * j + k] - x[3 * i + k];
                dd[k] = dx[3 * j + k] - dx[3 * i + k];
            }
            double r2 = dot3(d, d);
            double r = sqrt(r2);
            double ir3 = 1.0 / (r2 * r);
            double ddot = dot3(d, dd);
            for (int k = 0; k < 3; ++k) {
                a[k] += G * m[j] * d[k] * ir3;
                da[k] += G * dm[j] * d[k] * ir3 +
                         G * m[j] * (dd[k] * ir3 - 3.0 * d[k] * ddot * ir3 / r2);
            }
        }
        for (int k = 0; k < 3; ++k) {
            acc[3 * i + k] = a[k];
            dacc[3 * i + k] = da[k];
        }
    }
    for (int i = 0; i < 3 * n; ++i) {
        v[i] += h * acc[i];
        dv[i] += h * dacc[i];
    }
}

static void sun_tlm(const go_params *p, int n, const double *m,
                    const double *dm, double *x, const double *v, double *dx,
                    const double *dv) {
    double h = 0.5 * p->dt;
    double P[3] = {0, 0, 0}, dP[3] = {0, 0, 0};
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < 3; ++k) {
            P[k] += m[j] * v[3 * j + k];
            dP[k] += dm[j] * v[3 * j + k] + m[j] * dv[3 * j + k];
        }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            x[3 * i + k] += h * P[k] / p->m0;
            dx[3 * i + k] += h * dP[k] / p->m0;
        }
}

static int free_step_tlm1(const go_params *p, int n, const double *m,
                          const double *dm, double *x, double *v, double *dx,
                          double *dv, double *acc, double *dacc) {
    double mu = p->G * p->m0;
    kick_tlm(p, n, m, dm, x, v, dx, dv, acc, dacc);
    sun_tlm(p, n, m, dm, x, v, dx, dv);
    for (int i = 0; i < n; ++i) {
        int r = kepler_tlm(mu, V3(x, i), V3(v, i), p->dt, V3(dx, i), V3(dv, i),
                           V3(x, i), V3(v, i), V3(dx, i), V3(dv, i),
                           p->kepler_max_iter);
        if (r != GO_OK) return r;
    }
    sun_tlm(p, n, m, dm, x, v, dx, dv);
    kick_tlm(p, n, m, dm, x, v, dx, dv, acc, dacc);
    return GO_OK;
}

int go_free_tlm(const go_params *p, int n, const double *m, const double *x0,
                const double *v0, const double *dm, const double *dx0,
                const double *dv0, int64_t nsteps, double *xT, double *vT,
                double *dxT, double *dvT) {
    size_t N3 = 3 * (size_t)n;
    double *acc = (double *)malloc(sizeof(double) * N3);
    double *dacc = (double *)malloc(sizeof(double) * N3);
    if (!acc || !dacc) {
        free(acc);
        free(dacc);
        return GO_EINVAL;
    }
    memcpy(xT, x0, sizeof(double) * N3);
    memcpy(vT, v0, sizeof(double) * N3);
    memcpy(dxT, dx0, sizeof(double) * N3);
    memcpy(dvT, dv0, sizeof(double) * N3);
    int rcode = GO_OK;
    for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s)
        rcode = free_step_tlm1(p, n, m, dm, xT, vT, dxT, dvT, acc, dacc);
    free(acc);
    free(dacc);
    return rcode;
}

/* Adjoint (reverse-mode gradient) of the encounter-free map: by definition
 * the transpose of the tangent-linear map.  Plainly: store the state at the
 * start of every step; walking the steps backwards, form the Jacobian of
 * the step column by column with the tangent-linear model (inputs x, v, m;
 * outputs x, v) and apply its transpose to the incoming gradient.  The
 * mass gradient is the sum over steps of the mass columns' contributions. */
int go_free_adjoint(const go_params *p, int n, const double *m,
                    const double *x0, const double *v0, int64_t nsteps,
                    const double *gxT, const double *gvT, double *gx0,
                    double *gv0, double *gm) {
    size_t N3 = 3 * (size_t)n;
    size_t nin = 7 * (size_t)n, nout = 6 * (size_t)n;
    double *states = (double *)malloc(sizeof(double) * 6 * (size_t)n * (size_t)(nsteps + 1));
    double *J = (double *)malloc(sizeof(double) * nin * nout);
    double *w = (double *)malloc(sizeof(double) * (8 * N3 + 2 * (size_t)n + nout + nin));
    if (!states || !J || !w) {
        free(states);
        free(J);
        free(w);
        return GO_EINVAL;
    }
    double *xs = w, *vs = w + N3, *dx = w + 2 * N3, *dv = w + 3 * N3;
    double *acc = w + 4 * N3, *dacc = w + 5 * N3;
    double *dmv = w + 6 * N3;
    double *lam = w + 6 * N3 + (size_t)n;     /* nout */
    double *lin = lam + nout;                 /* nin  */
    int rcode = GO_OK;
    go_params q = *p;
    q.encounter_free = 1;
    memcpy(states, x0, sizeof(double) * N3);
    memcpy(states + N3, v0, sizeof(double) * N3);
    for (int64_t s = 0; s < nsteps && rcode == GO_OK; ++s) {
        double *src = states + 6 * (size_t)n * s, *dst = src + 6 * (size_t)n;
        memcpy(dst, src, sizeof(double) * 6 * (size_t)n);
        rcode = go_free_step(&q, n, m, dst, dst + N3, 1);
    }
    for (size_t k = 0; k < N3; ++k) {
        lam[k] = gxT[k];
        lam[N3 + k] = gvT[k];
    }
    for (int i = 0; i < n; ++i) gm[i] = 0.0;
    for (int64_t s = nsteps - 1; s >= 0 && rcode == GO_OK; --s) {
        const double *st0 = states + 6 * (size_t)n * s;
        for (size_t c = 0; c < nin && rcode == GO_OK; ++c) {
            memcpy(xs, st0, sizeof(double) * N3);
            memcpy(vs, st0 + N3, sizeof(double) * N3);
            memset(dx, 0, sizeof(double) * N3);
            memset(dv, 0, sizeof(double) * N3);
            memset(dmv, 0, sizeof(double) * (size_t)n);
            if (c < N3) dx[c] = 1.0;
            else if (c < 2 * N3) dv[c - N3] = 1.0;
            else dmv[c - 2 * N3] = 1.0;
            rcode = free_step_tlm1(&q, n, m, dmv, xs, vs, dx, dv, acc, dacc);
            for (size_t r = 0; r < N3; ++r) {
                J[r * nin + c] = dx[r];
                J[(N3 + r) * nin + c] = dv[r];
            }
        }
        for (size_t c = 0; c < nin; ++c) {
            double acc_ = 0.0;
            for (size_t r = 0; r < nout; ++r) acc_ += J[r * nin + c] * lam[r];
            lin[c] = acc_;
        }
        for (size_t k = 0; k < nout; ++k) lam[k] = lin[k];
        for (int i = 0; i < n; ++i) gm[i] += lin[2 * N3 + i];
    }
    for (size_t k = 0; k < N3; ++k) {
        gx0[k] = lam[k];
        gv0[k] = lam[N3 + k];
    }
    free(states);
    free(J);
    free(w);
    return rcode;
}
